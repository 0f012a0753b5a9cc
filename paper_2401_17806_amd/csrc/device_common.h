// Device helpers shared by the operator and CG kernels (gfx950, wave64).
//
// Operator form used on the device (equivalent to eq. pressure_final, derived from the
// reference factorisation of Section 3.4 and the split dual space of Section 3.2):
//
// For triangle i with affine map x = P0 + J xi (eq. linmap), A_i = det J = 2|T_i|,
// G = J^{-1}, and an edge alpha shared with triangle r:
//   * the dual mass matrix of the edge is A_i/3 M^L + A_r/3 M^R (eq. MassMatrixD); both
//     halves carry the main Lagrange basis, so static condensation onto the p+1 shared
//     edge nodes gives Mhat^{-1} in closed form: the projected gradient on the edge nodes is
//       x_H = (A_i g_i + A_r g_r)/(A_i + A_r) + 3 |Gamma| n (C delta)/(A_i + A_r),
//     with g_s = grad p_s at the edge nodes, delta = p_r - p_i at the edge nodes (jump term
//     of eq. ad5.2, C = S0^{-1} M1), and inside each half ghat = grad p_s + sum_m Delta_m chi_m
//     with Delta = x_H - g_s;
//   * the divergence D = -Q^T (Section 3.3) tested with phi_k then gives
//       (K p)_i = -A_i sum_{de} (G G^T)_{de} S_{de} p_i
//                 + sum_alpha [ |Gamma| M1 (n . x_H) on the edge nodes
//                               - A_i sum_d Pt_alpha,d (G Delta)_d ].
// Everything per element is the two edge vectors of the triangle (32 bytes) and its
// neighbour table: no per-element operator is stored (Section 3.4.1).
//
// Work split: three lanes per triangle, lane alpha owning local edge alpha.  Each lane works
// in the triangle's frame relabelled so that its edge is local edge 0 (a cyclic renaming of
// the vertices = a DOF permutation plus new edge vectors), so all lanes run the same code on
// the same reference matrices (uniform, scalar-cache resident) and only data differ.  The
// volume term is split by rotation orbits of the nodes: each lane computes the rows of the
// orbit representatives in its own frame, which together cover every row once.  The three
// partial rows are combined through LDS in a fixed order (deterministic).
#pragma once

#include "sld_internal.h"

namespace sld_dev {

// Treatment of a wall edge (neighbour code < 0) in the operator cores.
//   kWallAbsent:   the pressure operator of eq. pressure_final: wall dual cells carry
//                  prescribed velocity and take no part (the sub-triangle's share of the volume
//                  term is given back).
//   kWallDirichlet: diffusion solves: the wall cell's gradient takes the jump to the boundary
//                  data, here zero (the data enter the right-hand side): the interior-edge form
//                  with a neighbour of zero area whose trace is zero.
//   kWallFlux:     diffusion solves, zero flux: the wall cell keeps its sub-triangle stiffness
//                  (the full-triangle volume term stands) and adds nothing.
enum WallKind { kWallAbsent = 0, kWallDirichlet = 1, kWallFlux = 2 };

constexpr int kBlockTri = 3 * kTriPerBlock;      // 192 threads: three lanes per triangle
constexpr int kBlockFlat = 256;                  // threads of flat (per-DOF) kernels
constexpr int kBlockCG = 4 * kTriPerBlock;       // 256 threads: CG iteration, one wave per role

template <int P>
struct Tab {
    static constexpr int N = (P + 1) * (P + 2) / 2;
    int na[N] = {}, nb[N] = {};
    int rot[3][N] = {};     // rot[ar][l]: original index of node l of the frame relabelled by ar
    int rep[N] = {};        // orbit representatives (rows of the volume term per lane)
    int nrep = 0;
    int centre = -1;        // node fixed by the rotation (p divisible by 3), handled by lane 0
    constexpr Tab() {
        int k = 0;
        for (int b = 0; b <= P; ++b)
            for (int a = 0; a <= P - b; ++a) { na[k] = a; nb[k] = b; ++k; }
        for (int l = 0; l < N; ++l) {
            int a = na[l], b = nb[l], c = P - a - b;
            rot[0][l] = main_idx(P, a, b);
            rot[1][l] = main_idx(P, c, a);   // v'0 = v1, v'1 = v2, v'2 = v0
            rot[2][l] = main_idx(P, b, c);   // v'0 = v2, v'1 = v0, v'2 = v1
        }
        bool seen[N] = {};
        for (int l = 0; l < N; ++l) {
            if (seen[l]) continue;
            if (rot[1][l] == l) {
                centre = l;
                seen[l] = true;
                continue;
            }
            rep[nrep++] = l;
            seen[rot[0][l]] = seen[rot[1][l]] = seen[rot[2][l]] = true;
        }
    }
};

template <int P>
__device__ __forceinline__ int rot_sel(int al, int l) {
    constexpr Tab<P> T{};
    return al == 0 ? T.rot[0][l] : (al == 1 ? T.rot[1][l] : T.rot[2][l]);
}

struct Geo {
    double A;                    // det J = 2 |T|
    double G00, G01, G10, G11;   // G = J^{-1}, G[d][c] = d xi_d / d x_c
};

__device__ __forceinline__ Geo make_geo(double e1x, double e1y, double e2x, double e2y) {
    Geo g;
    g.A = e1x * e2y - e1y * e2x;
    const double inv = 1.0 / g.A;
    g.G00 = e2y * inv;
    g.G01 = -e2x * inv;
    g.G10 = -e1y * inv;
    g.G11 = e1x * inv;
    return g;
}

// Edge vectors of a triangle relabelled so that local edge ar becomes edge 0:
// ar = 0: (e1, e2); ar = 1: (e2 - e1, -e1); ar = 2: (-e2, e1 - e2).
__device__ __forceinline__ void relabel(double4 e, int ar, double& e1x, double& e1y, double& e2x,
                                        double& e2y) {
    const double a1x = e.z - e.x, a1y = e.w - e.y;
    e1x = ar == 0 ? e.x : (ar == 1 ? a1x : -e.z);
    e1y = ar == 0 ? e.y : (ar == 1 ? a1y : -e.w);
    e2x = ar == 0 ? e.z : (ar == 1 ? -e.x : -a1x);
    e2y = ar == 0 ? e.w : (ar == 1 ? -e.y : -a1y);
}

// fused multiply-add in the arithmetic type of the operands
__device__ __forceinline__ double mad(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float mad(float a, float b, float c) { return fmaf(a, b, c); }

// The reference matrices are uniform across a wave, so they are read with scalar loads into
// SGPRs and used as FMA operands.  Left alone, the compiler issues the scalar loads of a whole
// contraction stage (or, in a loop over tiles, of all stages) far ahead of their use; at p = 3
// that is hundreds of SGPRs, which it spills into VGPR lanes and reads back one v_readlane at a
// time (about 600 extra vector instructions per wave and tile).  fence_ref hands back the same
// reference through an empty asm statement that takes `dep`, a result of the previous small
// contraction, as input: the loads of the next one cannot be issued before that result exists,
// so only one contraction's matrices (at most 20 doubles) are live at a time.  The arithmetic
// is unchanged.  Measured on the 512x512x2, p = 3 CG iteration: 121.5 -> 112.6 us (FP64) and
// 78.0 -> 72.4 us (FP32); 128x128x2, p = 3: 11.29 -> 10.43 us.  At p = 2 and 4 the ordering
// cost more than it saved (the p = 2 cavity mesh 20.9 -> 21.9 us, 256x256x2 at p = 4 56.1 ->
// 61.6 us), so only p = 3 takes the fenced forms below.
template <class T, typename D>
__device__ __forceinline__ const T& fence_ref(const T& r, const D& dep) {
    int z = 0;
    __asm__ volatile("" : "+s"(z) : "v"(dep));
    return *(&r + z);
}

// s_d = sum_l M(d, l) v_l for d = 0, 1, 2, with M(d, l) = mat(R, d, l) (one row of each of three
// reference matrices); at p = 3 one fenced contraction per matrix, dep the previous result
template <int P, class Ops, typename Real, int N, class F, typename D>
__device__ __forceinline__ void contract3(const Ops& R, F mat, const Real (&v)[N], Real& s0,
                                          Real& s1, Real& s2, const D& dep) {
    s0 = s1 = s2 = Real(0);
    if constexpr (P == 3) {
        const Ops& R0 = fence_ref(R, dep);
#pragma unroll
        for (int l = 0; l < N; ++l) s0 = mad(mat(R0, 0, l), v[l], s0);
        const Ops& R1 = fence_ref(R, s0);
#pragma unroll
        for (int l = 0; l < N; ++l) s1 = mad(mat(R1, 1, l), v[l], s1);
        const Ops& R2 = fence_ref(R, s1);
#pragma unroll
        for (int l = 0; l < N; ++l) s2 = mad(mat(R2, 2, l), v[l], s2);
    } else {
        (void)dep;
#pragma unroll
        for (int l = 0; l < N; ++l) {
            s0 = mad(mat(R, 0, l), v[l], s0);
            s1 = mad(mat(R, 1, l), v[l], s1);
            s2 = mad(mat(R, 2, l), v[l], s2);
        }
    }
}

// the reference for the next contraction: fenced on dep at p = 3, R itself otherwise
template <int P, class Ops, typename D>
__device__ __forceinline__ const Ops& next_ref(const Ops& R, const D& dep) {
    if constexpr (P == 3) return fence_ref(R, dep);
    (void)dep;
    return R;
}

// Edge-node derivatives of both sides at edge node m: ds = E[as][.][m] pl (this side, local
// edge as), dn = E[0][.][P - m] pr (the neighbour, relabelled so the edge is its edge 0)
template <int P, class Ops, typename Real, int N, typename D>
__device__ __forceinline__ void edge_derivs(const Ops& R, int as, int m, const Real (&pl)[N],
                                            const Real (&pr)[N], Real& ds0, Real& ds1,
                                            Real& dn0, Real& dn1, const D& dep) {
    ds0 = ds1 = dn0 = dn1 = Real(0);
    if constexpr (P == 3) {
        const Ops& Rm = fence_ref(R, dep);
#pragma unroll
        for (int l = 0; l < N; ++l) {
            ds0 = mad(Rm.E[as][0][m][l], pl[l], ds0);
            ds1 = mad(Rm.E[as][1][m][l], pl[l], ds1);
        }
        const Ops& Rn = fence_ref(R, ds1);
#pragma unroll
        for (int l = 0; l < N; ++l) {
            dn0 = mad(Rn.E[0][0][P - m][l], pr[l], dn0);
            dn1 = mad(Rn.E[0][1][P - m][l], pr[l], dn1);
        }
    } else {
        (void)dep;
#pragma unroll
        for (int l = 0; l < N; ++l) {
            ds0 = mad(R.E[as][0][m][l], pl[l], ds0);
            ds1 = mad(R.E[as][1][m][l], pl[l], ds1);
            dn0 = mad(R.E[0][0][P - m][l], pr[l], dn0);
            dn1 = mad(R.E[0][1][P - m][l], pr[l], dn1);
        }
    }
}

// geometric factors rounded to the arithmetic type
template <typename Real>
struct GeoR {
    Real A, G00, G01, G10, G11;
    __device__ __forceinline__ explicit GeoR(const Geo& g)
        : A((Real)g.A), G00((Real)g.G00), G01((Real)g.G01), G10((Real)g.G10), G11((Real)g.G11) {}
};

__device__ __forceinline__ int pick(int4 v, int al) { return al == 0 ? v.x : (al == 1 ? v.y : v.z); }

// Loaders of a main-grid vector value (t = triangle, l = DOF)
template <int N>
struct LoadPlain {
    const double* __restrict__ src;
    __device__ __forceinline__ double at(int64_t t, int l) const { return src[t * N + l]; }
};

// Core of lane `al` of a triangle: contributions to (K p)_i in the frame relabelled by al.
// pl holds p_i in that frame, pr the neighbour's DOFs in the neighbour's frame relabelled by
// ar (its shared edge is its local edge 0); e / er are the two triangles' edge vectors; nb < 0
// marks a wall edge.  y receives local rows: this lane's volume rows (orbit representatives)
// plus the full edge-al term.
template <int P, class Ops, typename Real>
__device__ __forceinline__ void edge_lane_core(int al, const Ops& R, double4 e, int nb, int ar,
                                               double4 er, const Real (&pl)[RefOps<P>::NPHI],
                                               const Real (&pr)[RefOps<P>::NPHI],
                                               Real (&y)[RefOps<P>::NPHI],
                                               int wall = kWallAbsent) {
    constexpr int N = RefOps<P>::NPHI;
    constexpr int NE = P + 1;
    constexpr Tab<P> T{};
    double e1x, e1y, e2x, e2y;
    relabel(e, al, e1x, e1y, e2x, e2y);
    // geometric factors in float64, then rounded to the arithmetic type
    const Geo gd = make_geo(e1x, e1y, e2x, e2y);
    const GeoR<Real> g(gd);
    const Real m00 = (Real)(gd.G00 * gd.G00 + gd.G01 * gd.G01);
    const Real m01 = (Real)(gd.G00 * gd.G10 + gd.G01 * gd.G11);
    const Real m11 = (Real)(gd.G10 * gd.G10 + gd.G11 * gd.G11);
#pragma unroll
    for (int k = 0; k < N; ++k) y[k] = Real(0);
    // volume term -A (m00 S0 + m01 S1 + m11 S2) p on this lane's rows
#pragma unroll
    for (int q = 0; q < T.nrep; ++q) {
        const int k = T.rep[q];
        Real s0, s1, s2;
        contract3<P>(R, [&](const Ops& Q, int d, int l) { return Q.S[d][k][l]; }, pl, s0, s1, s2,
                     q > 0 ? y[T.rep[q > 0 ? q - 1 : 0]] : pl[0]);
        y[k] = -g.A * (m00 * s0 + m01 * s1 + m11 * s2);
    }
    if (T.centre >= 0 && al == 0) {
        const int k = T.centre >= 0 ? T.centre : 0;
        Real s0, s1, s2;
        contract3<P>(R, [&](const Ops& Q, int d, int l) { return Q.S[d][k][l]; }, pl, s0, s1, s2,
                     y[T.rep[T.nrep - 1]]);
        y[k] = -g.A * (m00 * s0 + m01 * s1 + m11 * s2);
    }
    const Real snx = (Real)e1y, sny = (Real)(-e1x);  // |Gamma| n, outward, of local edge 0
    const bool ghost = nb < 0 && wall == kWallDirichlet;
    if (nb < 0 && wall == kWallFlux) return;
    if (nb < 0 && !ghost) {
        // wall edge: no dual coupling; give back this sub-triangle's share of the volume term
#pragma unroll
        for (int k = 0; k < N; ++k) {
            Real s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
            for (int l = 0; l < N; ++l) {
                s0 = mad(R.Sh[0][0][k][l], pl[l], s0);
                s1 = mad(R.Sh[0][1][k][l], pl[l], s1);
                s2 = mad(R.Sh[0][2][k][l], pl[l], s2);
            }
            y[k] += g.A * (m00 * s0 + m01 * s1 + m11 * s2);
        }
        return;
    }
    double f1x, f1y, f2x, f2y;
    relabel(er, ar, f1x, f1y, f2x, f2y);
    // a Dirichlet wall is an edge to a ghost neighbour of zero area and zero trace
    Geo grd = ghost ? Geo{0.0, 0.0, 0.0, 0.0, 0.0} : make_geo(f1x, f1y, f2x, f2y);
    const GeoR<Real> gr(grd);
    const Real wsum = (Real)(1.0 / (gd.A + grd.A));
    Real delta[NE];
#pragma unroll
    for (int m = 0; m < NE; ++m) delta[m] = (ghost ? Real(0) : pr[P - m]) - pl[m];  // edge-0 nodes are 0..P
    Real gd0[NE], gd1[NE], tn[NE];
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        Real ds0, ds1, dn0, dn1;
        edge_derivs<P>(R, 0, m, pl, pr, ds0, ds1, dn0, dn1, m > 0 ? gd1[m > 0 ? m - 1 : 0] : delta[0]);
        const Ops& Rc = next_ref<P>(R, dn1);
        const Real gsx = g.G00 * ds0 + g.G10 * ds1, gsy = g.G01 * ds0 + g.G11 * ds1;
        const Real gnx = gr.G00 * dn0 + gr.G10 * dn1, gny = gr.G01 * dn0 + gr.G11 * dn1;
        Real cd = 0;
#pragma unroll
        for (int q = 0; q < NE; ++q) cd = mad(Rc.C[m][q], delta[q], cd);
        const Real hx = (g.A * gsx + gr.A * gnx + Real(3) * snx * cd) * wsum;
        const Real hy = (g.A * gsy + gr.A * gny + Real(3) * sny * cd) * wsum;
        tn[m] = snx * hx + sny * hy;
        const Real dx = hx - gsx, dy = hy - gsy;
        gd0[m] = g.G00 * dx + g.G01 * dy;
        gd1[m] = g.G10 * dx + g.G11 * dy;
    }
    // line term |Gamma| int phi_k n.x_H on the edge nodes
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        const Ops& Rm = next_ref<P>(R, m > 0 ? y[m > 0 ? m - 1 : 0] : tn[NE - 1]);
        Real s = 0;
#pragma unroll
        for (int q = 0; q < NE; ++q) s = mad(Rm.M1[m][q], tn[q], s);
        y[m] += s;
    }
    // sub-triangle correction -A sum_d Pt_d (G Delta)_d
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const Ops& Rk = next_ref<P>(R, k > 0 ? y[k > 0 ? k - 1 : 0] : gd1[NE - 1]);
        Real s = 0;
#pragma unroll
        for (int m = 0; m < NE; ++m) {
            s = mad(Rk.Pt[0][0][k][m], gd0[m], s);
            s = mad(Rk.Pt[0][1][k][m], gd1[m], s);
        }
        y[k] = mad(-g.A, s, y[k]);
    }
}

// Natural-frame forms used by the CG iteration kernel, one wave per role: waves 0..2 take
// local edge AL of every triangle of a tile (one lane per triangle), wave 3 the volume term.
// pl = p_i in its own (natural) numbering; pr = the neighbour's DOFs relabelled by ar (its shared
// edge is its local edge 0); e / er are the two triangles' edge vectors (v1 - v0, v2 - v0).
// The result y holds this role's contribution to the rows of (K p)_i (natural numbering).

// Volume term -A (m00 S0 + m01 S1 + m11 S2) p over all rows.
template <int P, class Ops, typename Real>
__device__ __forceinline__ void volume_wave_core(const Ops& R, double4 e,
                                                 const Real (&pl)[RefOps<P>::NPHI],
                                                 Real (&y)[RefOps<P>::NPHI]) {
    constexpr int N = RefOps<P>::NPHI;
    const Geo gd = make_geo(e.x, e.y, e.z, e.w);
    const Real A = (Real)gd.A;
    const Real m00 = (Real)(gd.G00 * gd.G00 + gd.G01 * gd.G01);
    const Real m01 = (Real)(gd.G00 * gd.G10 + gd.G01 * gd.G11);
    const Real m11 = (Real)(gd.G10 * gd.G10 + gd.G11 * gd.G11);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        Real s0, s1, s2;
        contract3<P>(R, [&](const Ops& Q, int d, int l) { return Q.S[d][k][l]; }, pl, s0, s1, s2,
                     k > 0 ? y[k > 0 ? k - 1 : 0] : pl[0]);
        y[k] = -A * (m00 * s0 + m01 * s1 + m11 * s2);
    }
}

// Edge AL (compile time) of triangle i: the dual coupling through that edge (edge-node
// gradients of both sides, jump, projected gradient x_H, line term and sub-triangle
// correction), or on a wall edge the sub-triangle share of the volume term given back.
template <int P, int AL, class Ops, typename Real>
__device__ __forceinline__ void edge_wave_core(const Ops& R, double4 e, int nb, int ar, double4 er,
                                               const Real (&pl)[RefOps<P>::NPHI],
                                               const Real (&pr)[RefOps<P>::NPHI],
                                               Real (&y)[RefOps<P>::NPHI],
                                               int wall = kWallAbsent) {
    constexpr int N = RefOps<P>::NPHI;
    constexpr int NE = P + 1;
    const Geo gd = make_geo(e.x, e.y, e.z, e.w);
    const GeoR<Real> g(gd);
#pragma unroll
    for (int k = 0; k < N; ++k) y[k] = Real(0);
    const bool ghost = nb < 0 && wall == kWallDirichlet;
    if (nb < 0 && wall == kWallFlux) return;
    if (nb < 0 && !ghost) {
        const Real m00 = (Real)(gd.G00 * gd.G00 + gd.G01 * gd.G01);
        const Real m01 = (Real)(gd.G00 * gd.G10 + gd.G01 * gd.G11);
        const Real m11 = (Real)(gd.G10 * gd.G10 + gd.G11 * gd.G11);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            Real s0, s1, s2;
            contract3<P>(R, [&](const Ops& Q, int d, int l) { return Q.Sh[AL][d][k][l]; }, pl, s0,
                         s1, s2, k > 0 ? y[k > 0 ? k - 1 : 0] : pl[0]);
            y[k] = g.A * (m00 * s0 + m01 * s1 + m11 * s2);
        }
        return;
    }
    // |Gamma| n, outward: the edge vector v_{AL+1} - v_AL turned clockwise
    const double ex = AL == 0 ? e.x : (AL == 1 ? e.z - e.x : -e.z);
    const double ey = AL == 0 ? e.y : (AL == 1 ? e.w - e.y : -e.w);
    const Real snx = (Real)ey, sny = (Real)(-ex);
    double f1x, f1y, f2x, f2y;
    relabel(er, ar, f1x, f1y, f2x, f2y);
    // a Dirichlet wall is an edge to a ghost neighbour of zero area and zero trace
    Geo grd = ghost ? Geo{0.0, 0.0, 0.0, 0.0, 0.0} : make_geo(f1x, f1y, f2x, f2y);
    const GeoR<Real> gr(grd);
    const Real wsum = (Real)(1.0 / (gd.A + grd.A));
    Real delta[NE];
#pragma unroll
    for (int m = 0; m < NE; ++m)
        delta[m] = (ghost ? Real(0) : pr[P - m]) - pl[edge_node(P, AL, m)];
    Real gd0[NE], gd1[NE], tn[NE];
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        Real ds0, ds1, dn0, dn1;
        edge_derivs<P>(R, AL, m, pl, pr, ds0, ds1, dn0, dn1, m > 0 ? gd1[m > 0 ? m - 1 : 0] : delta[0]);
        const Ops& Rc = next_ref<P>(R, dn1);
        const Real gsx = g.G00 * ds0 + g.G10 * ds1, gsy = g.G01 * ds0 + g.G11 * ds1;
        const Real gnx = gr.G00 * dn0 + gr.G10 * dn1, gny = gr.G01 * dn0 + gr.G11 * dn1;
        Real cd = 0;
#pragma unroll
        for (int q = 0; q < NE; ++q) cd = mad(Rc.C[m][q], delta[q], cd);
        const Real hx = (g.A * gsx + gr.A * gnx + Real(3) * snx * cd) * wsum;
        const Real hy = (g.A * gsy + gr.A * gny + Real(3) * sny * cd) * wsum;
        tn[m] = snx * hx + sny * hy;
        const Real dx = hx - gsx, dy = hy - gsy;
        gd0[m] = g.G00 * dx + g.G01 * dy;
        gd1[m] = g.G10 * dx + g.G11 * dy;
    }
    // line term |Gamma| int phi_k n.x_H on the edge nodes
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        const Ops& Rm = next_ref<P>(R, m > 0 ? y[edge_node(P, AL, m > 0 ? m - 1 : 0)] : tn[NE - 1]);
        Real s = 0;
#pragma unroll
        for (int q = 0; q < NE; ++q) s = mad(Rm.M1[m][q], tn[q], s);
        y[edge_node(P, AL, m)] = s;
    }
    // sub-triangle correction -A sum_d Pt_d (G Delta)_d
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const Ops& Rk = next_ref<P>(R, k > 0 ? y[k > 0 ? k - 1 : 0] : gd1[NE - 1]);
        Real s = 0;
#pragma unroll
        for (int m = 0; m < NE; ++m) {
            s = mad(Rk.Pt[AL][0][k][m], gd0[m], s);
            s = mad(Rk.Pt[AL][1][k][m], gd1[m], s);
        }
        y[k] = mad(-g.A, s, y[k]);
    }
}

// Lane `al` of triangle i with p read through a loader (global memory).
template <int P, class L>
__device__ __forceinline__ void schur_edge_lane(int64_t i, int al, const RefOps<P>& R,
                                                const double4* __restrict__ geo,
                                                const int4* __restrict__ nbr, const L& ld,
                                                double (&pl)[RefOps<P>::NPHI],
                                                double (&y)[RefOps<P>::NPHI],
                                                int wall = kWallAbsent) {
    constexpr int N = RefOps<P>::NPHI;
#pragma unroll
    for (int l = 0; l < N; ++l) pl[l] = ld.at(i, rot_sel<P>(al, l));
    const int nb = pick(nbr[i], al);
    double pr[N];
    double4 er = make_double4(0, 0, 0, 0);
    int ar = 0;
    if (nb >= 0) {
        const int64_t r = nb >> 2;
        ar = nb & 3;
#pragma unroll
        for (int l = 0; l < N; ++l) pr[l] = ld.at(r, rot_sel<P>(ar, l));
        er = geo[r];
    } else {
#pragma unroll
        for (int l = 0; l < N; ++l) pr[l] = 0.0;
    }
    edge_lane_core<P>(al, R, geo[i], nb, ar, er, pl, pr, y, wall);
}

// Scatter a lane's local rows to LDS slot al in natural numbering.
template <int P>
__device__ __forceinline__ void lds_scatter(double* slot_base /* [4][N] of this triangle */, int al,
                                            const double (&y)[RefOps<P>::NPHI]) {
    constexpr int N = RefOps<P>::NPHI;
#pragma unroll
    for (int k = 0; k < N; ++k) slot_base[al * N + rot_sel<P>(al, k)] = y[k];
}

// Lane data movement of a float64 within a wave through DPP (no memory access).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double readlane_f64(double x, int lane) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wave, the same in every lane: pairs and quads (quad permutes),
// then the four quads of each row of 16 lanes (rotations by 4 and 8), then the four rows' sums
// read from lanes 0, 16, 32, 48.  Fixed order, bitwise identical in every lane.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x124>(v);  // row_ror:4
    v += dpp_f64<0x128>(v);  // row_ror:8
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Deterministic block sum of NV values; result returned in every thread.
template <int NV, int NT>
__device__ __forceinline__ void block_sum_all(double (&v)[NV]) {
    __shared__ double sh[NV][NT / 64];
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] = wave_sum(v[c]);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) sh[c][wid] = v[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        double s = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += sh[c][w];
        v[c] = s;
    }
}

// Sum of partial[0..n) in a fixed order, identical in every block (n <= a few thousand).
template <int NT>
__device__ __forceinline__ double reduce_partials(const double* __restrict__ partial, int n) {
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < n; b += NT) v[0] += partial[b];
    // the butterfly mixes lanes in a fixed pattern: the same in every block
    block_sum_all<1, NT>(v);
    return v[0];
}

}  // namespace sld_dev
