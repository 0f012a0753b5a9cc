// HIP kernels (gfx950) of the pressure Schur-complement path.
//
// Operator form used on the device (equivalent to eq. pressure_final, derived from the
// reference factorisation of Section 2.4 and the split dual space of Section 2.2):
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
//   * the divergence D = -Q^T (Section 2.3) tested with phi_k then gives
//       (K p)_i = -A_i sum_{de} (G G^T)_{de} S_{de} p_i
//                 + sum_alpha [ |Gamma| M1 (n . x_H) on the edge nodes
//                               - A_i sum_d Pt_alpha,d (G Delta)_d ].
// Everything per element is the two edge vectors of the triangle (32 bytes) and its
// neighbour table: no per-element operator is stored (Section 2.4.1).
//
// A neighbour is read in its own frame relabelled so that the shared edge becomes its local
// edge 0 (cyclic relabelling of the vertices: a DOF permutation and new edge vectors), so
// that every lane uses the same reference matrices and the reference data stay uniform.
#include "sld_internal.h"

namespace {

constexpr int kBlock = 128;  // threads per block (2 waves of 64)

template <int P>
struct Tab {
    static constexpr int N = (P + 1) * (P + 2) / 2;
    int na[N] = {}, nb[N] = {};
    int rot[3][N] = {};  // rot[ar][l]: original index of node l of the frame relabelled by ar
    int edge[3][P + 1] = {};
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
        for (int al = 0; al < 3; ++al)
            for (int m = 0; m <= P; ++m) edge[al][m] = edge_node(P, al, m);
    }
};

struct Geo {
    double A;            // det J = 2 |T|
    double G00, G01, G10, G11;  // G = J^{-1}, G[d][c] = d xi_d / d x_c
};

__device__ __forceinline__ Geo make_geo(double e1x, double e1y, double e2x, double e2y) {
    Geo g;
    g.A = e1x * e2y - e1y * e2x;
    double inv = 1.0 / g.A;
    g.G00 = e2y * inv;
    g.G01 = -e2x * inv;
    g.G10 = -e1y * inv;
    g.G11 = e1x * inv;
    return g;
}

// Edge vectors of a triangle relabelled so that local edge ar becomes edge 0.
__device__ __forceinline__ void relabel(double4 e, int ar, double& e1x, double& e1y, double& e2x,
                                        double& e2y) {
    // ar = 0: (e1, e2); ar = 1: (e2 - e1, -e1); ar = 2: (-e2, e1 - e2)
    double a1x = e.z - e.x, a1y = e.w - e.y;
    e1x = ar == 0 ? e.x : (ar == 1 ? a1x : -e.z);
    e1y = ar == 0 ? e.y : (ar == 1 ? a1y : -e.w);
    e2x = ar == 0 ? e.z : (ar == 1 ? -e.x : -a1x);
    e2y = ar == 0 ? e.w : (ar == 1 ? -e.y : -a1y);
}

// Plain loader: v[l] = src[t][l]
template <int N>
struct LoadPlain {
    const double* __restrict__ src;
    __device__ __forceinline__ double at(int64_t t, int l) const { return src[t * N + l]; }
};

// CG direction loader: v[l] = r[t][l] + beta * d_old[t][l]
template <int N>
struct LoadDir {
    const double* __restrict__ r;
    const double* __restrict__ d;
    double beta;
    __device__ __forceinline__ double at(int64_t t, int l) const {
        return fma(beta, d[t * N + l], r[t * N + l]);
    }
};

// y = K p on triangle i (paper sign).  Loads p of i and its neighbours through L.
template <int P, class L>
__device__ __forceinline__ void schur_row(int64_t i, const RefOps<P>& R, const double4* __restrict__ geo,
                                          const int4* __restrict__ nbr, const L& ld,
                                          double (&pi)[RefOps<P>::NPHI], double (&y)[RefOps<P>::NPHI]) {
    constexpr int N = RefOps<P>::NPHI;
    constexpr int NE = P + 1;
    constexpr Tab<P> T{};
#pragma unroll
    for (int l = 0; l < N; ++l) pi[l] = ld.at(i, l);
    const double4 e = geo[i];
    const Geo g = make_geo(e.x, e.y, e.z, e.w);
    const double m00 = g.G00 * g.G00 + g.G01 * g.G01;
    const double m01 = g.G00 * g.G10 + g.G01 * g.G11;
    const double m11 = g.G10 * g.G10 + g.G11 * g.G11;
    // volume term over the whole triangle: -A (m00 S0 + m01 S1 + m11 S2) p
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int l = 0; l < N; ++l) {
            s0 = fma(R.S[0][k][l], pi[l], s0);
            s1 = fma(R.S[1][k][l], pi[l], s1);
            s2 = fma(R.S[2][k][l], pi[l], s2);
        }
        y[k] = -g.A * (m00 * s0 + m01 * s1 + m11 * s2);
    }
    const int4 nb4 = nbr[i];
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const int nb = al == 0 ? nb4.x : (al == 1 ? nb4.y : nb4.z);
        // scaled outward normal |Gamma| n of edge al: edge vector (ex, ey) -> (ey, -ex)
        double ex, ey;
        if (al == 0) { ex = e.x; ey = e.y; }
        else if (al == 1) { ex = e.z - e.x; ey = e.w - e.y; }
        else { ex = -e.z; ey = -e.w; }
        const double snx = ey, sny = -ex;
        if (nb < 0) {
            // wall edge: no dual coupling; remove this half's share of the volume term
#pragma unroll
            for (int k = 0; k < N; ++k) {
                double s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
                for (int l = 0; l < N; ++l) {
                    s0 = fma(R.Sh[al][0][k][l], pi[l], s0);
                    s1 = fma(R.Sh[al][1][k][l], pi[l], s1);
                    s2 = fma(R.Sh[al][2][k][l], pi[l], s2);
                }
                y[k] += g.A * (m00 * s0 + m01 * s1 + m11 * s2);
            }
            continue;
        }
        const int64_t r = nb >> 2;
        const int ar = nb & 3;
        // neighbour DOFs in the relabelled frame (its shared edge is edge 0)
        double pr[N];
#pragma unroll
        for (int l = 0; l < N; ++l) {
            const int src = ar == 0 ? T.rot[0][l] : (ar == 1 ? T.rot[1][l] : T.rot[2][l]);
            pr[l] = ld.at(r, src);
        }
        double f1x, f1y, f2x, f2y;
        relabel(geo[r], ar, f1x, f1y, f2x, f2y);
        const Geo gr = make_geo(f1x, f1y, f2x, f2y);
        const double wsum = 1.0 / (g.A + gr.A);
        double xH[NE][2], dl[NE][2];
        double delta[NE];
#pragma unroll
        for (int m = 0; m < NE; ++m) delta[m] = pr[T.edge[0][P - m]] - pi[T.edge[al][m]];
#pragma unroll
        for (int m = 0; m < NE; ++m) {
            // self gradient at edge node m
            double ds0 = 0, ds1 = 0, dn0 = 0, dn1 = 0;
#pragma unroll
            for (int l = 0; l < N; ++l) {
                ds0 = fma(R.E[al][0][m][l], pi[l], ds0);
                ds1 = fma(R.E[al][1][m][l], pi[l], ds1);
                dn0 = fma(R.E[0][0][P - m][l], pr[l], dn0);
                dn1 = fma(R.E[0][1][P - m][l], pr[l], dn1);
            }
            const double gsx = g.G00 * ds0 + g.G10 * ds1, gsy = g.G01 * ds0 + g.G11 * ds1;
            const double gnx = gr.G00 * dn0 + gr.G10 * dn1, gny = gr.G01 * dn0 + gr.G11 * dn1;
            double cd = 0;
#pragma unroll
            for (int q = 0; q < NE; ++q) cd = fma(R.C[m][q], delta[q], cd);
            const double hx = (g.A * gsx + gr.A * gnx + 3.0 * snx * cd) * wsum;
            const double hy = (g.A * gsy + gr.A * gny + 3.0 * sny * cd) * wsum;
            xH[m][0] = hx;
            xH[m][1] = hy;
            dl[m][0] = hx - gsx;
            dl[m][1] = hy - gsy;
        }
        // line term |Gamma| int phi_k n.x_H
        double tn[NE];
#pragma unroll
        for (int m = 0; m < NE; ++m) tn[m] = snx * xH[m][0] + sny * xH[m][1];
#pragma unroll
        for (int m = 0; m < NE; ++m) {
            double s = 0;
#pragma unroll
            for (int q = 0; q < NE; ++q) s = fma(R.M1[m][q], tn[q], s);
            y[T.edge[al][m]] += s;
        }
        // sub-triangle correction -A sum_d Pt_d (G Delta)_d
        double gd0[NE], gd1[NE];
#pragma unroll
        for (int m = 0; m < NE; ++m) {
            gd0[m] = g.G00 * dl[m][0] + g.G01 * dl[m][1];
            gd1[m] = g.G10 * dl[m][0] + g.G11 * dl[m][1];
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double s = 0;
#pragma unroll
            for (int m = 0; m < NE; ++m) {
                s = fma(R.Pt[al][0][k][m], gd0[m], s);
                s = fma(R.Pt[al][1][k][m], gd1[m], s);
            }
            y[k] = fma(-g.A, s, y[k]);
        }
    }
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_schur_apply(const RefOps<P>* __restrict__ ops,
                                                        const double4* __restrict__ geo,
                                                        const int4* __restrict__ nbr, int64_t ne,
                                                        const double* __restrict__ p,
                                                        double* __restrict__ out, double scale) {
    constexpr int N = RefOps<P>::NPHI;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= ne) return;
    double pi[N], y[N];
    LoadPlain<N> ld{p};
    schur_row<P>(i, *ops, geo, nbr, ld, pi, y);
#pragma unroll
    for (int k = 0; k < N; ++k) out[i * N + k] = scale * y[k];
}

// ---------------------------------------------------------------- gradient (lane per edge)
template <int P>
__global__ __launch_bounds__(kBlock) void k_gradient(const RefOps<P>* __restrict__ ops,
                                                     const double4* __restrict__ geo,
                                                     const int4* __restrict__ edges, int64_t nd,
                                                     const double* __restrict__ p,
                                                     const double* vstar, double coef,
                                                     double* out) {
    constexpr int N = RefOps<P>::NPHI;
    constexpr int NE = P + 1;
    constexpr int NI = N - NE;
    constexpr int NPSI = (P + 1) * (P + 1);
    constexpr Tab<P> T{};
    const RefOps<P>& R = *ops;
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nd) return;
    const int4 ed = edges[j];
    double* o = out + j * 2 * NPSI;
    const double* vs = vstar ? vstar + j * 2 * NPSI : nullptr;
    if (ed.y < 0) {
#pragma unroll
        for (int k = 0; k < 2 * NPSI; ++k) o[k] = vs ? vs[k] : 0.0;
        return;
    }
    double pl[N], pr[N];
#pragma unroll
    for (int l = 0; l < N; ++l) {
        const int sl = ed.z == 0 ? T.rot[0][l] : (ed.z == 1 ? T.rot[1][l] : T.rot[2][l]);
        const int sr = ed.w == 0 ? T.rot[0][l] : (ed.w == 1 ? T.rot[1][l] : T.rot[2][l]);
        pl[l] = p[(int64_t)ed.x * N + sl];
        pr[l] = p[(int64_t)ed.y * N + sr];
    }
    double a1x, a1y, a2x, a2y, b1x, b1y, b2x, b2y;
    relabel(geo[ed.x], ed.z, a1x, a1y, a2x, a2y);
    relabel(geo[ed.y], ed.w, b1x, b1y, b2x, b2y);
    const Geo gl = make_geo(a1x, a1y, a2x, a2y);
    const Geo gr = make_geo(b1x, b1y, b2x, b2y);
    const double snx = a1y, sny = -a1x;  // |Gamma| n_j, l's edge A -> B is e1'
    const double wsum = 1.0 / (gl.A + gr.A);
    // gradients at every node of both halves (half 0 of each relabelled frame)
    double hl[N][2], hr[N][2];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        double a0 = 0, a1 = 0, b0 = 0, b1 = 0;
#pragma unroll
        for (int l = 0; l < N; ++l) {
            a0 = fma(R.Hn[0][0][n][l], pl[l], a0);
            a1 = fma(R.Hn[0][1][n][l], pl[l], a1);
            b0 = fma(R.Hn[0][0][n][l], pr[l], b0);
            b1 = fma(R.Hn[0][1][n][l], pr[l], b1);
        }
        hl[n][0] = gl.G00 * a0 + gl.G10 * a1;
        hl[n][1] = gl.G01 * a0 + gl.G11 * a1;
        hr[n][0] = gr.G00 * b0 + gr.G10 * b1;
        hr[n][1] = gr.G01 * b0 + gr.G11 * b1;
    }
    double delta[NE];
#pragma unroll
    for (int m = 0; m < NE; ++m) delta[m] = pr[T.edge[0][P - m]] - pl[T.edge[0][m]];
    double xH[NE][2], dL[NE][2], dR[NE][2];
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        double cd = 0;
#pragma unroll
        for (int q = 0; q < NE; ++q) cd = fma(R.C[m][q], delta[q], cd);
        const int hm = main_idx(P, P - m, m);       // l's half node of edge node m
        const int hmr = main_idx(P, m, P - m);      // r's half node of l's edge node m
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const double sn = c == 0 ? snx : sny;
            xH[m][c] = (gl.A * hl[hm][c] + gr.A * hr[hmr][c] + 3.0 * sn * cd) * wsum;
        }
    }
#pragma unroll
    for (int m = 0; m < NE; ++m)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            dL[m][c] = xH[m][c] - hl[main_idx(P, P - m, m)][c];
            // r's own edge node m_r corresponds to l's node P - m_r
            dR[m][c] = xH[P - m][c] - hr[main_idx(P, P - m, m)][c];
        }
    // interior nodes of each half: g - Z Delta
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        int ii = 0;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const int a = T.na[n], b = T.nb[n];
            if (a + b < P) {
                double zl = 0, zr = 0;
#pragma unroll
                for (int m = 0; m < NE; ++m) {
                    zl = fma(R.Z[ii][m], dL[m][c], zl);
                    zr = fma(R.Z[ii][m], dR[m][c], zr);
                }
                const int kl = b * (P + 1) + a;                 // dual DOF of l's node (a,b)
                const int kr = (P - b) * (P + 1) + (P - a);     // dual DOF of r's node (a,b)
                const double vl = hl[n][c] - zl, vr = hr[n][c] - zr;
                o[c * NPSI + kl] = vs ? fma(coef, vl, vs[c * NPSI + kl]) : coef * vl;
                o[c * NPSI + kr] = vs ? fma(coef, vr, vs[c * NPSI + kr]) : coef * vr;
                ++ii;
            }
        }
#pragma unroll
        for (int m = 0; m < NE; ++m) {
            const int kd = m * (P + 1) + (P - m);  // dual diagonal node (a, b) = (P - m, m)
            o[c * NPSI + kd] = vs ? fma(coef, xH[m][c], vs[c * NPSI + kd]) : coef * xH[m][c];
        }
    }
    (void)NI;
}

// ---------------------------------------------------------------- divergence (lane per triangle)
template <int P>
__global__ __launch_bounds__(kBlock) void k_divergence(const RefOps<P>* __restrict__ ops,
                                                       const double4* __restrict__ geo,
                                                       const int4* __restrict__ nbr,
                                                       const int4* __restrict__ tedges, int64_t ne,
                                                       const double* __restrict__ v, double scale,
                                                       double* __restrict__ out) {
    constexpr int N = RefOps<P>::NPHI;
    constexpr int NE = P + 1;
    constexpr int NPSI = (P + 1) * (P + 1);
    constexpr Tab<P> T{};
    const RefOps<P>& R = *ops;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= ne) return;
    const double4 e = geo[i];
    const Geo g = make_geo(e.x, e.y, e.z, e.w);
    const int4 nb4 = nbr[i];
    const int4 te4 = tedges[i];
    double y[N];
#pragma unroll
    for (int k = 0; k < N; ++k) y[k] = 0;
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const int nb = al == 0 ? nb4.x : (al == 1 ? nb4.y : nb4.z);
        if (nb < 0) continue;
        const int te = al == 0 ? te4.x : (al == 1 ? te4.y : te4.z);
        const int64_t j = te >> 1;
        const int beta = te & 1;
        double ex, ey;
        if (al == 0) { ex = e.x; ey = e.y; }
        else if (al == 1) { ex = e.z - e.x; ey = e.w - e.y; }
        else { ex = -e.z; ey = -e.w; }
        const double snx = ey, sny = -ex;
        const double* vj = v + j * 2 * NPSI;
        double vh[N][2];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const int a = T.na[n], b = T.nb[n];
            const int k = beta ? (P - b) * (P + 1) + (P - a) : b * (P + 1) + a;
            vh[n][0] = vj[k];
            vh[n][1] = vj[NPSI + k];
        }
        // line term on the edge nodes (half nodes (P-m, m))
        double tn[NE];
#pragma unroll
        for (int m = 0; m < NE; ++m) {
            const int n = main_idx(P, P - m, m);
            tn[m] = snx * vh[n][0] + sny * vh[n][1];
        }
#pragma unroll
        for (int m = 0; m < NE; ++m) {
            double s = 0;
#pragma unroll
            for (int q = 0; q < NE; ++q) s = fma(R.M1[m][q], tn[q], s);
            y[T.edge[al][m]] += s;
        }
        double w0[N], w1[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            w0[n] = g.G00 * vh[n][0] + g.G01 * vh[n][1];
            w1[n] = g.G10 * vh[n][0] + g.G11 * vh[n][1];
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double s = 0;
#pragma unroll
            for (int n = 0; n < N; ++n) {
                s = fma(R.W[al][0][k][n], w0[n], s);
                s = fma(R.W[al][1][k][n], w1[n], s);
            }
            y[k] = fma(-g.A, s, y[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < N; ++k) out[i * N + k] = scale * y[k];
}

// ---------------------------------------------------------------- reductions
// Deterministic block sum: wave butterfly then waves in order; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
    __shared__ double sh[NV][kBlock / 64];
#pragma unroll
    for (int c = 0; c < NV; ++c)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) sh[c][wid] = v[c];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            double s = 0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) s += sh[c][w];
            v[c] = s;
        }
    __syncthreads();
}

// Publish this block's partial sums; returns true in the block that finished last, whose
// v[] then holds the grand totals (summed in block order, deterministic).
template <int NV>
__device__ bool grid_sum(double (&v)[NV], double* __restrict__ partial, unsigned* counter) {
    __shared__ bool last;
    block_sum<NV>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) partial[(int64_t)c * gridDim.x + blockIdx.x] = v[c];
        __threadfence();
        const unsigned t = atomicAdd(counter, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    double acc[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        acc[c] = 0;
        for (unsigned b = threadIdx.x; b < gridDim.x; b += kBlock)
            acc[c] += __hip_atomic_load(partial + (int64_t)c * gridDim.x + b, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    }
    block_sum<NV>(acc);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) v[c] = acc[c];
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return threadIdx.x == 0;
}

typedef CgScalars S;

// mean of b (projection onto the complement of the constant vector)
template <int P>
__global__ __launch_bounds__(kBlock) void k_cg_mean(const double* __restrict__ b, int64_t ne,
                                                    double* partial, unsigned* counter, double* scal) {
    constexpr int N = RefOps<P>::NPHI;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {0};
    if (i < ne)
#pragma unroll
        for (int k = 0; k < N; ++k) v[0] += b[i * N + k];
    if (grid_sum<1>(v, partial, counter)) scal[S::MEAN] = v[0] / (double)(ne * N);
}

// b_int = b - mean; r = -b_int + (warm ? K x : 0); d = 0; rr, bb
template <int P>
__global__ __launch_bounds__(kBlock) void k_cg_init(const double* __restrict__ b, const double* __restrict__ kx,
                                                    int64_t ne, double* __restrict__ bint,
                                                    double* __restrict__ x, double* __restrict__ r,
                                                    double* __restrict__ d0, double* __restrict__ d1,
                                                    int warm, double rtol, int maxit,
                                                    double* partial, unsigned* counter, double* scal) {
    constexpr int N = RefOps<P>::NPHI;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const double mean = scal[S::MEAN];
    double v[2] = {0, 0};
    if (i < ne) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const int64_t o = i * N + k;
            const double bi = b[o] - mean;
            bint[o] = bi;
            const double ri = warm ? kx[o] - bi : -bi;
            r[o] = ri;
            if (!warm) x[o] = 0.0;
            d0[o] = 0.0;
            d1[o] = 0.0;
            v[0] = fma(ri, ri, v[0]);
            v[1] = fma(bi, bi, v[1]);
        }
    }
    if (grid_sum<2>(v, partial, counter)) {
        scal[S::RR] = v[0];
        scal[S::BB] = v[1];
        scal[S::TOL2] = rtol * rtol * v[1];
        scal[S::BETA] = 0.0;
        scal[S::ALPHA] = 0.0;
        scal[S::ITER] = 0.0;
        scal[S::MAXIT] = (double)maxit;
        scal[S::DONE] = (v[0] <= rtol * rtol * v[1]) ? 1.0 : 0.0;
    }
}

// d_new = r + beta d_old ; q = -K d_new ; dq = d_new . q ; alpha = rr / dq
template <int P>
__global__ __launch_bounds__(kBlock) void k_cg_apply(const RefOps<P>* __restrict__ ops,
                                                     const double4* __restrict__ geo,
                                                     const int4* __restrict__ nbr, int64_t ne,
                                                     const double* __restrict__ r,
                                                     const double* __restrict__ dold,
                                                     double* __restrict__ dnew, double* __restrict__ q,
                                                     double* partial, unsigned* counter, double* scal) {
    constexpr int N = RefOps<P>::NPHI;
    if (scal[S::DONE] != 0.0) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const double beta = scal[S::BETA];
    double v[1] = {0};
    if (i < ne) {
        double di[N], y[N];
        LoadDir<N> ld{r, dold, beta};
        schur_row<P>(i, *ops, geo, nbr, ld, di, y);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            dnew[i * N + k] = di[k];
            q[i * N + k] = -y[k];
            v[0] = fma(di[k], -y[k], v[0]);
        }
    }
    if (grid_sum<1>(v, partial, counter)) {
        const double dq = v[0];
        scal[S::DQ] = dq;
        if (!(dq > 0.0) || !isfinite(dq)) {
            scal[S::DONE] = 3.0;
            scal[S::ALPHA] = 0.0;
        } else {
            scal[S::ALPHA] = scal[S::RR] / dq;
        }
    }
}

// x += alpha d ; r -= alpha q ; rr_new ; beta ; convergence
template <int P>
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t ne, double* __restrict__ x,
                                                      double* __restrict__ r,
                                                      const double* __restrict__ d,
                                                      const double* __restrict__ q,
                                                      double* partial, unsigned* counter, double* scal) {
    constexpr int N = RefOps<P>::NPHI;
    if (scal[S::DONE] != 0.0) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const double alpha = scal[S::ALPHA];
    double v[1] = {0};
    if (i < ne) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const int64_t o = i * N + k;
            x[o] = fma(alpha, d[o], x[o]);
            const double rn = fma(-alpha, q[o], r[o]);
            r[o] = rn;
            v[0] = fma(rn, rn, v[0]);
        }
    }
    if (grid_sum<1>(v, partial, counter)) {
        const double rr = v[0];
        const double it = scal[S::ITER] + 1.0;
        scal[S::ITER] = it;
        scal[S::BETA] = rr / scal[S::RR];
        scal[S::RR] = rr;
        if (!isfinite(rr)) scal[S::DONE] = 3.0;
        else if (rr <= scal[S::TOL2]) scal[S::DONE] = 1.0;
        else if (it >= scal[S::MAXIT]) scal[S::DONE] = 2.0;
    }
}

// true residual ||K x - b_int||^2 and int x (gauge), kx = K x precomputed
template <int P>
__global__ __launch_bounds__(kBlock) void k_cg_resid(const RefOps<P>* __restrict__ ops,
                                                     const double4* __restrict__ geo, int64_t ne,
                                                     const double* __restrict__ kx,
                                                     const double* __restrict__ bint,
                                                     const double* __restrict__ x,
                                                     double* partial, unsigned* counter, double* scal) {
    constexpr int N = RefOps<P>::NPHI;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v[2] = {0, 0};
    if (i < ne) {
        const double4 e = geo[i];
        const double A = e.x * e.w - e.y * e.z;
        double s = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const int64_t o = i * N + k;
            const double t = kx[o] - bint[o];
            v[0] = fma(t, t, v[0]);
            s = fma(ops->w[k], x[o], s);
        }
        v[1] = A * s;
    }
    if (grid_sum<2>(v, partial, counter)) {
        scal[S::FLAG] = v[0];  // ||r_true||^2
        scal[S::MEAN] = v[1];  // int_Omega x
    }
}

__global__ __launch_bounds__(kBlock) void k_gauge_out(int64_t n, const double* __restrict__ x,
                                                      const double* scal, double inv_area,
                                                      double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    out[i] = x[i] - scal[S::MEAN] * inv_area;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <int P>
const RefOps<P>* ops_of(const sld_disc_s* d) { return reinterpret_cast<const RefOps<P>*>(d->ops_dev); }

#define SLD_DISPATCH(p, CALL)                 \
    switch (p) {                              \
        case 1: { constexpr int PP = 1; CALL; } break; \
        case 2: { constexpr int PP = 2; CALL; } break; \
        case 3: { constexpr int PP = 3; CALL; } break; \
        case 4: { constexpr int PP = 4; CALL; } break; \
        default: return hipErrorInvalidValue;  \
    }

}  // namespace

hipError_t launch_schur_apply(const sld_disc_s* d, const double* p, double* out, double scale,
                              hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_schur_apply<PP>, dim3(nblk(m->ne)), dim3(kBlock), 0, s,
                                          ops_of<PP>(d), m->geo, m->nbr, m->ne, p, out, scale));
    return hipGetLastError();
}

hipError_t launch_gradient(const sld_disc_s* d, const double* p, const double* vstar, double coef,
                           double* out, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_gradient<PP>, dim3(nblk(m->nd)), dim3(kBlock), 0, s,
                                          ops_of<PP>(d), m->geo, m->edges, m->nd, p, vstar, coef, out));
    return hipGetLastError();
}

hipError_t launch_divergence(const sld_disc_s* d, const double* v, double scale, double* out,
                             hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_divergence<PP>, dim3(nblk(m->ne)), dim3(kBlock), 0, s,
                                          ops_of<PP>(d), m->geo, m->nbr, m->tedges, m->ne, v, scale, out));
    return hipGetLastError();
}

hipError_t launch_cg_setup(const sld_disc_s* d, const double* b, const double* p0, bool warm,
                           double rtol, int maxit, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    const unsigned nb = nblk(m->ne);
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_cg_mean<PP>, dim3(nb), dim3(kBlock), 0, s, b, m->ne,
                                          w.partial, w.counter, w.scal));
    if (warm) {
        hipError_t e = hipMemcpyAsync(w.x, p0, sizeof(double) * m->ne * d->nphi,
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = launch_schur_apply(d, w.x, w.q, 1.0, s);
        if (e != hipSuccess) return e;
    }
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_cg_init<PP>, dim3(nb), dim3(kBlock), 0, s, b, w.q, m->ne,
                                          w.b, w.x, w.r, w.d[0], w.d[1], warm ? 1 : 0, rtol, maxit,
                                          w.partial, w.counter, w.scal));
    return hipGetLastError();
}

hipError_t launch_cg_iteration(const sld_disc_s* d, int parity, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    const unsigned nb = nblk(m->ne);
    const double* dold = w.d[parity];
    double* dnew = w.d[1 - parity];
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_cg_apply<PP>, dim3(nb), dim3(kBlock), 0, s, ops_of<PP>(d),
                                          m->geo, m->nbr, m->ne, w.r, dold, dnew, w.q, w.partial,
                                          w.counter, w.scal));
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_cg_update<PP>, dim3(nb), dim3(kBlock), 0, s, m->ne, w.x,
                                          w.r, dnew, w.q, w.partial, w.counter, w.scal));
    return hipGetLastError();
}

hipError_t launch_cg_apply_only(const sld_disc_s* d, int parity, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_cg_apply<PP>, dim3(nblk(m->ne)), dim3(kBlock), 0, s,
                                          ops_of<PP>(d), m->geo, m->nbr, m->ne, w.r, w.d[parity],
                                          w.d[1 - parity], w.q, w.partial, w.counter, w.scal));
    return hipGetLastError();
}

hipError_t launch_cg_update_only(const sld_disc_s* d, int parity, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_cg_update<PP>, dim3(nblk(m->ne)), dim3(kBlock), 0, s,
                                          m->ne, w.x, w.r, w.d[1 - parity], w.q, w.partial,
                                          w.counter, w.scal));
    return hipGetLastError();
}

hipError_t launch_cg_finish(const sld_disc_s* d, double* p_out, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    const unsigned nb = nblk(m->ne);
    hipError_t e = launch_schur_apply(d, w.x, w.q, 1.0, s);
    if (e != hipSuccess) return e;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_cg_resid<PP>, dim3(nb), dim3(kBlock), 0, s, ops_of<PP>(d),
                                          m->geo, m->ne, w.q, w.b, w.x, w.partial, w.counter, w.scal));
    const int64_t n = m->ne * d->nphi;
    hipLaunchKernelGGL(k_gauge_out, dim3(nblk(n)), dim3(kBlock), 0, s, n, w.x, w.scal,
                       1.0 / m->area_total, p_out);
    return hipGetLastError();
}
