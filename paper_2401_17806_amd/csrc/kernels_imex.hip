// Grid transfers between the main and the dual space (Section 4, eqs. d2m and m2d) and the
// right-hand side of the viscous solve, for the semi-Lagrangian IMEX step.
//
// dual -> main (eq. d2m): vbar_i = Mbar_i^{-1} sum_j U_ij^T vhat_j.  On triangle i's half of
// the dual cell of its local edge alpha the dual basis is the sub-triangle's Lagrange basis, so
// U_ij^T vhat_j = A_i V_alpha vh (vh: the half's nodal values) and Mbar_i = A_i Mref; the areas
// cancel and vbar_i = sum_alpha Ldm[alpha] vh_alpha with reference tables only.
//
// main -> dual (eq. m2d): vhat_j = Mhat_j^{-1} (U_lj vbar_l + U_rj vbar_r).  Restricted to one
// half, vbar_s is a polynomial of degree p in the half's coordinates, so U_sj vbar_s =
// (A_s/3) Mref a_s with a_s its values at the half's nodes, and Mhat_j = (A_l/3) Mref (+) (A_r/3)
// Mref glued on the p+1 shared edge nodes.  Static condensation onto those nodes gives the
// projection in closed form: on the edge u_H = (A_l a_l,H + A_r a_r,H) / (A_l + A_r) (the two
// halves' interface Schur complements are the same matrix), and inside each half
// u_I = a_I - Z (u_H - a_H).  A wall cell is its left half alone: u = a there.
#include "device_common.h"

using namespace sld_dev;

namespace {

constexpr int kBlockX = 128;

// One thread per triangle: out(i, c, :) = sum_alpha Ldm[alpha] vh_alpha(c).  vd [nd][nc][Npsi];
// out element (i, c, l) at out[i * o_is + c * o_cs + l].
template <int P>
__global__ __launch_bounds__(kBlockX) void k_dual_to_main(const RefOps<P>* __restrict__ ops,
                                                         const int4* __restrict__ tedges, int64_t ne,
                                                         const double* __restrict__ vd, int nc,
                                                         double* __restrict__ out, int64_t o_is,
                                                         int64_t o_cs) {
    constexpr int N = RefOps<P>::NPHI;
    constexpr int NPSI = (P + 1) * (P + 1);
    constexpr Tab<P> T{};
    const RefOps<P>& R = *ops;
    const int64_t i = (int64_t)blockIdx.x * kBlockX + threadIdx.x;
    if (i >= ne) return;
    const int4 te4 = tedges[i];
    for (int c = 0; c < nc; ++c) {
        double y[N];
#pragma unroll
        for (int l = 0; l < N; ++l) y[l] = 0.0;
#pragma unroll
        for (int al = 0; al < 3; ++al) {
            const int te = al == 0 ? te4.x : (al == 1 ? te4.y : te4.z);
            const int64_t j = te >> 1;
            const int beta = te & 1;
            const double* vj = vd + (j * nc + c) * NPSI;
            double vh[N];
#pragma unroll
            for (int n = 0; n < N; ++n) {
                const int a = T.na[n], b = T.nb[n];
                vh[n] = vj[beta ? (P - b) * (P + 1) + (P - a) : b * (P + 1) + a];
            }
#pragma unroll
            for (int l = 0; l < N; ++l) {
                double s = 0.0;
#pragma unroll
                for (int n = 0; n < N; ++n) s = fma(R.Ldm[al][l][n], vh[n], s);
                y[l] += s;
            }
        }
        double* o = out + i * o_is + c * o_cs;
#pragma unroll
        for (int l = 0; l < N; ++l) o[l] = y[l];
    }
}

// One thread per edge: out(j, c, :) [nd][nc][Npsi] from vm element (i, c, l) at
// vm[i * v_is + c * v_cs + l].
template <int P>
__global__ __launch_bounds__(kBlockX) void k_main_to_dual(const RefOps<P>* __restrict__ ops,
                                                         const double4* __restrict__ geo,
                                                         const int4* __restrict__ edges, int64_t nd,
                                                         const double* __restrict__ vm, int nc,
                                                         int64_t v_is, int64_t v_cs,
                                                         double* __restrict__ out) {
    constexpr int N = RefOps<P>::NPHI;
    constexpr int NE = P + 1;
    constexpr int NPSI = (P + 1) * (P + 1);
    constexpr Tab<P> T{};
    const RefOps<P>& R = *ops;
    const int64_t j = (int64_t)blockIdx.x * kBlockX + threadIdx.x;
    if (j >= nd) return;
    const int4 ed = edges[j];
    const bool wall = ed.y < 0;
    double wl = 1.0, wr = 0.0;
    if (!wall) {
        const double4 el = geo[ed.x], er = geo[ed.y];
        const double Al = el.x * el.w - el.y * el.z, Ar = er.x * er.w - er.y * er.z;
        wl = Al / (Al + Ar);
        wr = Ar / (Al + Ar);
    }
    for (int c = 0; c < nc; ++c) {
        double* o = out + (j * nc + c) * NPSI;
        // values of each side's polynomial at its half's nodes (frames relabelled so that the
        // shared edge is local edge 0)
        double al[N], ar[N];
        {
            const double* src = vm + (int64_t)ed.x * v_is + c * v_cs;
            double pl[N];
#pragma unroll
            for (int l = 0; l < N; ++l) pl[l] = src[rot_sel<P>(ed.z, l)];
#pragma unroll
            for (int n = 0; n < N; ++n) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < N; ++l) s = fma(R.Iv[n][l], pl[l], s);
                al[n] = s;
            }
        }
        if (!wall) {
            const double* src = vm + (int64_t)ed.y * v_is + c * v_cs;
            double pr[N];
#pragma unroll
            for (int l = 0; l < N; ++l) pr[l] = src[rot_sel<P>(ed.w, l)];
#pragma unroll
            for (int n = 0; n < N; ++n) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < N; ++l) s = fma(R.Iv[n][l], pr[l], s);
                ar[n] = s;
            }
        } else {
#pragma unroll
            for (int n = 0; n < N; ++n) ar[n] = 0.0;
        }
        // edge nodes: l's node m is r's node P - m
        double uH[NE], dL[NE], dR[NE];
#pragma unroll
        for (int m = 0; m < NE; ++m) {
            const double a_l = al[main_idx(P, P - m, m)];
            const double a_r = ar[main_idx(P, m, P - m)];
            uH[m] = wall ? a_l : wl * a_l + wr * a_r;
        }
#pragma unroll
        for (int m = 0; m < NE; ++m) {
            dL[m] = uH[m] - al[main_idx(P, P - m, m)];
            dR[m] = uH[P - m] - ar[main_idx(P, P - m, m)];
        }
        int ii = 0;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const int a = T.na[n], b = T.nb[n];
            if (a + b < P) {
                double zl = 0.0, zr = 0.0;
#pragma unroll
                for (int m = 0; m < NE; ++m) {
                    zl = fma(R.Z[ii][m], dL[m], zl);
                    zr = fma(R.Z[ii][m], dR[m], zr);
                }
                o[b * (P + 1) + a] = al[n] - zl;
                o[(P - b) * (P + 1) + (P - a)] = wall ? 0.0 : ar[n] - zr;
                ++ii;
            }
        }
#pragma unroll
        for (int m = 0; m < NE; ++m) o[m * (P + 1) + (P - m)] = uH[m];
    }
}

// b[i][k] = scale * A_i (Mref f_i)_k + gcoef * gb[i][k] and x0[i][l] = f_i,l for component c of
// f (element (i, c, l) at f[i * f_is + c * f_cs + l]); b, gb and x0 are [ne][Nphi].
template <int P>
__global__ __launch_bounds__(kBlockX) void k_mass_rhs(const RefOps<P>* __restrict__ ops,
                                                     const double4* __restrict__ geo, int64_t ne,
                                                     const double* __restrict__ f, int64_t f_is,
                                                     int64_t f_cs, int c, double scale,
                                                     const double* __restrict__ gb, double gcoef,
                                                     double* __restrict__ b, double* __restrict__ x0) {
    constexpr int N = RefOps<P>::NPHI;
    const RefOps<P>& R = *ops;
    const int64_t i = (int64_t)blockIdx.x * kBlockX + threadIdx.x;
    if (i >= ne) return;
    const double4 e = geo[i];
    const double A = e.x * e.w - e.y * e.z;
    const double* src = f + i * f_is + c * f_cs;
    double v[N];
#pragma unroll
    for (int l = 0; l < N; ++l) v[l] = src[l];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(R.Mref[k][l], v[l], s);
        b[i * N + k] = scale * A * s + (gb ? gcoef * gb[i * N + k] : 0.0);
        if (x0) x0[i * N + k] = v[k];
    }
}

// G_b of Dirichlet data on wall edges: for each triangle, the diffusion operator's wall-cell
// terms with the triangle's own field zero and the data u_b (at the p+1 edge nodes, counted
// from v_alpha) as the ghost trace -- the interior-edge form with a neighbour of zero area:
// on the edge nodes x_H = 3 |Gamma| n (C u_b) / A, then the line term |Gamma| M1 (n . x_H) and
// the sub-triangle correction -A sum_d Pt_alpha,d (G x_H)_d.
template <int P>
__global__ __launch_bounds__(kBlockX) void k_dirichlet_rhs(const RefOps<P>* __restrict__ ops,
                                                          const double4* __restrict__ geo,
                                                          const int4* __restrict__ nbr,
                                                          const int4* __restrict__ tedges, int64_t ne,
                                                          const unsigned char* __restrict__ mask,
                                                          const double* __restrict__ values,
                                                          double* __restrict__ out) {
    constexpr int N = RefOps<P>::NPHI;
    constexpr int NE = P + 1;
    const RefOps<P>& R = *ops;
    const int64_t i = (int64_t)blockIdx.x * kBlockX + threadIdx.x;
    if (i >= ne) return;
    const double4 e = geo[i];
    const Geo g = make_geo(e.x, e.y, e.z, e.w);
    const int4 nb4 = nbr[i], te4 = tedges[i];
    double y[N];
#pragma unroll
    for (int k = 0; k < N; ++k) y[k] = 0.0;
    for (int al = 0; al < 3; ++al) {
        const int nb = al == 0 ? nb4.x : (al == 1 ? nb4.y : nb4.z);
        if (nb >= 0) continue;
        const int64_t j = (al == 0 ? te4.x : (al == 1 ? te4.y : te4.z)) >> 1;
        if (!mask[j]) continue;
        double ex, ey;
        if (al == 0) { ex = e.x; ey = e.y; }
        else if (al == 1) { ex = e.z - e.x; ey = e.w - e.y; }
        else { ex = -e.z; ey = -e.w; }
        const double snx = ey, sny = -ex;
        const double* ub = values + j * NE;
        double tn[NE], gd0[NE], gd1[NE];
#pragma unroll
        for (int m = 0; m < NE; ++m) {
            double cd = 0.0;
#pragma unroll
            for (int q = 0; q < NE; ++q) cd = fma(R.C[m][q], ub[q], cd);
            const double hx = 3.0 * snx * cd / g.A, hy = 3.0 * sny * cd / g.A;
            tn[m] = snx * hx + sny * hy;
            gd0[m] = g.G00 * hx + g.G01 * hy;
            gd1[m] = g.G10 * hx + g.G11 * hy;
        }
#pragma unroll
        for (int m = 0; m < NE; ++m) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NE; ++q) s = fma(R.M1[m][q], tn[q], s);
            y[edge_node(P, al, m)] += s;
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < NE; ++m) {
                s = fma(R.Pt[al][0][k][m], gd0[m], s);
                s = fma(R.Pt[al][1][k][m], gd1[m], s);
            }
            y[k] = fma(-g.A, s, y[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < N; ++k) out[i * N + k] = y[k];
}

// Boussinesq: v*[j][1][:] += coef * t[j][:] on interior dual cells (buoyancy (0, g beta T) of
// eqs. nc.2 / pressure_IMEX over the step), and no-slip: zero velocity on the wall cells.
template <int P>
__global__ __launch_bounds__(kBlockX) void k_buoyancy(const int4* __restrict__ edges, int64_t nd,
                                                     const double* __restrict__ t, double coef,
                                                     double* __restrict__ vs) {
    constexpr int NPSI = (P + 1) * (P + 1);
    const int64_t j = (int64_t)blockIdx.x * kBlockX + threadIdx.x;
    if (j >= nd) return;
    double* o = vs + j * 2 * NPSI;
    if (edges[j].y < 0) {
#pragma unroll
        for (int k = 0; k < 2 * NPSI; ++k) o[k] = 0.0;
        return;
    }
#pragma unroll
    for (int k = 0; k < NPSI; ++k) o[NPSI + k] = fma(coef, t[j * NPSI + k], o[NPSI + k]);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlockX - 1) / kBlockX); }

template <int P>
const RefOps<P>* ops_of(const sld_disc_s* d) { return reinterpret_cast<const RefOps<P>*>(d->ops_dev); }

}  // namespace

#define SLD_DISPATCH(p, CALL)                                   \
    switch (p) {                                                \
        case 1: { constexpr int PP = 1; CALL; } break;          \
        case 2: { constexpr int PP = 2; CALL; } break;          \
        case 3: { constexpr int PP = 3; CALL; } break;          \
        case 4: { constexpr int PP = 4; CALL; } break;          \
        default: return hipErrorInvalidValue;                   \
    }

hipError_t launch_dual_to_main(const sld_disc_s* d, const double* vd, int nc, double* out,
                               int64_t o_is, int64_t o_cs, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_dual_to_main<PP>, dim3(nblk(m->ne)), dim3(kBlockX), 0,
                                          s, ops_of<PP>(d), m->tedges, m->ne, vd, nc, out, o_is,
                                          o_cs));
    return hipGetLastError();
}

hipError_t launch_main_to_dual(const sld_disc_s* d, const double* vm, int nc, int64_t v_is,
                               int64_t v_cs, double* out, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_main_to_dual<PP>, dim3(nblk(m->nd)), dim3(kBlockX), 0,
                                          s, ops_of<PP>(d), m->geo, m->edges, m->nd, vm, nc, v_is,
                                          v_cs, out));
    return hipGetLastError();
}

hipError_t launch_mass_rhs(const sld_disc_s* d, const double* f, int64_t f_is, int64_t f_cs, int c,
                           double scale, const double* gb, double gcoef, double* b, double* x0,
                           hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_mass_rhs<PP>, dim3(nblk(m->ne)), dim3(kBlockX), 0, s,
                                          ops_of<PP>(d), m->geo, m->ne, f, f_is, f_cs, c, scale, gb,
                                          gcoef, b, x0));
    return hipGetLastError();
}

hipError_t launch_dirichlet_rhs(const sld_disc_s* d, const unsigned char* edge_mask,
                                const double* values, double* out, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_dirichlet_rhs<PP>, dim3(nblk(m->ne)), dim3(kBlockX), 0,
                                          s, ops_of<PP>(d), m->geo, m->nbr, m->tedges, m->ne,
                                          edge_mask, values, out));
    return hipGetLastError();
}

hipError_t launch_buoyancy(const sld_disc_s* d, const double* t, double coef, double* vs,
                           hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_buoyancy<PP>, dim3(nblk(m->nd)), dim3(kBlockX), 0, s,
                                          m->edges, m->nd, t, coef, vs));
    return hipGetLastError();
}
