// Standalone operator kernels: Schur apply K p, gradient Mhat^{-1} Q p (eq. ad4.2) and
// divergence D v (eq. D).  See device_common.h for the operator form.
#include "device_common.h"

using namespace sld_dev;

namespace {

constexpr int kBlockEdge = 128;

template <int P>
__global__ __launch_bounds__(kBlockTri) void k_schur_apply(const RefOps<P>* __restrict__ ops,
                                                           const double4* __restrict__ geo,
                                                           const int4* __restrict__ nbr, int64_t ne,
                                                           const double* __restrict__ p,
                                                           double* __restrict__ out, double scale) {
    constexpr int N = RefOps<P>::NPHI;
    __shared__ double sm[kTriPerBlock][4][N];
    const int tl = threadIdx.x / 3, al = threadIdx.x - 3 * (threadIdx.x / 3);
    const int64_t i = (int64_t)blockIdx.x * kTriPerBlock + tl;
    const bool valid = i < ne;
    if (valid) {
        double pl[N], y[N];
        LoadPlain<N> ld{p};
        schur_edge_lane<P>(i, al, *ops, geo, nbr, ld, pl, y);
        lds_scatter<P>(&sm[tl][0][0], al, y);
    }
    __syncthreads();
    if (valid) {
        for (int k = al; k < N; k += 3)
            out[i * N + k] = scale * (sm[tl][0][k] + sm[tl][1][k] + sm[tl][2][k]);
    }
}

// ---------------------------------------------------------------- gradient (lane per edge)
template <int P>
__global__ __launch_bounds__(kBlockEdge) void k_gradient(const RefOps<P>* __restrict__ ops,
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
    const int64_t j = (int64_t)blockIdx.x * kBlockEdge + threadIdx.x;
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
    for (int m = 0; m < NE; ++m) delta[m] = pr[(P - m)] - pl[m];
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
__global__ __launch_bounds__(kBlockEdge) void k_divergence(const RefOps<P>* __restrict__ ops,
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
    const int64_t i = (int64_t)blockIdx.x * kBlockEdge + threadIdx.x;
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
            y[edge_node(P, al, m)] += s;
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


inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

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

hipError_t launch_schur_apply(const sld_disc_s* d, const double* p, double* out, double scale,
                              hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_schur_apply<PP>, dim3(nblk(m->ne, kTriPerBlock)),
                                          dim3(kBlockTri), 0, s, ops_of<PP>(d), m->geo, m->nbr,
                                          m->ne, p, out, scale));
    return hipGetLastError();
}

hipError_t launch_gradient(const sld_disc_s* d, const double* p, const double* vstar, double coef,
                           double* out, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_gradient<PP>, dim3(nblk(m->nd, kBlockEdge)),
                                          dim3(kBlockEdge), 0, s, ops_of<PP>(d), m->geo, m->edges,
                                          m->nd, p, vstar, coef, out));
    return hipGetLastError();
}

hipError_t launch_divergence(const sld_disc_s* d, const double* v, double scale, double* out,
                             hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_divergence<PP>, dim3(nblk(m->ne, kBlockEdge)),
                                          dim3(kBlockEdge), 0, s, ops_of<PP>(d), m->geo, m->nbr,
                                          m->tedges, m->ne, v, scale, out));
    return hipGetLastError();
}
