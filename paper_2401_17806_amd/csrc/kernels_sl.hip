// Semi-Lagrangian advection of main-grid DG fields (Section 3.5; the Gauss-point projection of
// the SL-IMEX stages, eq. intstage).
//
// One thread per (triangle, Gauss point).  The thread follows the backward characteristic
// from its Gauss point cell by cell with straight (explicit Euler) segments: inside the current
// cell the velocity is that cell's DG velocity at the segment's start, the segment ends where
// the ray leaves the cell (the first barycentric coordinate to reach zero, ties to the lowest
// vertex) or where the remaining time runs out.  Crossing an interior edge continues in the
// neighbour at the same point, expressed in the neighbour's barycentric coordinates through the
// shared edge (so periodic boxes need no coordinate wrap); a wall edge, or a cell whose velocity
// points straight back out, ends the walk where it is.  The fields are evaluated at the foot
// with the DG polynomial of the cell reached, staged in LDS, and projected onto the main basis
// of the starting triangle (q_new = M_ref^{-1} sum_g w_g phi(xi_g) q(foot_g)).
//
// Everything per cell is read from the caller-order tables (edge vectors, neighbour codes): no
// absolute coordinates are needed.
#include "device_common.h"

using namespace sld_dev;

namespace {

constexpr int kSlBlock = 256;
constexpr int kSlMaxSteps = 1024;  // segments per point (CFL-sized steps need a handful)

// Main Lagrange basis of degree P at (xi, eta): product form over the integer barycentric
// coordinates of each node, L_m(t) = prod_{q<m} (t - q) / (q + 1).
template <int P>
__device__ __forceinline__ void eval_phi(double xi, double eta, double (&phi)[RefOps<P>::NPHI]) {
    double la[P + 1], lb[P + 1], lc[P + 1];
    const double ta = P * xi, tb = P * eta, tc = P * (1.0 - xi - eta);
    la[0] = lb[0] = lc[0] = 1.0;
#pragma unroll
    for (int m = 1; m <= P; ++m) {
        const double inv = 1.0 / m;
        la[m] = la[m - 1] * (ta - (m - 1)) * inv;
        lb[m] = lb[m - 1] * (tb - (m - 1)) * inv;
        lc[m] = lc[m - 1] * (tc - (m - 1)) * inv;
    }
    int k = 0;
#pragma unroll
    for (int b = 0; b <= P; ++b)
#pragma unroll
        for (int a = 0; a <= P - b; ++a, ++k) phi[k] = la[a] * lb[b] * lc[P - a - b];
}

template <int P>
__global__ __launch_bounds__(kSlBlock) void k_sl_advect(const SlOps<P>* __restrict__ sl,
                                                        const double4* __restrict__ geo,
                                                        const int4* __restrict__ nbr, int64_t ne,
                                                        const double* __restrict__ vbar,
                                                        const double* __restrict__ q, int nc,
                                                        double dt, double* __restrict__ out) {
    constexpr int N = RefOps<P>::NPHI;
    constexpr int NG = SlOps<P>::NG;
    constexpr int TB = kSlBlock / NG;  // triangles per block
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double* sq = reinterpret_cast<double*>(lds_raw);  // [TB][NG][nc] values at the feet
    double* sv = sq + (size_t)kSlBlock * nc;          // [TB][2][N] velocity of the block's cells
    double* sf = sv + (size_t)TB * 2 * N;             // [TB][nc][N] fields of the block's cells
    double* sp = sf + (size_t)TB * nc * N;            // [N][NG] projection matrix
    const int tloc = threadIdx.x / NG, g = threadIdx.x - (threadIdx.x / NG) * NG;
    const int64_t tri0 = (int64_t)blockIdx.x * TB;
    const int64_t i = tri0 + tloc;
    const int64_t nt = (ne - tri0) < TB ? (ne - tri0) : TB;
    // the block's own cells (where most walks start and, at moderate CFL, end) staged in LDS
    // with coalesced loads
    for (int f = threadIdx.x; f < (int)nt * 2 * N; f += kSlBlock) sv[f] = vbar[tri0 * 2 * N + f];
    for (int f = threadIdx.x; f < (int)nt * nc * N; f += kSlBlock) sf[f] = q[tri0 * nc * N + f];
    for (int f = threadIdx.x; f < N * NG; f += kSlBlock) sp[f] = (&sl->proj[0][0])[f];
    __syncthreads();
    if (tloc < TB && i < ne) {
        int64_t c = i;
        double l1 = sl->pts[g][0], l2 = sl->pts[g][1];
        double l0 = 1.0 - l1 - l2;
        double tau = dt;
        for (int step = 0; step < kSlMaxSteps; ++step) {
            double phi[N];
            eval_phi<P>(l1, l2, phi);
            double ux = 0.0, uy = 0.0;
            const bool own = c >= tri0 && c < tri0 + nt;
            const double* vc = own ? sv + (c - tri0) * 2 * N : vbar + c * 2 * N;
#pragma unroll
            for (int l = 0; l < N; ++l) {
                ux = fma(vc[l], phi[l], ux);
                uy = fma(vc[N + l], phi[l], uy);
            }
            const double4 e = geo[c];
            const Geo gd = make_geo(e.x, e.y, e.z, e.w);
            const double d1 = gd.G00 * ux + gd.G01 * uy;  // reference velocity
            const double d2 = gd.G10 * ux + gd.G11 * uy;
            const double dl[3] = {-(d1 + d2), d1, d2};
            const double lam[3] = {l0, l1, l2};
            // the coordinate that reaches zero first (smallest lam_k / dl_k over dl_k > 0;
            // ties to the lowest k), compared by cross-multiplication; one division, and only
            // when the segment leaves the cell
            int k_star = -1;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (dl[k] > 0.0) {
                    if (k_star < 0) {
                        k_star = k;
                    } else {
                        const double lk = k_star == 0 ? lam[0] : (k_star == 1 ? lam[1] : lam[2]);
                        const double dk = k_star == 0 ? dl[0] : (k_star == 1 ? dl[1] : dl[2]);
                        if (lam[k] * dk < lk * dl[k]) k_star = k;
                    }
                }
            }
            const double lks = k_star == 0 ? lam[0] : (k_star == 1 ? lam[1] : lam[2]);
            const double dks = k_star == 0 ? dl[0] : (k_star == 1 ? dl[1] : dl[2]);
            if (k_star < 0 || lks >= tau * dks) {
                l0 -= tau * dl[0];
                l1 -= tau * dl[1];
                l2 -= tau * dl[2];
                break;
            }
            const double s_star = lks / dks;
            if (s_star <= 0.0) break;  // cannot move: stop here
            double nl[3] = {fmax(l0 - s_star * dl[0], 0.0), fmax(l1 - s_star * dl[1], 0.0),
                            fmax(l2 - s_star * dl[2], 0.0)};
            nl[k_star] = 0.0;
            tau -= s_star;
            const int alpha = k_star == 2 ? 0 : k_star + 1;  // edge opposite vertex k_star
            const int nb = pick(nbr[c], alpha);
            if (nb < 0) {  // wall: the foot stays on the wall
                l0 = nl[0];
                l1 = nl[1];
                l2 = nl[2];
                break;
            }
            // position along v_alpha -> v_alpha+1; the neighbour's edge ar runs the other way
            const double t = fmin(fmax(nl[alpha == 2 ? 0 : alpha + 1], 0.0), 1.0);
            const int ar = nb & 3;
            double ml[3] = {0.0, 0.0, 0.0};
            ml[ar] = t;
            ml[ar == 2 ? 0 : ar + 1] = 1.0 - t;
            l0 = ml[0];
            l1 = ml[1];
            l2 = ml[2];
            c = nb >> 2;
        }
        double phi[N];
        eval_phi<P>(l1, l2, phi);
        const double* qc = (c >= tri0 && c < tri0 + nt) ? sf + (c - tri0) * nc * N
                                                        : q + c * (int64_t)nc * N;
        for (int cmp = 0; cmp < nc; ++cmp) {
            double v = 0.0;
#pragma unroll
            for (int l = 0; l < N; ++l) v = fma(qc[cmp * N + l], phi[l], v);
            sq[(tloc * NG + g) * nc + cmp] = v;
        }
    }
    __syncthreads();
    // projection onto the main basis of each starting triangle (fixed summation order)
    const int nout = (int)nt * nc * N;
    for (int f = threadIdx.x; f < nout; f += kSlBlock) {
        const int t = f / (nc * N);
        const int rem = f - t * nc * N;
        const int cmp = rem / N, k = rem - (rem / N) * N;
        double s = 0.0;
#pragma unroll
        for (int gg = 0; gg < NG; ++gg) s = fma(sp[k * NG + gg], sq[(t * NG + gg) * nc + cmp], s);
        out[(tri0 + t) * nc * N + rem] = s;
    }
}

}  // namespace

template <int P>
size_t sl_lds_bytes(int nc) {
    constexpr int N = RefOps<P>::NPHI, TB = kSlBlock / SlOps<P>::NG;
    return sizeof(double) * ((size_t)kSlBlock * nc + (size_t)TB * (2 + nc) * N +
                             (size_t)N * SlOps<P>::NG);
}

hipError_t launch_sl_advect(const sld_disc_s* d, const double* vbar, const double* q, int nc,
                            double dt, double* out, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    switch (d->p) {
#define SLD_SL(PP)                                                                               \
    case PP: {                                                                                   \
        constexpr int TB = kSlBlock / SlOps<PP>::NG;                                             \
        const unsigned nb = (unsigned)((m->ne + TB - 1) / TB);                                   \
        const size_t lds = sl_lds_bytes<PP>(nc);                                                 \
        hipLaunchKernelGGL(k_sl_advect<PP>, dim3(nb), dim3(kSlBlock), lds, s,                    \
                           reinterpret_cast<const SlOps<PP>*>(d->sl_dev), m->geo, m->nbr, m->ne, \
                           vbar, q, nc, dt, out);                                                \
    } break;
        SLD_SL(1)
        SLD_SL(2)
        SLD_SL(3)
        SLD_SL(4)
#undef SLD_SL
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
