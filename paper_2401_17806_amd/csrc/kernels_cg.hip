// Matrix-free conjugate gradients on -K (Section 3.3: the pressure system of eq.
// pressure_final is symmetric, so CG applies; K itself is negative semi-definite).
//
// One iteration = ONE kernel on a fixed grid of G blocks (k_cg_step).  Launch k reads the
// state (r, q, d)_{k-1} written by launch k-1 (ping-pong buffers by parity) and the G
// partials of four dot products of launch k-1, and in a single pass over the triangles
//   alpha_{k-1} = rr_{k-1} / dq_{k-1}
//   rr_k(rec)   = rr_{k-1} - 2 alpha rq_{k-1} + alpha^2 qq_{k-1}     (one-step recurrence
//                 from a directly summed rr_{k-1}, so rounding does not accumulate)
//   beta_{k-1}  = rr_k(rec) / rr_{k-1}
//   r_k = r_{k-1} - alpha q_{k-1},  d_k = r_k + beta d_{k-1},  x += alpha d_{k-1}
//   q_k = -K d_k   (neighbours' r_k, d_k are recomputed from their (r, q, d)_{k-1})
//   partials of rr_k = r_k.r_k, dq_k = d_k.q_k, rq_k = r_k.q_k, qq_k = q_k.q_k.
// In exact arithmetic this is plain CG (Section 3.3).  The kShift instantiation solves the
// viscous system of the IMEX step instead: K is replaced by K - sigma Mbar (Mbar_i = A_i Mref,
// sigma = scal[SIGMA] > 0), i.e. CG on sigma Mbar - K, which is positive definite.
// Global scalars are never published
// through in-kernel atomics: every block sums the previous launch's partials itself in a
// fixed order, so all blocks take bitwise identical decisions and results are deterministic.
// The iteration counter is double-buffered by parity for the same reason.
#include <mutex>

#include "device_common.h"

using namespace sld_dev;

namespace {

typedef CgScalars S;

// blocks of the FP32 iteration and of the kernels that write or read its dot partials (the MFMA
// form runs on the FP64 grid)
inline int rel_grid(const CgWork& w) { return w.use_mx ? w.grid : w.grid32; }

// row k of Mref v
template <int P>
__device__ __forceinline__ double mass_row(const RefOps<P>& R, int k,
                                           const double (&v)[RefOps<P>::NPHI]) {
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < RefOps<P>::NPHI; ++l) s = fma(R.Mref[k][l], v[l], s);
    return s;
}

// (K - sigma Mbar) x on row k of triangle i, from the lanes' sum kx of (K x)_ik
template <int P>
__device__ __forceinline__ double shifted_row(const RefOps<P>& R, const double4* __restrict__ geo,
                                              const double* __restrict__ x, int64_t i, int k,
                                              double kx, double sigma) {
    constexpr int N = RefOps<P>::NPHI;
    if (sigma == 0.0) return kx;
    const double4 e = geo[i];
    const double A = e.x * e.w - e.y * e.z;
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < N; ++l) s = fma(R.Mref[k][l], x[i * N + l], s);
    return fma(-sigma * A, s, kx);
}

// Wall treatment of local edge al of internal triangle i: the pressure operator has no wall
// cells; the mass-shifted (diffusion) system has Dirichlet or zero-flux wall cells, the
// Dirichlet edges flagged in wall_i (bit al).
__device__ __forceinline__ int wall_kind(bool diffusion, const unsigned char* __restrict__ wall_i,
                                         int64_t i, int al) {
    if (!diffusion) return kWallAbsent;
    return (wall_i != nullptr && ((wall_i[i] >> al) & 1)) ? kWallDirichlet : kWallFlux;
}

// r = K x - b_int (true residual of the CG system -K x = -b_int) and its rr partials.
template <int P>
__global__ __launch_bounds__(kBlockTri) void k_cg_resid(const RefOps<P>* __restrict__ ops,
                                                        const double4* __restrict__ geo,
                                                        const int4* __restrict__ nbr, int64_t ne,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ bint,
                                                        double* __restrict__ r,
                                                        double* __restrict__ part_out,
                                                        const double* __restrict__ scal,
                                                        double sigma,
                                                        const unsigned char* __restrict__ wall_i,
                                                        int always) {
    constexpr int N = RefOps<P>::NPHI;
    // (skipped when the setup found a zero right-hand side, unless asked for regardless)
    if (!always && scal[S::DONE] != 0.0) return;
    __shared__ double sm[kTriPerBlock][4][N];
    const int tl = threadIdx.x / 3, al = threadIdx.x - 3 * (threadIdx.x / 3);
    double acc[1] = {0.0};
    for (int64_t tile = blockIdx.x; tile * kTriPerBlock < ne; tile += gridDim.x) {
        const int64_t i = tile * kTriPerBlock + tl;
        const bool valid = i < ne;
        if (valid) {
            double pl[N], y[N];
            LoadPlain<N> ld{x};
            schur_edge_lane<P>(i, al, *ops, geo, nbr, ld, pl, y,
                               wall_kind(sigma != 0.0, wall_i, i, al));
            lds_scatter<P>(&sm[tl][0][0], al, y);
        }
        __syncthreads();
        if (valid) {
            for (int k = al; k < N; k += 3) {
                const double v = shifted_row<P>(*ops, geo, x, i, k,
                                                sm[tl][0][k] + sm[tl][1][k] + sm[tl][2][k], sigma) -
                                 bint[i * N + k];
                r[i * N + k] = v;
                acc[0] = fma(v, v, acc[0]);
            }
        }
        __syncthreads();
    }
    block_sum_all<1, kBlockTri>(acc);
    if (threadIdx.x == 0) part_out[blockIdx.x] = acc[0];
}

// The previous launch's G partials of the four CG dots, summed in a fixed order (every block
// gets bitwise the same totals); four partials per thread and dot are in flight at a time.
// The same sum with its first pass (partials threadIdx.x + u NT, u < 4) requested ahead of it;
// the order of the additions is the same.
template <int NT>
struct DotPartials {
    double w[4][4];
    __device__ __forceinline__ void load(const double* __restrict__ part_in, int G, int b0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = b0 + u * NT;
#pragma unroll
            for (int c = 0; c < 4; ++c) w[u][c] = b < G ? part_in[c * G + b] : 0.0;
        }
    }
    __device__ __forceinline__ void add(double (&v)[4]) const {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] += w[u][c];
    }
    // v = the totals, given the first pass loaded
    __device__ __forceinline__ void sum(const double* __restrict__ part_in, int G, double (&v)[4]) {
        add(v);
        for (int b0 = threadIdx.x + 4 * NT; b0 < G; b0 += 4 * NT) {
            load(part_in, G, b0);
            add(v);
        }
        block_sum_all<4, NT>(v);
    }
};

template <int NT>
__device__ __forceinline__ void sum_dot_partials(const double* __restrict__ part_in, int G,
                                                 double (&v)[4]) {
    for (int b0 = threadIdx.x; b0 < G; b0 += 4 * NT) {
        double w[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = b0 + u * NT;
#pragma unroll
            for (int c = 0; c < 4; ++c) w[u][c] = b < G ? part_in[c * G + b] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] += w[u][c];
    }
    block_sum_all<4, NT>(v);
}

// Centring of the FP32 operator inputs.  Every piece of K that one lane or wave evaluates -- the
// volume term and the coupling through one edge -- maps constants to zero: the reference
// stiffness and edge-derivative rows sum to zero and the jump of a constant vanishes (the
// pressure operator's wall pieces give back a sub-triangle stiffness share, which does the
// same).  So the piece may subtract any one value c from all the DOFs it reads, its own and the
// neighbour's, without changing its result in exact arithmetic.  In FP32 it changes a lot: for
// the smooth modes that CG resolves last, the DOFs a piece reads agree to many digits, the
// reference contractions cancel them, and the rounding of those sums (relative to |p|, not to
// the differences) swamps the small result.  With c = the triangle's first DOF the sums see
// only the local variation.  Measured on the 512x512x2, p = 3 Taylor-Green pressure solve: the
// mixed form's FP32 iterations fall from 28758 to 19491 (FP64 CG: 17765), the same count as with
// the operator evaluated in FP64 arithmetic on FP32 vectors.  The FP64 kernel is left as it is.
// v -= c on every entry
template <typename Real, int N>
__device__ __forceinline__ void centre(Real (&v)[N], Real c) {
#pragma unroll
    for (int l = 0; l < N; ++l) v[l] -= c;
}

// Dynamic LDS of k_cg_step, in words of the arithmetic type: sd [(T + hmax) N] directions d_k
// of the tile then of its halo; sr [T N] residuals r_k of the tile; sm [T][R][N] partial rows
// (R = 4 roles in the one-tile-per-block variant, 3 lanes otherwise).
inline size_t step_lds_bytes(int nphi, int hmax, size_t real_bytes, bool front) {
    return real_bytes * (size_t)nphi *
           (size_t)(kTriPerBlock + hmax + kTriPerBlock + (front ? 4 : 3) * kTriPerBlock);
}

// kFront: the grid has one tile per block (cache-resident meshes, latency-bound).  The tile's
// state and its halo ids are requested at entry, together with the scalars; the previous
// launch's dot partials follow as soon as the iteration scalar shows there are any, so these
// latencies overlap (requesting more at entry -- the halo values, the phase-2 geometry, the
// partials unconditionally -- measured slower).  With several tiles per block the loads follow
// the tile loop.
template <int P, typename Real, class Ops, bool kFront, bool kShift, bool kStream>
__global__ __launch_bounds__(kFront ? kBlockCG : kBlockTri) void k_cg_step(const Ops* __restrict__ ops,
                                                       const double4* __restrict__ geo,
                                                       const double4* __restrict__ geo_nb,
                                                       const int4* __restrict__ nbr,
                                                       const int* __restrict__ halo_pad, int hmax,
                                                       int64_t ne,
                                                       const unsigned char* __restrict__ wall_i,
                                                       Real* __restrict__ x,
                                                       const Real* __restrict__ r_in,
                                                       const Real* __restrict__ q_in,
                                                       const Real* __restrict__ d_in,
                                                       Real* __restrict__ r_out,
                                                       Real* __restrict__ q_out,
                                                       Real* __restrict__ d_out,
                                                       const double* __restrict__ part_in,
                                                       double* __restrict__ part_out,
                                                       double* __restrict__ scal, int parity) {
    constexpr int N = RefOps<P>::NPHI;
    constexpr int T = kTriPerBlock;
    constexpr int NT = kFront ? kBlockCG : kBlockTri;  // threads
    constexpr int R = kFront ? 4 : 3;                  // partial rows per triangle
    constexpr int PER = (T * N + NT - 1) / NT;  // tile entries per thread
    constexpr int HB = 4;                                     // halo entries per thread and batch
    // FP32 operator inputs centred per piece (see centre above)
    constexpr bool kCentre = sizeof(Real) == 4 && !kShift;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Real* sd = reinterpret_cast<Real*>(lds_raw);
    Real* sr = sd + (size_t)(T + hmax) * N;
    Real* sm = sr + (size_t)T * N;
    const int G = gridDim.x;
    const int hs = hmax > 0 ? hmax : 1;  // row stride of halo_pad
    const int nhe = hmax * N;            // halo entries (padded) of a tile
    // This block's tiles: one contiguous chunk of the (Morton-ordered) tile range.  The
    // dispatcher places block b on XCD b mod 8, so logical chunk (b mod 8) * G/8 + b/8 gives
    // the blocks of one XCD a contiguous stretch of the mesh whose halos stay in that XCD's L2.
    // G is a multiple of 8 (host side), so the map is a bijection onto the G chunks.
    const int64_t ntiles = (ne + T - 1) / T;
    const int lb = (int)(blockIdx.x & 7) * (G >> 3) + (int)(blockIdx.x >> 3);
    const int64_t per = (ntiles + G - 1) / G;
    const int64_t t_begin = lb * per;
    const int64_t t_end = (lb + 1) * per < ntiles ? (lb + 1) * per : ntiles;

    Real vd[PER], vq[PER], vr[PER], vx[PER];
    int hid[HB];
    // state of tile `tile` into registers
    auto load_own = [&](int64_t tile) {
        const int64_t i0 = tile * T;
        const int nown = (int)((ne - i0) < T ? (ne - i0) : T) * N;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int f = threadIdx.x + u * NT;
            if (f < nown) {
                const int64_t o = i0 * N + f;
                vd[u] = d_in[o];
                vq[u] = q_in[o];
                vr[u] = r_in[o];
                vx[u] = x[o];
            }
        }
    };
    // halo triangle ids of one batch of halo entries (-1: padding)
    auto load_hid = [&](int64_t tile, int e0) {
#pragma unroll
        for (int u = 0; u < HB; ++u) {
            const int e = e0 + threadIdx.x + u * NT;
            hid[u] = e < nhe ? halo_pad[tile * hs + e / N] : -1;
        }
    };
    // FP32 state, one tile per block: the dot partials are requested first (whatever the
    // iteration count; unused on the first launch), since loads return in order and the sum
    // then need not wait for the tile's state.  Measured on a 128x128x2, p = 3 mesh: 2% faster
    // per FP32 iteration, but 4% slower per FP64 one, which keeps the order below.
    constexpr bool kEarlyPartials = kFront && sizeof(Real) == 4;
    DotPartials<NT> dp;
    if constexpr (kFront) {
        if constexpr (kEarlyPartials) dp.load(part_in, G, threadIdx.x);
        if (t_begin < t_end) {
            load_own(t_begin);
            load_hid(t_begin, 0);
        }
    }
    const double done = scal[S::DONE];
    const double it = scal[S::ITER0 + parity];
    double alpha = 0.0, beta = 0.0;
    if (it > 0.0) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        if constexpr (kEarlyPartials) dp.sum(part_in, G, v);
        else sum_dot_partials<NT>(part_in, G, v);
        const double rr = v[0], dq = v[1], rq = v[2], qq = v[3];
        if (done != 0.0) return;
        // every block takes the same decision from the same sums
        int stop = 0;
        if (!isfinite(rr)) stop = 3;
        else if (rr <= scal[S::TOL2]) stop = S::kConverged;
        else if (rr <= scal[S::RTH]) stop = S::kRefresh;
        else if (!(dq > 0.0) || !isfinite(dq)) stop = S::kBreakdown;
        else if (it > scal[S::MAXIT]) stop = S::kMaxit;
        if (stop) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                scal[S::DONE] = (double)stop;
                scal[S::RR] = rr;
                scal[S::ITER] = it - 1.0;  // iterations whose update reached x
            }
            return;
        }
        alpha = rr / dq;
        const double rr_next = fma(alpha * alpha, qq, fma(-2.0 * alpha, rq, rr));
        beta = rr_next / rr;
    } else if (done != 0.0) {
        return;
    }
    const Real ra = (Real)alpha, rb = (Real)beta;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t tile = t_begin; tile < t_end; ++tile) {
        const int64_t i0 = tile * T;
        const int nown = (int)((ne - i0) < T ? (ne - i0) : T) * N;
        const int64_t base = i0 * N;
        // phase 1: state update of the tile (coalesced) and directions of tile + halo into LDS
        if constexpr (kFront) {
            // the loads were issued at entry.  The state is stored non-temporally: the next
            // launch reads it after the kernel boundary (from the memory-side cache, never from
            // this XCD's L2), and streaming stores were measured 3% faster per iteration on a
            // 128x128x2, p = 3 mesh
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int f = threadIdx.x + u * NT;
                if (f < nown) {
                    const int64_t o = base + f;
                    const Real rk = mad(-ra, vq[u], vr[u]);
                    const Real dk = mad(rb, vd[u], rk);
                    __builtin_nontemporal_store(mad(ra, vd[u], vx[u]), &x[o]);
                    __builtin_nontemporal_store(rk, &r_out[o]);
                    __builtin_nontemporal_store(dk, &d_out[o]);
                    sd[f] = dk;
                    sr[f] = rk;
                    acc[0] = fma((double)rk, (double)rk, acc[0]);
                }
            }
            for (int e0 = 0; e0 < nhe; e0 += HB * NT) {
                if (e0 > 0) load_hid(tile, e0);
                Real hd[HB], hq[HB], hr[HB];
#pragma unroll
                for (int u = 0; u < HB; ++u) {
                    if (hid[u] >= 0) {
                        const int e = e0 + threadIdx.x + u * NT;
                        const int64_t o = (int64_t)hid[u] * N + (e - (e / N) * N);
                        hd[u] = d_in[o];
                        hq[u] = q_in[o];
                        hr[u] = r_in[o];
                    }
                }
#pragma unroll
                for (int u = 0; u < HB; ++u) {
                    if (hid[u] >= 0) {
                        const int e = e0 + threadIdx.x + u * NT;
                        sd[T * N + e] = mad(rb, hd[u], mad(-ra, hq[u], hr[u]));
                    }
                }
            }
        } else {
            // several tiles per block: plain loops (fewer live registers, higher occupancy).
            // x is private to the tile; when the working set outgrows the memory-side cache it
            // is streamed with non-temporal accesses, leaving that cache to the vectors the
            // neighbours' halos read
            for (int f = threadIdx.x; f < nown; f += NT) {
                const int64_t o = base + f;
                const Real dprev = d_in[o];
                const Real rk = mad(-ra, q_in[o], r_in[o]);
                const Real dk = mad(rb, dprev, rk);
                // (a compile-time choice: a runtime branch lets the compiler merge the two
                // accesses and drop the non-temporal hint)
                if constexpr (kStream)
                    __builtin_nontemporal_store(mad(ra, dprev, __builtin_nontemporal_load(&x[o])), &x[o]);
                else
                    x[o] = mad(ra, dprev, x[o]);
                r_out[o] = rk;
                d_out[o] = dk;
                sd[f] = dk;
                sr[f] = rk;
                acc[0] = fma((double)rk, (double)rk, acc[0]);
            }
            // halo ids of two entries first, then their values (two gathers in flight)
            for (int e0 = threadIdx.x; e0 < nhe; e0 += 2 * NT) {
                int id2[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int e = e0 + u * NT;
                    id2[u] = e < nhe ? halo_pad[tile * hs + e / N] : -1;
                }
                Real hd[2], hq[2], hr[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    if (id2[u] >= 0) {
                        const int e = e0 + u * NT;
                        const int64_t o = (int64_t)id2[u] * N + (e - (e / N) * N);
                        hd[u] = d_in[o];
                        hq[u] = q_in[o];
                        hr[u] = r_in[o];
                    }
                }
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    if (id2[u] >= 0) sd[T * N + e0 + u * NT] = mad(rb, hd[u], mad(-ra, hq[u], hr[u]));
            }
        }
        __syncthreads();
        if constexpr (kFront) {
            // phase 2: one wave per role (waves 0..2: local edge 0..2, wave 3: volume term), one
            // lane per triangle, operands from LDS.  Four waves per tile keep the SIMDs of a
            // CU evenly loaded when the grid is a single tile per block.
            const int role = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
            const int lane = threadIdx.x & 63;
            const int64_t i = i0 + lane;
            if (i < ne) {
                Real pl[N], y[N];
#pragma unroll
                for (int l = 0; l < N; ++l) pl[l] = sd[lane * N + l];
                [[maybe_unused]] const Real c = pl[0];
                const double4 e = geo[i];
                if (role == 3) {
                    if constexpr (kCentre) centre(pl, c);
                    volume_wave_core<P, Ops, Real>(*ops, e, pl, y);
                    if constexpr (kShift) {
                        const double sa = -scal[S::SIGMA] * (e.x * e.w - e.y * e.z);
#pragma unroll
                        for (int k = 0; k < N; ++k) y[k] = fma(sa, mass_row<P>(*ops, k, pl), y[k]);
                    }
                } else {
                    const int4 nb4 = nbr[i];
                    const int nb = pick(nb4, role);
                    const int slot = (nb4.w >> (10 * role)) & 1023;
                    Real pr[N];
                    int ar = 0;
                    // the neighbour's geometry from the per-edge copy, requested with nbr[i]
                    // rather than after it: 1.4% faster per iteration on a 128x128x2, p = 3
                    // mesh, where the launch is latency-bound
                    const double4 er = geo_nb[i * 3 + role];
                    if (nb >= 0) {
                        ar = nb & 3;
#pragma unroll
                        for (int l = 0; l < N; ++l) pr[l] = sd[slot * N + rot_sel<P>(ar, l)];
                        if constexpr (kCentre) centre(pr, c);
                    } else {
#pragma unroll
                        for (int l = 0; l < N; ++l) pr[l] = Real(0);
                    }
                    if constexpr (kCentre) centre(pl, c);
                    const int wk = wall_kind(kShift, wall_i, i, role);
                    if (role == 0) edge_wave_core<P, 0, Ops, Real>(*ops, e, nb, ar, er, pl, pr, y, wk);
                    else if (role == 1) edge_wave_core<P, 1, Ops, Real>(*ops, e, nb, ar, er, pl, pr, y, wk);
                    else edge_wave_core<P, 2, Ops, Real>(*ops, e, nb, ar, er, pl, pr, y, wk);
                }
#pragma unroll
                for (int k = 0; k < N; ++k) sm[(lane * 4 + role) * N + k] = y[k];
            }
        } else {
            // phase 2: three lanes per triangle (lane al owns local edge al, in the frame
            // relabelled so that it is edge 0), operands from LDS
            const int tl = threadIdx.x / 3, al = threadIdx.x - 3 * (threadIdx.x / 3);
            const int64_t i = i0 + tl;
            if (i < ne) {
                const int4 nb4 = nbr[i];
                const int nb = pick(nb4, al);
                const int slot = (nb4.w >> (10 * al)) & 1023;
                Real pl[N], pr[N], y[N];
#pragma unroll
                for (int l = 0; l < N; ++l) pl[l] = sd[tl * N + rot_sel<P>(al, l)];
                int ar = 0;
                double4 er = make_double4(0, 0, 0, 0);
                if (nb >= 0) {
                    ar = nb & 3;
#pragma unroll
                    for (int l = 0; l < N; ++l) pr[l] = sd[slot * N + rot_sel<P>(ar, l)];
                    if constexpr (kCentre) centre(pr, pl[0]);
                    // (the bandwidth-bound several-tiles variant reads the neighbour's geometry
                    // through its id: the per-edge copy in geo_nb measured 3% slower here)
                    er = geo[nb >> 2];
                } else {
#pragma unroll
                    for (int l = 0; l < N; ++l) pr[l] = Real(0);
                }
                if constexpr (kCentre) centre(pl, pl[0]);
                const double4 ei = geo[i];
                edge_lane_core<P, Ops, Real>(al, *ops, ei, nb, ar, er, pl, pr, y,
                                             wall_kind(kShift, wall_i, i, al));
                if constexpr (kShift) {
                    // this lane's rows (rotation-orbit representatives, the centre on lane 0);
                    // Mref is invariant under the relabelling
                    constexpr Tab<P> TT{};
                    const double sa = -scal[S::SIGMA] * (ei.x * ei.w - ei.y * ei.z);
#pragma unroll
                    for (int q = 0; q < TT.nrep; ++q)
                        y[TT.rep[q]] = fma(sa, mass_row<P>(*ops, TT.rep[q], pl), y[TT.rep[q]]);
                    if (TT.centre >= 0 && al == 0) {
                        const int kc = TT.centre >= 0 ? TT.centre : 0;
                        y[kc] = fma(sa, mass_row<P>(*ops, kc, pl), y[kc]);
                    }
                }
#pragma unroll
                for (int k = 0; k < N; ++k) sm[(tl * 3 + al) * N + rot_sel<P>(al, k)] = y[k];
            }
        }
        __syncthreads();
        // phase 3: q_k = -K d_k (coalesced) and the dot products
        for (int f = threadIdx.x; f < nown; f += NT) {
            const int t = f / N, k = f - t * N;
            Real qk = (sm[(t * R) * N + k] + sm[(t * R + 1) * N + k]) + sm[(t * R + 2) * N + k];
            if constexpr (R == 4) qk += sm[(t * R + 3) * N + k];
            qk = -qk;
            if constexpr (kFront) __builtin_nontemporal_store(qk, &q_out[base + f]);
            else q_out[base + f] = qk;
            const double dk = sd[f], rk = sr[f], qd = qk;
            acc[1] = fma(dk, qd, acc[1]);
            acc[2] = fma(rk, qd, acc[2]);
            acc[3] = fma(qd, qd, acc[3]);
        }
        __syncthreads();
    }
    block_sum_all<4, NT>(acc);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) part_out[c * G + blockIdx.x] = acc[c];
        if (blockIdx.x == 0) scal[S::ITER0 + (1 - parity)] = it + 1.0;
    }
}

// ---------------------------------------------------------------- setup and finish
// wall_i[i] (internal order): bit al set when local edge al of the triangle is a wall edge
// flagged Dirichlet in edge_mask [nd] (caller's edge numbering; NULL: none)
__global__ __launch_bounds__(kBlockFlat) void k_wall_mask(int64_t ne, const int* __restrict__ perm,
                                                          const int4* __restrict__ nbr,
                                                          const int4* __restrict__ tedges,
                                                          const unsigned char* __restrict__ edge_mask,
                                                          unsigned char* __restrict__ wall_i) {
    const int64_t i = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x;
    if (i >= ne) return;
    const int t = perm[i];
    const int4 nb = nbr[t], te = tedges[t];
    unsigned char bits = 0;
    if (edge_mask) {
        if (nb.x < 0 && edge_mask[te.x >> 1]) bits |= 1;
        if (nb.y < 0 && edge_mask[te.y >> 1]) bits |= 2;
        if (nb.z < 0 && edge_mask[te.z >> 1]) bits |= 4;
    }
    wall_i[i] = bits;
}

// partials of sum(b)
__global__ __launch_bounds__(kBlockFlat) void k_sum_partials(const double* __restrict__ b, int64_t n,
                                                             double* __restrict__ part) {
    double acc[1] = {0.0};
    for (int64_t t = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlockFlat)
        acc[0] += b[t];
    block_sum_all<1, kBlockFlat>(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// one block: scal[idx] = scale * sum(part[0..nb))
__global__ __launch_bounds__(kBlockFlat) void k_scal_reduce(const double* __restrict__ part, int nb,
                                                            double* __restrict__ scal, int idx,
                                                            double scale) {
    const double s = reduce_partials<kBlockFlat>(part, nb);
    if (threadIdx.x == 0) scal[idx] = scale * s;
}

// b_int = b - mean in internal order (gathered through perm); x = 0 (cold) or the gathered
// initial guess (warm); e = d0 = q0 = 0; partials of |b_int|^2
__global__ __launch_bounds__(kBlockFlat) void k_cg_prep(const double* __restrict__ b,
                                                        const double* __restrict__ p0,
                                                        const int* __restrict__ perm, int nphi,
                                                        int64_t n, double* __restrict__ bint,
                                                        double* __restrict__ x, int warm,
                                                        double* __restrict__ e,
                                                        double* __restrict__ d0,
                                                        double* __restrict__ d1,
                                                        double* __restrict__ part,
                                                        const double* __restrict__ scal) {
    const double mean = scal[S::MEAN];
    double acc[1] = {0.0};
    for (int64_t t = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlockFlat) {
        const int64_t i = t / nphi;
        const int64_t src = (int64_t)perm[i] * nphi + (t - i * nphi);
        const double v = b[src] - mean;
        bint[t] = v;
        x[t] = warm ? p0[src] : 0.0;
        e[t] = 0.0;
        d0[t] = 0.0;
        d1[t] = 0.0;
        acc[0] = fma(v, v, acc[0]);
    }
    block_sum_all<1, kBlockFlat>(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// one block: BB, TOL2, ITER, DONE, MAXIT
__global__ __launch_bounds__(kBlockFlat) void k_cg_scal_init(const double* __restrict__ part, int nb,
                                                             double* __restrict__ scal, double rtol,
                                                             int maxit, double sigma) {
    const double bb = reduce_partials<kBlockFlat>(part, nb);
    if (threadIdx.x == 0) {
        scal[S::BB] = bb;
        scal[S::TOL2] = rtol * rtol * bb;
        scal[S::ITER] = 0.0;
        scal[S::ITER0] = 0.0;
        scal[S::ITER1] = 0.0;
        scal[S::MAXIT] = (double)maxit;
        scal[S::RR] = 0.0;
        scal[S::ZERO] = bb == 0.0 ? 1.0 : 0.0;
        scal[S::DONE] = bb == 0.0 ? 1.0 : 0.0;
        scal[S::SIGMA] = sigma;
        scal[S::RTH] = 0.0;
        scal[S::TOLU] = rtol * rtol * bb;
    }
}

// partials of |K x - b_int|^2 and int x (gauge), kx = K x
template <int P>
__global__ __launch_bounds__(kBlockFlat) void k_finish_partials(const RefOps<P>* __restrict__ ops,
                                                                const double4* __restrict__ geo,
                                                                int64_t ne, const double* __restrict__ kx,
                                                                const double* __restrict__ bint,
                                                                const double* __restrict__ x,
                                                                double* __restrict__ part) {
    constexpr int N = RefOps<P>::NPHI;
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x; i < ne;
         i += (int64_t)gridDim.x * kBlockFlat) {
        const double4 e = geo[i];
        const double A = e.x * e.w - e.y * e.z;
        double s = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const int64_t o = i * N + k;
            const double t = kx[o] - bint[o];
            acc[0] = fma(t, t, acc[0]);
            s = fma(ops->w[k], x[o], s);
        }
        acc[1] = fma(A, s, acc[1]);
    }
    block_sum_all<2, kBlockFlat>(acc);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc[0];
        part[gridDim.x + blockIdx.x] = acc[1];
    }
}

__global__ __launch_bounds__(kBlockFlat) void k_finish_reduce(const double* __restrict__ part, int nb,
                                                              double* __restrict__ scal) {
    const double a = reduce_partials<kBlockFlat>(part, nb);
    const double b = reduce_partials<kBlockFlat>(part + nb, nb);
    if (threadIdx.x == 0) {
        scal[S::RTRUE] = a;
        scal[S::INTX] = b;
    }
}

// p (caller order) = x (internal order) - int x / |Omega|, scattered through perm
__global__ __launch_bounds__(kBlockFlat) void k_gauge_out(int64_t n, int nphi,
                                                          const int* __restrict__ perm,
                                                          const double* __restrict__ x,
                                                          const double* __restrict__ scal,
                                                          double inv_area, double* __restrict__ out) {
    const double shift = scal[S::INTX] * inv_area;
    const bool zero = scal[S::ZERO] != 0.0;
    for (int64_t t = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlockFlat) {
        const int64_t i = t / nphi;
        out[(int64_t)perm[i] * nphi + (t - i * nphi)] = zero ? 0.0 : x[t] - shift;
    }
}

// K p in internal order (the standalone operator kernel on the internal tables)
template <int P>
__global__ __launch_bounds__(kBlockTri) void k_apply_internal(const RefOps<P>* __restrict__ ops,
                                                              const double4* __restrict__ geo,
                                                              const int4* __restrict__ nbr,
                                                              int64_t ne,
                                                              const double* __restrict__ p,
                                                              double* __restrict__ out,
                                                              double sigma,
                                                              const unsigned char* __restrict__ wall_i) {
    constexpr int N = RefOps<P>::NPHI;
    __shared__ double sm[kTriPerBlock][4][N];
    const int tl = threadIdx.x / 3, al = threadIdx.x - 3 * (threadIdx.x / 3);
    const int64_t i = (int64_t)blockIdx.x * kTriPerBlock + tl;
    const bool valid = i < ne;
    if (valid) {
        double pl[N], y[N];
        LoadPlain<N> ld{p};
        schur_edge_lane<P>(i, al, *ops, geo, nbr, ld, pl, y, wall_kind(sigma != 0.0, wall_i, i, al));
        lds_scatter<P>(&sm[tl][0][0], al, y);
    }
    __syncthreads();
    if (valid)
        for (int k = al; k < N; k += 3)
            out[i * N + k] = shifted_row<P>(*ops, geo, p, i, k,
                                            sm[tl][0][k] + sm[tl][1][k] + sm[tl][2][k], sigma);
}

// ---------------------------------------------------------------- mixed precision
// One FP32 Krylov process (the k_cg_step<float> iterations, with the correction accumulated in
// e32) refreshed by FP64 "reliable updates": x += e (float64), r := K x - b recomputed in
// float64 and rounded back to the FP32 residual, keeping the search direction.  All FP32
// quantities are scaled by s = 1/||b_int|| so the tolerance is relative and FP32 stays in range.

// one block: s from |b_int|^2 and the inner scalars
__global__ __launch_bounds__(kBlockFlat) void k_rel_init(double* __restrict__ scal,
                                                         double* __restrict__ scal_in, double rtol,
                                                         int maxit) {
    if (threadIdx.x == 0) {
        const double bb = scal[S::BB];
        scal[S::IRS] = bb > 0.0 ? 1.0 / sqrt(bb) : 0.0;
        scal_in[S::DONE] = scal[S::DONE];  // zero right-hand side: nothing to do
        scal_in[S::ITER] = 0.0;
        scal_in[S::ITER0] = 0.0;
        scal_in[S::ITER1] = 0.0;
        scal_in[S::RR] = 0.0;
        scal_in[S::TOL2] = rtol * rtol;  // relative: the scaled right-hand side has unit norm
        scal_in[S::MAXIT] = (double)maxit;
        scal_in[S::RTH] = 0.0;  // the FP32 process is refreshed by the host's reliable updates
    }
}

// r32 = s r64; partials of r32.r32 and r32.q32 into the rr / rq slots of the current state
// (dq and qq of that state are unchanged: d and q are kept), and of |s r64 - r32_old|^2 (the gap
// between the refreshed and the recursive FP32 residual) into gap_part.  init: also e = q = d = 0.
__global__ __launch_bounds__(kBlockFlat) void k_rel_to32(int64_t n, const double* __restrict__ r64,
                                                         const double* __restrict__ scal,
                                                         float* __restrict__ r32,
                                                         float* __restrict__ q32,
                                                         float* __restrict__ d32,
                                                         float* __restrict__ e, int init,
                                                         double* __restrict__ part,
                                                         double* __restrict__ gap_part) {
    const double sc = scal[S::IRS];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t t = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlockFlat) {
        const double rt = sc * r64[t];
        const float rv = (float)rt;
        const double g = rt - (double)r32[t];
        r32[t] = rv;
        if (init) {
            e[t] = 0.0f;
            q32[t] = 0.0f;
            d32[t] = 0.0f;
        }
        const double rd = rv;
        acc[0] = fma(rd, rd, acc[0]);
        acc[1] = fma(rd, (double)q32[t], acc[1]);
        acc[2] = fma(g, g, acc[2]);
    }
    block_sum_all<3, kBlockFlat>(acc);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc[0];                  // rr slot
        part[2 * gridDim.x + blockIdx.x] = acc[1];  // rq slot
        gap_part[blockIdx.x] = acc[2];
    }
}

// x += e / s (float64); e = 0
__global__ __launch_bounds__(kBlockFlat) void k_rel_accumulate(int64_t n, double* __restrict__ x,
                                                               float* __restrict__ e,
                                                               const double* __restrict__ scal) {
    const double sc = scal[S::IRS];
    const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
    for (int64_t t = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlockFlat) {
        x[t] = fma((double)e[t], inv, x[t]);
        e[t] = 0.0f;
    }
}

// restart the FP32 Krylov process (after it stopped on its own criterion)
__global__ void k_rel_restart(double* __restrict__ scal_in) {
    if (threadIdx.x == 0) {
        scal_in[S::DONE] = 0.0;
        scal_in[S::ITER] = 0.0;
        scal_in[S::ITER0] = 0.0;
        scal_in[S::ITER1] = 0.0;
    }
}

// one block: current recursive rr of the FP32 state (slot 0 of the partials) -> scal_in[RRNOW];
// optionally clear the inner DONE flag (resume after a reliable update)
__global__ __launch_bounds__(kBlockFlat) void k_rel_peek(const double* __restrict__ part, int nb,
                                                         double* __restrict__ scal_in, int resume) {
    const double rr = reduce_partials<kBlockFlat>(part, nb);
    if (threadIdx.x == 0) {
        scal_in[S::RRNOW] = rr;
        if (resume) scal_in[S::DONE] = 0.0;
    }
}

// ---------------------------------------------------------------- FP64 residual replacement
// The FP64 iteration kernel accumulates x_k - x into e, so its rounding is relative to the
// correction since the last replacement, not to x: x += e, e = 0 at each replacement.
__global__ __launch_bounds__(kBlockFlat) void k_cg_fold(int64_t n, double* __restrict__ x,
                                                        double* __restrict__ e) {
    for (int64_t t = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlockFlat) {
        x[t] += e[t];
        e[t] = 0.0;
    }
}

// The state the iteration kernel stopped on lives in the buffers of parity src; rt holds the
// recomputed residual K x - b_int (written into the free buffers of parity 1 - src).  r, d and q
// of the replaced state go to buffers 0 (the first launch of every captured block reads buffers
// 0), the partials of rr = r.r, dq = d.q, rq = r.q, qq = q.q of this state to the partial slot
// the first launch reads, and those of |rt - r_recursive|^2 to gap_part.
// (rs and r0 are the same buffer when src = 0: no __restrict__ here)
__global__ __launch_bounds__(kBlockFlat) void k_rep_state(int64_t n, const double* rt,
                                                          const double* rs, const double* qs,
                                                          const double* ds, double* r0, double* q0,
                                                          double* d0, int src,
                                                          double* __restrict__ part,
                                                          double* __restrict__ gap_part) {
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t t = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlockFlat) {
        const double r = rt[t], q = qs[t], dd = ds[t], g = r - rs[t];
        if (src == 0) {
            r0[t] = r;  // rt is buffer 1: move r; q and d are in place
        } else {
            q0[t] = q;  // rt is buffer 0 already: move q and d
            d0[t] = dd;
        }
        acc[0] = fma(r, r, acc[0]);
        acc[1] = fma(dd, q, acc[1]);
        acc[2] = fma(r, q, acc[2]);
        acc[3] = fma(q, q, acc[3]);
        acc[4] = fma(g, g, acc[4]);
    }
    block_sum_all<5, kBlockFlat>(acc);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) part[c * gridDim.x + blockIdx.x] = acc[c];
        gap_part[blockIdx.x] = acc[4];
    }
}

// one block: RR and GAP from the partials; resume the iteration from the replaced state, or
// restart it from the new residual when the gap shows the kept direction is no longer conjugate
__global__ __launch_bounds__(kBlockFlat) void k_rep_scal(const double* __restrict__ part,
                                                         const double* __restrict__ gap_part,
                                                         int nb, double* __restrict__ scal,
                                                         double factor2, double gapmax2) {
    const double rr = reduce_partials<kBlockFlat>(part, nb);
    const double gap = reduce_partials<kBlockFlat>(gap_part, nb);
    if (threadIdx.x == 0) {
        const double done_iters = scal[S::ITER];
        // stopped at rtol on the recursive residual, but the recomputed one misses the target:
        // aim the recursive residual lower
        if (scal[S::DONE] == (double)S::kConverged && rr > scal[S::TOLU])
            scal[S::TOL2] = 0.25 * scal[S::TOL2];
        scal[S::RR] = rr;
        scal[S::GAP] = gap;
        scal[S::RTH] = factor2 * rr;
        scal[S::DONE] = 0.0;
        if (gap > gapmax2 * rr) {
            // the next launch is a first launch: alpha = beta = 0, d = r
            scal[S::ITER0] = 0.0;
            scal[S::ITER1] = 0.0;
            scal[S::MAXIT] = scal[S::MAXIT] - done_iters;
        } else {
            scal[S::ITER0] = done_iters + 1.0;  // the launch that stopped, run again
            scal[S::ITER1] = done_iters;
        }
    }
}

// ---------------------------------------------------------------- pipelined CG
// Ghysels and Vanroose's pipelined CG on A = -K (or its FP64 residual-replacement form), for
// meshes whose tiles each fit one block.  With gamma_i = r_i.r_i and delta_i = w_i.r_i, w_i = A r_i:
//   q_i = A w_i
//   beta_i = gamma_i / gamma_{i-1},  alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1})
//   (first iteration: beta = 0, alpha = gamma / delta)
//   z_i = q_i + beta z_{i-1},  s_i = w_i + beta s_{i-1},  p_i = r_i + beta p_{i-1}
//   x += alpha p_i,  r_{i+1} = r_i - alpha s_i,  w_{i+1} = w_i - alpha z_i.
// In exact arithmetic the iterates are those of CG (Section 3.3).  The operator is applied to
// w_i, which the previous launch completed, so a launch evaluates it while the previous
// launch's partial sums of gamma and delta are still arriving; CG proper cannot start its
// operator before those sums give it alpha and beta.  Only w is read across tiles (the halo),
// so only w is double-buffered by parity; r, z, s, p and the correction e are updated in place.
// Scalars: alpha_i and gamma_i by parity in PA0 / PG0 (+1), like the iteration counter.

template <int P>
__global__ __launch_bounds__(kBlockCG) void k_pcg_step(const RefOps<P>* __restrict__ ops,
                                                       const double4* __restrict__ geo,
                                                       const double4* __restrict__ geo_nb,
                                                       const int4* __restrict__ nbr,
                                                       const int* __restrict__ halo_pad, int hmax,
                                                       int64_t ne, double* __restrict__ e,
                                                       double* __restrict__ r,
                                                       double* __restrict__ z,
                                                       double* __restrict__ sv,
                                                       double* __restrict__ pv,
                                                       const double* __restrict__ w_in,
                                                       double* __restrict__ w_out,
                                                       const double* __restrict__ part_in,
                                                       double* __restrict__ part_out,
                                                       double* __restrict__ scal, int parity) {
    constexpr int N = RefOps<P>::NPHI;
    constexpr int T = kTriPerBlock;
    constexpr int NT = kBlockCG;
    constexpr int PER = (T * N + NT - 1) / NT;  // tile entries per thread
    constexpr int HB = 4;                       // halo entries per thread and batch
    constexpr int PB = 4;                       // partials per thread requested at entry
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double* sw = reinterpret_cast<double*>(lds_raw);  // [(T + hmax) N]: w of the tile, then halo
    double* sm = sw + (size_t)(T + hmax) * N;          // [T][4][N]: rows of K w by role
    const int G = gridDim.x;
    const int hs = hmax > 0 ? hmax : 1;
    const int nhe = hmax * N;
    // one tile per block, by the same XCD-aware map as k_cg_step (G is a multiple of 8); the
    // blocks beyond the last tile contribute zero partials
    const int64_t tile = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
    const int64_t i0 = tile * T;
    if (i0 >= ne) {
        if (threadIdx.x == 0) {
            part_out[blockIdx.x] = 0.0;
            part_out[G + blockIdx.x] = 0.0;
        }
        return;
    }
    const int nown = (int)((ne - i0) < T ? (ne - i0) : T) * N;
    // the stop flag and the iteration count, read once for the whole block (block 0 of this
    // launch may set the flag while other blocks start)
    __shared__ double flags[2];
    if (threadIdx.x == 0) {
        flags[0] = scal[S::DONE];
        flags[1] = scal[S::ITER0 + parity];
    }
    __syncthreads();
    if (flags[0] != 0.0) return;
    const double it = flags[1];
    // entry: the tile's w and state, the halo ids, and this thread's first partials
    double vw[PER], vr[PER], vz[PER], vs[PER], vp[PER], ve[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int f = threadIdx.x + u * NT;
        if (f < nown) {
            const int64_t o = i0 * N + f;
            vw[u] = w_in[o];
            vr[u] = r[o];
            vz[u] = z[o];
            vs[u] = sv[o];
            vp[u] = pv[o];
            ve[u] = e[o];
        }
    }
    double pg[PB], pd[PB];
#pragma unroll
    for (int u = 0; u < PB; ++u) {
        const int b = threadIdx.x + u * NT;
        pg[u] = b < G ? part_in[b] : 0.0;
        pd[u] = b < G ? part_in[G + b] : 0.0;
    }
    for (int e0 = 0; e0 < nhe; e0 += HB * NT) {
        int hid[HB];
        double hw[HB];
#pragma unroll
        for (int u = 0; u < HB; ++u) {
            const int ee = e0 + threadIdx.x + u * NT;
            hid[u] = ee < nhe ? halo_pad[tile * hs + ee / N] : -1;
        }
#pragma unroll
        for (int u = 0; u < HB; ++u)
            if (hid[u] >= 0) {
                const int ee = e0 + threadIdx.x + u * NT;
                hw[u] = w_in[(int64_t)hid[u] * N + (ee - (ee / N) * N)];
            }
#pragma unroll
        for (int u = 0; u < HB; ++u)
            if (hid[u] >= 0) sw[T * N + e0 + threadIdx.x + u * NT] = hw[u];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int f = threadIdx.x + u * NT;
        if (f < nown) sw[f] = vw[u];
    }
    __syncthreads();
    // q = A w: one wave per role (waves 0..2: local edge 0..2, wave 3: volume term), one lane
    // per triangle, operands from LDS (the pressure operator: walls carry no dual coupling)
    {
        const int role = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int lane = threadIdx.x & 63;
        const int64_t i = i0 + lane;
        if (i < ne) {
            double pl[N], y[N];
#pragma unroll
            for (int l = 0; l < N; ++l) pl[l] = sw[lane * N + l];
            const double4 eg = geo[i];
            if (role == 3) {
                volume_wave_core<P, RefOps<P>, double>(*ops, eg, pl, y);
            } else {
                const int4 nb4 = nbr[i];
                const int nb = pick(nb4, role);
                const int slot = (nb4.w >> (10 * role)) & 1023;
                const double4 er = geo_nb[i * 3 + role];
                double pr[N];
                int ar = 0;
                if (nb >= 0) {
                    ar = nb & 3;
#pragma unroll
                    for (int l = 0; l < N; ++l) pr[l] = sw[slot * N + rot_sel<P>(ar, l)];
                } else {
#pragma unroll
                    for (int l = 0; l < N; ++l) pr[l] = 0.0;
                }
                if (role == 0) edge_wave_core<P, 0, RefOps<P>, double>(*ops, eg, nb, ar, er, pl, pr, y);
                else if (role == 1) edge_wave_core<P, 1, RefOps<P>, double>(*ops, eg, nb, ar, er, pl, pr, y);
                else edge_wave_core<P, 2, RefOps<P>, double>(*ops, eg, nb, ar, er, pl, pr, y);
            }
#pragma unroll
            for (int k = 0; k < N; ++k) sm[(lane * 4 + role) * N + k] = y[k];
        }
    }
    // gamma_i, delta_i: the previous launch's partials in a fixed order (the same in every block)
    double v[2] = {0.0, 0.0};
#pragma unroll
    for (int u = 0; u < PB; ++u) {
        v[0] += pg[u];
        v[1] += pd[u];
    }
    for (int b = threadIdx.x + PB * NT; b < G; b += NT) {
        v[0] += part_in[b];
        v[1] += part_in[G + b];
    }
    block_sum_all<2, NT>(v);  // (its barriers also complete the operator rows in sm)
    const double g = v[0], dl = v[1];
    int stop = 0;
    bool restart = false;
    double alpha = 0.0, beta = 0.0;
    if (!isfinite(g)) stop = S::kBreakdown;
    else if (g <= scal[S::TOL2]) stop = S::kConverged;
    else if (g <= scal[S::RTH] || it - scal[S::PLR] >= (double)kPcgSpan) stop = S::kRefresh;
    else if (it > scal[S::MAXIT]) stop = S::kMaxit;
    else if (it == 0.0) {
        if (!(dl > 0.0) || !isfinite(dl)) stop = S::kBreakdown;
        else alpha = g / dl;
    } else {
        beta = g / scal[S::PG0 + parity];
        const double den = dl - beta * g / scal[S::PA0 + parity];
        if (!isfinite(den)) {
            stop = S::kBreakdown;
        } else if (!(den > 0.0)) {
            // the recurrences of w, z and s have drifted from A r, A s and A p: a replacement
            // recomputes them, and the directions restart
            stop = S::kRefresh;
            restart = true;
        } else {
            alpha = g / den;
        }
    }
    if (stop) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            scal[S::DONE] = (double)stop;
            scal[S::RR] = g;
            scal[S::ITER] = it;  // updates that reached x
            // the scalars this state was reached with, for a replacement that keeps it
            scal[S::PA0] = scal[S::PA0 + parity];
            scal[S::PG0] = scal[S::PG0 + parity];
            if (restart) scal[S::GAP] = -1.0;  // read by k_pcg_rep_scal: restart
        }
        return;
    }
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int f = threadIdx.x + u * NT;
        if (f < nown) {
            const int t = f / N, k = f - t * N;
            double q = (sm[(t * 4) * N + k] + sm[(t * 4 + 1) * N + k]) + sm[(t * 4 + 2) * N + k];
            q += sm[(t * 4 + 3) * N + k];
            q = -q;
            const double zz = fma(beta, vz[u], q);
            const double ss = fma(beta, vs[u], vw[u]);
            const double pp = fma(beta, vp[u], vr[u]);
            const double rn = fma(-alpha, ss, vr[u]);
            const double wn = fma(-alpha, zz, vw[u]);
            const int64_t o = i0 * N + f;
            __builtin_nontemporal_store(zz, &z[o]);
            __builtin_nontemporal_store(ss, &sv[o]);
            __builtin_nontemporal_store(pp, &pv[o]);
            __builtin_nontemporal_store(fma(alpha, pp, ve[u]), &e[o]);
            __builtin_nontemporal_store(rn, &r[o]);
            __builtin_nontemporal_store(wn, &w_out[o]);
            acc[0] = fma(rn, rn, acc[0]);
            acc[1] = fma(wn, rn, acc[1]);
        }
    }
    block_sum_all<2, NT>(acc);
    if (threadIdx.x == 0) {
        part_out[blockIdx.x] = acc[0];
        part_out[G + blockIdx.x] = acc[1];
        if (blockIdx.x == 0) {
            scal[S::ITER0 + (1 - parity)] = it + 1.0;
            scal[S::PA0 + (1 - parity)] = alpha;
            scal[S::PG0 + (1 - parity)] = g;
        }
    }
}

// w = -Kr (Kr = K r given), partials of gamma = r.r and delta = w.r into part[0, G) and
// part[G, 2G); zero: also z = s = p = 0 (a first iteration follows)
__global__ __launch_bounds__(kBlockFlat) void k_pcg_dots(int64_t n, const double* __restrict__ r,
                                                         const double* __restrict__ kr,
                                                         double* __restrict__ w,
                                                         double* __restrict__ z,
                                                         double* __restrict__ sv,
                                                         double* __restrict__ pv, int zero,
                                                         double* __restrict__ part) {
    double acc[2] = {0.0, 0.0};
    for (int64_t t = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlockFlat) {
        const double rv = r[t], wv = -kr[t];
        w[t] = wv;
        if (zero) {
            z[t] = 0.0;
            sv[t] = 0.0;
            pv[t] = 0.0;
        }
        acc[0] = fma(rv, rv, acc[0]);
        acc[1] = fma(wv, rv, acc[1]);
    }
    block_sum_all<2, kBlockFlat>(acc);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc[0];
        part[gridDim.x + blockIdx.x] = acc[1];
    }
}

// out = -in
__global__ __launch_bounds__(kBlockFlat) void k_pcg_neg(int64_t n, const double* __restrict__ in,
                                                        double* __restrict__ out) {
    for (int64_t t = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlockFlat)
        out[t] = -in[t];
}

// replacement: r = rt (the recomputed residual), partials of |rt - r|^2 into gap_part
__global__ __launch_bounds__(kBlockFlat) void k_pcg_gap(int64_t n, const double* __restrict__ rt,
                                                        double* __restrict__ r,
                                                        double* __restrict__ gap_part) {
    double acc[1] = {0.0};
    for (int64_t t = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlockFlat) {
        const double v = rt[t], g = v - r[t];
        r[t] = v;
        acc[0] = fma(g, g, acc[0]);
    }
    block_sum_all<1, kBlockFlat>(acc);
    if (threadIdx.x == 0) gap_part[blockIdx.x] = acc[0];
}

// scalars after a replacement (one block): as k_rep_scal, but a restart also clears the
// directions (k_pcg_restart_dirs reads the decision from ITER0 / ITER1)
__global__ __launch_bounds__(kBlockFlat) void k_pcg_rep_scal(const double* __restrict__ part,
                                                             const double* __restrict__ gap_part,
                                                             int nb, double* __restrict__ scal,
                                                             double factor2, double gapmax2) {
    const double rr = reduce_partials<kBlockFlat>(part, nb);
    const double gap = reduce_partials<kBlockFlat>(gap_part, nb);
    if (threadIdx.x == 0) {
        const double done_iters = scal[S::ITER];
        const bool force = scal[S::GAP] < 0.0;  // the iteration asked for a restart
        if (scal[S::DONE] == (double)S::kConverged && rr > scal[S::TOLU])
            scal[S::TOL2] = 0.25 * scal[S::TOL2];
        scal[S::RR] = rr;
        scal[S::GAP] = gap;
        scal[S::RTH] = factor2 * rr;
        scal[S::DONE] = 0.0;
        if (force || gap > gapmax2 * rr) {
            scal[S::ITER0] = 0.0;  // a first iteration: beta = 0, z = s = p = 0
            scal[S::ITER1] = 0.0;
            scal[S::PLR] = 0.0;
            scal[S::MAXIT] = scal[S::MAXIT] - done_iters;
        } else {
            scal[S::ITER0] = done_iters;  // the launch that stopped, run again
            scal[S::ITER1] = done_iters;
            scal[S::PLR] = done_iters;
        }
    }
}

__global__ void k_pcg_scal_init(double* __restrict__ scal) {
    if (threadIdx.x == 0) {
        scal[S::PLR] = 0.0;
        scal[S::GAP] = 0.0;
    }
}

__global__ __launch_bounds__(kBlockFlat) void k_pcg_restart_dirs(int64_t n,
                                                                 const double* __restrict__ scal,
                                                                 double* __restrict__ z,
                                                                 double* __restrict__ sv,
                                                                 double* __restrict__ pv) {
    if (scal[S::ITER0] != 0.0 || scal[S::ITER] == 0.0) return;
    for (int64_t t = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlockFlat) {
        z[t] = 0.0;
        sv[t] = 0.0;
        pv[t] = 0.0;
    }
}

// ---------------------------------------------------------------- static CG workspace
// The workspace of sld_cg_solve_static, for callers that cannot allocate device memory: one
// array per device, held from the library's first use on that device until the process ends.
// In host code `scratch` names a host-side stand-in: only the address that hipGetSymbolAddress
// returns for the current device may be passed to kernels or copies.
static __device__ __align__(256) double scratch[kStaticCgDoubles];

}  // namespace

hipError_t cg_static_scratch(int device, double** out) {
    static std::mutex mu;
    static double* ptr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (ptr[device] == nullptr) {
        // the caller has made `device` current
        void* a = nullptr;
        hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[device] = static_cast<double*>(a);
    }
    *out = ptr[device];
    return hipSuccess;
}

namespace {

template <int P>
const RefOps<P>* ops_of(const sld_disc_s* d) { return reinterpret_cast<const RefOps<P>*>(d->ops_dev); }
template <int P>
const RefOps32<P>* ops32_of(const sld_disc_s* d) {
    return reinterpret_cast<const RefOps32<P>*>(d->ops32_dev);
}

#define SLD_DISPATCH(p, CALL)                                   \
    switch (p) {                                                \
        case 1: { constexpr int PP = 1; CALL; } break;          \
        case 2: { constexpr int PP = 2; CALL; } break;          \
        case 3: { constexpr int PP = 3; CALL; } break;          \
        case 4: { constexpr int PP = 4; CALL; } break;          \
        default: return hipErrorInvalidValue;                   \
    }

}  // namespace

hipError_t launch_cg_setup(const sld_disc_s* d, const double* b, const double* p0, bool warm,
                           double rtol, int maxit, double sigma, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    const int64_t n = m->ne * d->nphi;
    const int G = w.grid;
    hipLaunchKernelGGL(k_sum_partials, dim3(G), dim3(kBlockFlat), 0, s, b, n, w.part_s);
    // the shifted (viscous) system is nonsingular: no projection onto 1^perp
    hipLaunchKernelGGL(k_scal_reduce, dim3(1), dim3(kBlockFlat), 0, s, w.part_s, G, w.scal,
                       (int)S::MEAN, sigma > 0.0 ? 0.0 : 1.0 / (double)n);
    hipLaunchKernelGGL(k_cg_prep, dim3(G), dim3(kBlockFlat), 0, s, b, p0, m->perm, d->nphi, n, w.b,
                       w.x, warm ? 1 : 0, w.e, w.d[0], w.q[0], w.part_s, w.scal);
    hipLaunchKernelGGL(k_cg_scal_init, dim3(1), dim3(kBlockFlat), 0, s, w.part_s, G, w.scal, rtol,
                       maxit, sigma);
    // r_0 = K x - b_int (the residual of -K x = -b_int); q, d of "iteration -1" are zero
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_cg_resid<PP>, dim3(G), dim3(kBlockTri), 0, s,
                                          ops_of<PP>(d), m->geo_i, m->nbr_i, m->ne, w.x, w.b,
                                          w.r[0], w.part_s, w.scal, sigma, w.wall_i, 0));
    // first residual replacement once |r| has dropped by kReplaceFactor from |r_0|
    hipLaunchKernelGGL(k_scal_reduce, dim3(1), dim3(kBlockFlat), 0, s, w.part_s, G, w.scal,
                       (int)S::RTH, kReplaceFactor * kReplaceFactor);
    return hipGetLastError();
}

hipError_t launch_cg_fold(const sld_disc_s* d, hipStream_t s) {
    const CgWork& w = d->cg;
    hipLaunchKernelGGL(k_cg_fold, dim3(w.grid), dim3(kBlockFlat), 0, s, d->mesh->ne * d->nphi, w.x,
                       w.e);
    return hipGetLastError();
}

hipError_t launch_cg_replace(const sld_disc_s* d, int src, double sigma, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    const int G = w.grid;
    const int64_t n = m->ne * d->nphi;
    if (src != 0 && src != 1) return hipErrorInvalidValue;
    const int fr = 1 - src;  // the buffers of the state before: free
    hipLaunchKernelGGL(k_cg_fold, dim3(G), dim3(kBlockFlat), 0, s, n, w.x, w.e);
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_cg_resid<PP>, dim3(G), dim3(kBlockTri), 0, s,
                                          ops_of<PP>(d), m->geo_i, m->nbr_i, m->ne, w.x, w.b,
                                          w.r[fr], w.part_s, w.scal, sigma, w.wall_i, 1));
    hipLaunchKernelGGL(k_rep_state, dim3(G), dim3(kBlockFlat), 0, s, n, w.r[fr], w.r[src],
                       w.q[src], w.d[src], w.r[0], w.q[0], w.d[0], src, w.part, w.part_s);
    hipLaunchKernelGGL(k_rep_scal, dim3(1), dim3(kBlockFlat), 0, s, w.part, w.part_s, G, w.scal,
                       kReplaceFactor * kReplaceFactor, kGapRestart * kGapRestart);
    return hipGetLastError();
}

// Stream x (non-temporal) when the CG working set -- five vectors and the geometry -- exceeds
// half of the 256 MB memory-side cache: measured 6% faster on 512x512x2, p = 3 (240 MB), and
// 12% slower on 256x256x2, p = 4 (85 MB, cache-resident), where it pays to keep x cached.
inline int stream_x_for(const sld_disc_s* d, size_t word) {
    if (d->cg.stream_x >= 0) return d->cg.stream_x;
    const int64_t ne = d->mesh->ne;
    return (int64_t)5 * ne * d->nphi * (int64_t)word + ne * 48 > (int64_t(128) << 20) ? 1 : 0;
}

hipError_t launch_cg_step(const sld_disc_s* d, int parity, bool shift, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    const int G = w.grid;
    const int o = 1 - parity;
    if (G & 7) return hipErrorInvalidValue;  // the tile-chunk map needs a multiple of 8
    const bool front = w.front && (int64_t)G * kTriPerBlock >= m->ne;
    const bool sx = stream_x_for(d, sizeof(double)) != 0;
    if (!shift && w.use_pcg) return launch_pcg_step(d, parity, s);
    if (!shift && w.use_mx) return launch_cg_step_mx(d, parity, false, sx, s);
    const size_t lds = step_lds_bytes(d->nphi, m->hmax, sizeof(double), front);
#define SLD_STEP64(F, SH, ST)                                                                   \
    SLD_DISPATCH(d->p, hipLaunchKernelGGL((k_cg_step<PP, double, RefOps<PP>, F, SH, ST>), dim3(G), \
                                          dim3(F ? kBlockCG : kBlockTri), lds, s, ops_of<PP>(d), \
                                          m->geo_i, m->geo_nb,                                  \
                                          m->nbr_i, m->halo_pad, m->hmax, m->ne, w.wall_i, w.e, \
                                          w.r[parity], w.q[parity], w.d[parity], w.r[o],        \
                                          w.q[o], w.d[o], w.part + parity * 4 * G,              \
                                          w.part + o * 4 * G, w.scal, parity))
    if (front) {
        if (shift) {
            SLD_STEP64(true, true, false);
        } else {
            SLD_STEP64(true, false, false);
        }
    } else if (sx) {
        if (shift) {
            SLD_STEP64(false, true, true);
        } else {
            SLD_STEP64(false, false, true);
        }
    } else {
        if (shift) {
            SLD_STEP64(false, true, false);
        } else {
            SLD_STEP64(false, false, false);
        }
    }
#undef SLD_STEP64
    return hipGetLastError();
}

// Grid of the CG iteration kernel.  Meshes whose tiles all fit on the device at once run the
// one-tile-per-block (front-loaded, four-role) variant; larger meshes run as many blocks as the
// device keeps resident (occupancy calculator, for this degree's kernel and LDS size), each
// owning a chunk of tiles.  The grid is a multiple of 8 for the per-XCD tile-chunk map.
int cg_grid_for(const sld_disc_s* d, bool* front) {
    const sld_mesh_s* m = d->mesh;
    const int64_t tiles = (m->ne + kTriPerBlock - 1) / kTriPerBlock;
    int per_front = 0, per_lanes = 0, cus = 0;
    hipError_t e = hipSuccess;
    const size_t lds_f = step_lds_bytes(d->nphi, m->hmax, sizeof(double), true);
    const size_t lds_l = step_lds_bytes(d->nphi, m->hmax, sizeof(double), false);
    SLD_DISPATCH(d->p, e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                           &per_front, (k_cg_step<PP, double, RefOps<PP>, true, false, false>), kBlockCG,
                           lds_f));
    if (e == hipSuccess)
        SLD_DISPATCH(d->p, e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                               &per_lanes, (k_cg_step<PP, double, RefOps<PP>, false, false, false>), kBlockTri,
                               lds_l));
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device);
    const bool ok = e == hipSuccess && cus > 0;
    const int64_t res_front = ok ? (int64_t)per_front * cus : 0;
    const int64_t res_lanes = ok && per_lanes > 0 ? (int64_t)per_lanes * cus : 1024;
    int64_t g;
    if (tiles <= res_front) {
        *front = true;
        g = tiles;
    } else {
        *front = false;
        g = tiles < res_lanes ? tiles : res_lanes;
        if (g > kCgMaxGrid) g = kCgMaxGrid;
    }
    return (int)((g + 7) & ~int64_t(7));
}

// Grid of the FP32 three-lane iteration.  It holds fewer registers than the FP64 kernel, so
// more of its blocks stay resident; when its working set is well beyond the cache-resident
// range (above 64 MiB: five vectors and the geometry) the grid is all of them.  Measured per
// FP32 iteration, p = 3: 512x512x2 (130 MB) 74.6 us at the FP64 grid of 1024 blocks, 72.1 us
// at 1536, 79.4 us at 2048; 256x256x2 (33 MB) 26.0 us at 1024, 27.3 us at 1536.  The
// one-tile-per-block variant keeps the FP64 grid.
int cg_grid32_for(const sld_disc_s* d, int grid, bool front) {
    const sld_mesh_s* m = d->mesh;
    if (front) return grid;
    if ((int64_t)5 * m->ne * d->nphi * 4 + m->ne * 48 <= (int64_t(64) << 20)) return grid;
    const int64_t tiles = (m->ne + kTriPerBlock - 1) / kTriPerBlock;
    int per = 0, cus = 0;
    const size_t lds = step_lds_bytes(d->nphi, m->hmax, sizeof(float), false);
    hipError_t e = hipSuccess;
    SLD_DISPATCH(d->p, e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                           &per, (k_cg_step<PP, float, RefOps32<PP>, false, false, false>), kBlockTri,
                           lds));
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device);
    if (e != hipSuccess || per <= 0 || cus <= 0) return grid;
    int64_t g = std::min<int64_t>(tiles, (int64_t)per * cus);
    g = std::min<int64_t>(g, kCgMaxGrid);
    g = (g + 7) & ~int64_t(7);
    return g > grid ? (int)g : grid;
}

hipError_t launch_wall_mask(const sld_disc_s* d, const unsigned char* edge_mask, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    hipLaunchKernelGGL(k_wall_mask, dim3((unsigned)((m->ne + kBlockFlat - 1) / kBlockFlat)),
                       dim3(kBlockFlat), 0, s, m->ne, m->perm, m->nbr, m->tedges, edge_mask,
                       d->cg.wall_i);
    return hipGetLastError();
}

hipError_t launch_cg_finish(const sld_disc_s* d, double* p_out, double sigma, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    const int G = w.grid;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_apply_internal<PP>,
                                          dim3((unsigned)((m->ne + kTriPerBlock - 1) / kTriPerBlock)),
                                          dim3(kBlockTri), 0, s, ops_of<PP>(d), m->geo_i, m->nbr_i,
                                          m->ne, w.x, w.q[0], sigma, w.wall_i));
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_finish_partials<PP>, dim3(G), dim3(kBlockFlat), 0, s,
                                          ops_of<PP>(d), m->geo_i, m->ne, w.q[0], w.b, w.x,
                                          w.part_s));
    hipLaunchKernelGGL(k_finish_reduce, dim3(1), dim3(kBlockFlat), 0, s, w.part_s, G, w.scal);
    const int64_t n = m->ne * d->nphi;
    // the gauge int p = 0 fixes the pressure's constant; the viscous solution has none to fix
    hipLaunchKernelGGL(k_gauge_out, dim3(G), dim3(kBlockFlat), 0, s, n, d->nphi, m->perm, w.x,
                       w.scal, sigma > 0.0 ? 0.0 : 1.0 / m->area_total, p_out);
    return hipGetLastError();
}

hipError_t launch_cg_step32(const sld_disc_s* d, int parity, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    const int G = rel_grid(w);
    const int o = 1 - parity;
    if (G & 7) return hipErrorInvalidValue;  // the tile-chunk map needs a multiple of 8
    const bool front = w.front && (int64_t)G * kTriPerBlock >= m->ne;
    const size_t lds = step_lds_bytes(d->nphi, m->hmax, sizeof(float), front);
    const bool sx = stream_x_for(d, sizeof(float)) != 0;
    if (w.use_mx) return launch_cg_step_mx(d, parity, true, sx, s);
#define SLD_STEP32(F, ST)                                                                       \
    SLD_DISPATCH(d->p, hipLaunchKernelGGL((k_cg_step<PP, float, RefOps32<PP>, F, false, ST>), dim3(G), \
                                          dim3(F ? kBlockCG : kBlockTri), lds, s, ops32_of<PP>(d), \
                                          m->geo_i, m->geo_nb,                                  \
                                          m->nbr_i, m->halo_pad, m->hmax, m->ne, w.wall_i, w.e32, \
                                          w.r32[parity], w.q32[parity], w.d32[parity],          \
                                          w.r32[o], w.q32[o], w.d32[o],                         \
                                          w.part32 + parity * 4 * G, w.part32 + o * 4 * G,      \
                                          w.scal_in, parity))
    if (front) {
        SLD_STEP32(true, false);
    } else if (sx) {
        SLD_STEP32(false, true);
    } else {
        SLD_STEP32(false, false);
    }
#undef SLD_STEP32
    return hipGetLastError();
}

// mixed-precision setup: the FP64 setup left r64 = K x - b_int in w.r[0]
hipError_t launch_rel_init(const sld_disc_s* d, double rtol, int maxit, hipStream_t s) {
    const CgWork& w = d->cg;
    const int64_t n = d->mesh->ne * d->nphi;
    hipLaunchKernelGGL(k_rel_init, dim3(1), dim3(kBlockFlat), 0, s, w.scal, w.scal_in, rtol, maxit);
    hipLaunchKernelGGL(k_rel_to32, dim3(rel_grid(w)), dim3(kBlockFlat), 0, s, n, w.r[0], w.scal, w.r32[0],
                       w.q32[0], w.d32[0], w.e32, 1, w.part32, w.part_s);
    return hipGetLastError();
}

// reliable update on the current state (buffers 0 after an even number of iterations):
// x += e; r64 = K x - b_int (float64, |r64|^2 -> scal[RR]); r32 = s r64, keeping d and q;
// |s r64 - r32_recursive|^2 -> scal_in[GAP]
hipError_t launch_rel_update(const sld_disc_s* d, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    const int64_t n = m->ne * d->nphi;
    hipLaunchKernelGGL(k_rel_accumulate, dim3(w.grid), dim3(kBlockFlat), 0, s, n, w.x, w.e32, w.scal);
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_cg_resid<PP>, dim3(w.grid), dim3(kBlockTri), 0, s,
                                          ops_of<PP>(d), m->geo_i, m->nbr_i, m->ne, w.x, w.b,
                                          w.r[0], w.part_s, w.scal, 0.0, w.wall_i, 0));
    hipLaunchKernelGGL(k_scal_reduce, dim3(1), dim3(kBlockFlat), 0, s, w.part_s, w.grid, w.scal,
                       (int)S::RR, 1.0);
    hipLaunchKernelGGL(k_rel_to32, dim3(rel_grid(w)), dim3(kBlockFlat), 0, s, n, w.r[0], w.scal, w.r32[0],
                       w.q32[0], w.d32[0], w.e32, 0, w.part32, w.part_s);
    hipLaunchKernelGGL(k_scal_reduce, dim3(1), dim3(kBlockFlat), 0, s, w.part_s, rel_grid(w), w.scal_in,
                       (int)S::GAP, 1.0);
    return hipGetLastError();
}

// restart the FP32 Krylov process from the refreshed residual: d = q = 0 (the next iteration
// takes d = r), iteration counters and the stop flag cleared
hipError_t launch_rel_restart(const sld_disc_s* d, hipStream_t s) {
    const CgWork& w = d->cg;
    const int64_t n = d->mesh->ne * d->nphi;
    hipLaunchKernelGGL(k_rel_to32, dim3(rel_grid(w)), dim3(kBlockFlat), 0, s, n, w.r[0], w.scal, w.r32[0],
                       w.q32[0], w.d32[0], w.e32, 1, w.part32, w.part_s);
    hipLaunchKernelGGL(k_rel_restart, dim3(1), dim3(64), 0, s, w.scal_in);
    return hipGetLastError();
}

hipError_t launch_rel_peek(const sld_disc_s* d, int resume, hipStream_t s) {
    const CgWork& w = d->cg;
    hipLaunchKernelGGL(k_rel_peek, dim3(1), dim3(kBlockFlat), 0, s, w.part32, rel_grid(w), w.scal_in,
                       resume);
    return hipGetLastError();
}

// ---------------------------------------------------------------- pipelined CG launchers
// Buffers: r = r[0], z = q[0], s = q[1], p = r[1], w = d[parity] (read) / d[1 - parity]
// (written), the correction e; d[1] is scratch during the setup and a replacement.

bool pcg_possible(const sld_disc_s* d) {
    const CgWork& w = d->cg;
    return w.front && w.grid > 0 && (int64_t)w.grid * kTriPerBlock >= d->mesh->ne;
}

namespace {
// out = K v (internal order; the pressure operator)
hipError_t apply_k(const sld_disc_s* d, const double* v, double* out, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_apply_internal<PP>,
                                          dim3((unsigned)((m->ne + kTriPerBlock - 1) / kTriPerBlock)),
                                          dim3(kBlockTri), 0, s, ops_of<PP>(d), m->geo_i, m->nbr_i,
                                          m->ne, v, out, 0.0, d->cg.wall_i));
    return hipGetLastError();
}
}  // namespace

hipError_t launch_pcg_step(const sld_disc_s* d, int parity, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    const int G = w.grid;
    if (!pcg_possible(d) || (G & 7)) return hipErrorInvalidValue;
    const int o = 1 - parity;
    const size_t lds = sizeof(double) * (size_t)d->nphi *
                       (size_t)(kTriPerBlock + m->hmax + 4 * kTriPerBlock);
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_pcg_step<PP>, dim3(G), dim3(kBlockCG), lds, s,
                                          ops_of<PP>(d), m->geo_i, m->geo_nb, m->nbr_i,
                                          m->halo_pad, m->hmax, m->ne, w.e, w.r[0], w.q[0],
                                          w.q[1], w.r[1], w.d[parity], w.d[o],
                                          w.part + parity * 4 * G, w.part + o * 4 * G, w.scal,
                                          parity));
    return hipGetLastError();
}

// after launch_cg_setup (r_0 = K x - b_int in r[0]): w_0 = A r_0, z = s = p = 0, the partials of
// gamma_0 and delta_0 where the first launch (parity 0) reads them
hipError_t launch_pcg_init(const sld_disc_s* d, hipStream_t s) {
    const CgWork& w = d->cg;
    const int64_t n = d->mesh->ne * d->nphi;
    hipError_t e = apply_k(d, w.r[0], w.d[1], s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pcg_dots, dim3(w.grid), dim3(kBlockFlat), 0, s, n, w.r[0], w.d[1], w.d[0],
                       w.q[0], w.q[1], w.r[1], 1, w.part);
    // first replacement once |r| has dropped by kPcgReplaceFactor (the setup left the partials of
    // |r_0|^2 in part_s)
    hipLaunchKernelGGL(k_scal_reduce, dim3(1), dim3(kBlockFlat), 0, s, w.part_s, w.grid, w.scal,
                       (int)S::RTH, kPcgReplaceFactor * kPcgReplaceFactor);
    hipLaunchKernelGGL(k_pcg_scal_init, dim3(1), dim3(64), 0, s, w.scal);
    return hipGetLastError();
}

// Residual replacement: x += e, e = 0; r = K x - b_int recomputed (|r - r_recursive|^2 -> GAP);
// w = A r, s = A p, z = A s recomputed so that the recurrences hold again; gamma, delta summed;
// the scalars as after a classic replacement, a restart also clearing z, s and p
hipError_t launch_pcg_replace(const sld_disc_s* d, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    const int G = w.grid;
    const int64_t n = m->ne * d->nphi;
    double* tmp = w.d[1];
    hipLaunchKernelGGL(k_cg_fold, dim3(G), dim3(kBlockFlat), 0, s, n, w.x, w.e);
    SLD_DISPATCH(d->p, hipLaunchKernelGGL(k_cg_resid<PP>, dim3(G), dim3(kBlockTri), 0, s,
                                          ops_of<PP>(d), m->geo_i, m->nbr_i, m->ne, w.x, w.b, tmp,
                                          w.part_s, w.scal, 0.0, w.wall_i, 1));
    hipLaunchKernelGGL(k_pcg_gap, dim3(G), dim3(kBlockFlat), 0, s, n, tmp, w.r[0], w.part_s + G);
    hipError_t e = apply_k(d, w.r[1], tmp, s);  // K p
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pcg_neg, dim3(G), dim3(kBlockFlat), 0, s, n, tmp, w.q[1]);
    e = apply_k(d, w.q[1], tmp, s);  // K s
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pcg_neg, dim3(G), dim3(kBlockFlat), 0, s, n, tmp, w.q[0]);
    e = apply_k(d, w.r[0], tmp, s);  // K r
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pcg_dots, dim3(G), dim3(kBlockFlat), 0, s, n, w.r[0], tmp, w.d[0], w.q[0],
                       w.q[1], w.r[1], 0, w.part);
    hipLaunchKernelGGL(k_pcg_rep_scal, dim3(1), dim3(kBlockFlat), 0, s, w.part, w.part_s + G, G,
                       w.scal, kPcgReplaceFactor * kPcgReplaceFactor, kGapRestart * kGapRestart);
    hipLaunchKernelGGL(k_pcg_restart_dirs, dim3(G), dim3(kBlockFlat), 0, s, n, w.scal, w.q[0],
                       w.q[1], w.r[1]);
    return hipGetLastError();
}
