// The pressure operator K (eq. pressure_final) with its reference contractions on the matrix
// cores, tile by tile: the standalone apply and the CG iteration for meshes without wall edges.
//
// Per tile of 64 triangles (a contiguous range of the internal Morton order) and its halo (the
// out-of-tile neighbours), one block of four waves:
//   G1  (all waves)   the reference derivatives of d at every edge node of every tile and halo
//                     triangle: E1 * d, one 16-triangle column block per wave and turn;
//   edge nodes        (waves 0..2: local edge alpha = wave, one lane per triangle) the closed
//                     form of Mhat_j^{-1} on the edge's nodes from both sides' derivatives and
//                     the jump, giving the normal flux and the sub-triangle correction
//                     (z of mx.h; the same algebra as the VALU operator core);
//   G2  (all waves)   (K d)_t = W2 * z_t, the volume term's inputs -A m_de d formed on the fly;
//                     wave w owns tile triangles 16 w .. 16 w + 15 and holds their rows in its
//                     output registers.
// The geometry enters only in the pointwise work (Section 3.4.1: operators = reference matrices
// x geometry), so no per-element matrix is formed or stored.
#include <cstring>
#include <mutex>

#include "device_common.h"
#include "mx.h"

using namespace sld_dev;

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kMxThreads = 256;
constexpr int T = kTriPerBlock;  // 64 triangles per tile = 4 column blocks of 16

// main index of node m (0..P) of local edge al (runtime al; see edge_node)
template <int P>
__device__ __forceinline__ int edge_node_rt(int al, int m) {
    const int a = al == 0 ? m : (al == 1 ? P - m : 0);
    const int b = al == 0 ? 0 : (al == 1 ? m : P - m);
    return b * (P + 1) - (b * (b - 1)) / 2 + a;
}

__device__ __forceinline__ void split3(float x, __bf16& h, __bf16& m, __bf16& l) {
    h = (__bf16)x;
    const float r = x - (float)h;   // exact: x and h agree in their leading 8 bits
    m = (__bf16)r;
    l = (__bf16)(r - (float)m);
}

__device__ __forceinline__ bf8v load_bf8(const uint16_t* p) {
    const uint4 u = *reinterpret_cast<const uint4*>(p);
    return __builtin_bit_cast(bf8v, u);
}

// Output row of element j of a lane in lane group g (16 x 16 blocks): the FP64 instruction
// places row i at element i / 4 of lane group i % 4, the BF16 one at element i % 4 of lane
// group i / 4 (both measured on gfx950 with one-hot operands).
template <typename Real>
__device__ __forceinline__ int out_row(int g, int j) { return sizeof(Real) == 8 ? 4 * j + g : 4 * g + j; }

// A operands held in registers by one lane for the whole launch
template <int P, typename Real>
struct MxFrag;

template <int P>
struct MxFrag<P, double> {
    using D = MxDims<P>;
    double a1[2][D::KS1];
    double a2[D::KS2];
    __device__ __forceinline__ void load(const MxTab<P>* __restrict__ tab, int lane) {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int ks = 0; ks < D::KS1; ++ks) a1[rb][ks] = tab->a1[rb][ks][lane];
#pragma unroll
        for (int ks = 0; ks < D::KS2; ++ks) a2[ks] = tab->a2[ks][lane];
    }
};

template <int P>
struct MxFrag<P, float> {
    using D = MxDims<P>;
    bf8v a1[2][3];
    bf8v a2[D::KS232][3];
    __device__ __forceinline__ void load(const MxTab<P>* __restrict__ tab, int lane) {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int s = 0; s < 3; ++s) a1[rb][s] = load_bf8(&tab->b1[rb][s][lane][0]);
#pragma unroll
        for (int ks = 0; ks < D::KS232; ++ks)
#pragma unroll
            for (int s = 0; s < 3; ++s) a2[ks][s] = load_bf8(&tab->b2[ks][s][lane][0]);
    }
};

// six split products of one BF3 k-step: small terms into `lo`, hi * hi into `hi`
__device__ __forceinline__ void bf3_mma(const bf8v (&a)[3], const float (&bv)[8], f4v& hi, f4v& lo) {
    bf8v bh, bm, bl;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        __bf16 h, m, l;
        split3(bv[e], h, m, l);
        bh[e] = h;
        bm[e] = m;
        bl[e] = l;
    }
    lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], bh, lo, 0, 0, 0);
    lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], bm, lo, 0, 0, 0);
    lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bl, lo, 0, 0, 0);
    lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], bh, lo, 0, 0, 0);
    lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bm, lo, 0, 0, 0);
    hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bh, hi, 0, 0, 0);
}

// LDS of one block, in words of Real: sd [(T + hmax) N] directions of the tile then its halo;
// sr [T N] residuals (CG only); se [(T + hmax) R1] edge-node derivatives; sz [T KE] the edge
// part of z.
template <int P>
inline size_t mx_lds_words(int hmax) {
    using D = MxDims<P>;
    return (size_t)(T + hmax) * D::N + (size_t)T * D::N + (size_t)(T + hmax) * D::R1 + (size_t)T * D::KE;
}

// The operator on one tile whose directions (tile then halo, zero where padded) are in sd:
// returns in y four rows of (K d)_t for t = 16 wave + (lane & 15), g = lane / 16.
// (y[j] is row out_row<Real>(g, j).)  The caller separates the next tile's LDS writes from G2's
// reads with a barrier.  Requires every edge to have a neighbour (no walls).
template <int P, typename Real, class Ops>
__device__ __forceinline__ void mx_tile_op(const Ops& R, const MxFrag<P, Real>& F,
                                           const double4* __restrict__ geo,
                                           const int4* __restrict__ nbr,
                                           const int* __restrict__ halo_row, int hmax, int64_t i0,
                                           int64_t ne, const Real* sd, Real* se, Real* sz,
                                           Real (&y)[4]) {
    using D = MxDims<P>;
    constexpr int N = D::N, NE = D::NE, R1 = D::R1, KE = D::KE;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
    const int nslots = T + hmax;
    const int ncb = (nslots + 15) >> 4;
    // ---- G1: edge-node derivatives of every tile and halo triangle
    for (int cb = wave; cb < ncb; cb += 4) {
        const int s0 = cb * 16;
        // halo lists are sorted with the padding last: a column block of padding ends the work
        if (s0 >= T && halo_row[s0 - T] < 0) break;
        const int slot = s0 + li;
        const bool sv = slot < nslots;
        if constexpr (sizeof(Real) == 8) {
            d4v acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < D::KS1; ++ks) {
                const int l = 4 * ks + g;
                const double b = (sv && l < N) ? (double)sd[slot * N + l] : 0.0;
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(F.a1[0][ks], b, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(F.a1[1][ks], b, acc1, 0, 0, 0);
            }
            if (sv) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r0 = out_row<double>(g, j), r1 = 16 + r0;
                    if (r0 < R1) se[slot * R1 + r0] = (Real)acc0[j];
                    if (r1 < R1) se[slot * R1 + r1] = (Real)acc1[j];
                }
            }
        } else {
            float bv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int l = 8 * g + e;
                bv[e] = (sv && l < N) ? (float)sd[slot * N + l] : 0.0f;
            }
            f4v h0 = {0, 0, 0, 0}, l0 = {0, 0, 0, 0}, h1 = {0, 0, 0, 0}, l1 = {0, 0, 0, 0};
            bf3_mma(F.a1[0], bv, h0, l0);
            bf3_mma(F.a1[1], bv, h1, l1);
            if (sv) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r0 = out_row<float>(g, j), r1 = 16 + r0;
                    if (r0 < R1) se[slot * R1 + r0] = (Real)(h0[j] + l0[j]);
                    if (r1 < R1) se[slot * R1 + r1] = (Real)(h1[j] + l1[j]);
                }
            }
        }
    }
    __syncthreads();
    // ---- edge nodes: wave al < 3 takes local edge al of tile triangle `lane`
    if (wave < 3) {
        const int al = wave;
        const int t = lane;
        const int64_t i = i0 + t;
        if (i < ne) {
            const int4 nb4 = nbr[i];
            const int nb = pick(nb4, al);
            const double4 e = geo[i];
            Real* z = sz + t * KE + al * 3 * NE;
            if (nb < 0) {
                // (not reached: the host runs this operator on meshes without wall edges)
#pragma unroll
                for (int m = 0; m < 3 * NE; ++m) z[m] = Real(0);
            } else {
                const int slot = (nb4.w >> (10 * al)) & 1023;
                const int ar = nb & 3;
                const double4 er = geo[nb >> 2];
                const Geo gd = make_geo(e.x, e.y, e.z, e.w);
                const GeoR<Real> gg(gd);
                const Geo grd = make_geo(er.x, er.y, er.z, er.w);
                const GeoR<Real> gr(grd);
                const Real wsum = (Real)(1.0 / (gd.A + grd.A));
                // |Gamma| n, outward: the edge vector v_{al+1} - v_al turned clockwise
                const double ex = al == 0 ? e.x : (al == 1 ? e.z - e.x : -e.z);
                const double ey = al == 0 ? e.y : (al == 1 ? e.w - e.y : -e.w);
                const Real snx = (Real)ey, sny = (Real)(-ex);
                Real delta[NE];
#pragma unroll
                for (int m = 0; m < NE; ++m)
                    delta[m] = sd[slot * N + edge_node_rt<P>(ar, P - m)] - sd[t * N + edge_node_rt<P>(al, m)];
                const Real* dso = se + t * R1 + al * 2 * NE;
                const Real* dsn = se + slot * R1 + ar * 2 * NE;
#pragma unroll
                for (int m = 0; m < NE; ++m) {
                    const Real ds0 = dso[m], ds1 = dso[NE + m];
                    const Real dn0 = dsn[P - m], dn1 = dsn[NE + P - m];
                    const Real gsx = gg.G00 * ds0 + gg.G10 * ds1, gsy = gg.G01 * ds0 + gg.G11 * ds1;
                    const Real gnx = gr.G00 * dn0 + gr.G10 * dn1, gny = gr.G01 * dn0 + gr.G11 * dn1;
                    Real cd = 0;
#pragma unroll
                    for (int q = 0; q < NE; ++q) cd = mad((Real)R.C[m][q], delta[q], cd);
                    const Real hx = (gg.A * gsx + gr.A * gnx + Real(3) * snx * cd) * wsum;
                    const Real hy = (gg.A * gsy + gr.A * gny + Real(3) * sny * cd) * wsum;
                    const Real dx = hx - gsx, dy = hy - gsy;
                    z[m] = snx * hx + sny * hy;
                    z[NE + m] = -gg.A * (gg.G00 * dx + gg.G01 * dy);
                    z[2 * NE + m] = -gg.A * (gg.G10 * dx + gg.G11 * dy);
                }
            }
        }
    }
    __syncthreads();
    // ---- G2: rows of (K d)_t, t = 16 wave + li
    const int t = 16 * wave + li;
    const int64_t i = i0 + t;
    Real cf[3] = {Real(0), Real(0), Real(0)};  // -A m00, -A m01, -A m11
    if (i < ne) {
        const double4 e = geo[i];
        const Geo gd = make_geo(e.x, e.y, e.z, e.w);
        cf[0] = (Real)(-gd.A * (gd.G00 * gd.G00 + gd.G01 * gd.G01));
        cf[1] = (Real)(-gd.A * (gd.G00 * gd.G10 + gd.G01 * gd.G11));
        cf[2] = (Real)(-gd.A * (gd.G10 * gd.G10 + gd.G11 * gd.G11));
    }
    const Real* zt = sz + t * KE;
    const Real* dt = sd + t * N;
    if constexpr (sizeof(Real) == 8) {
        d4v acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < D::KSE; ++ks) {
            const int kk = 4 * ks + g;
            const double b = kk < KE ? (double)zt[kk] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(F.a2[ks], b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int kv = 0; kv < D::KSV; ++kv) {
            const int c = kv / D::KS1;                 // volume component (compile time)
            const int l = 4 * (kv - c * D::KS1) + g;
            const double b = l < N ? (double)(cf[c] * dt[l]) : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(F.a2[D::KSE + kv], b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) y[j] = (Real)acc[j];
    } else {
        f4v hi = {0, 0, 0, 0}, lo = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < D::KSE32; ++ks) {
            float bv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int kk = 32 * ks + 8 * g + e;
                bv[e] = kk < KE ? (float)zt[kk] : 0.0f;
            }
            bf3_mma(F.a2[ks], bv, hi, lo);
        }
#pragma unroll
        for (int kv = 0; kv < D::KSV32; ++kv) {
            // positions 32 kv + 8 g + e: component 2 kv + g / 2, node 8 (g % 2) + e
            const int c = 2 * kv + (g >> 1);
            const Real cc = c == 0 ? cf[0] : (c == 1 ? cf[1] : cf[2]);
            float bv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int l = 8 * (g & 1) + e;
                bv[e] = (c < 3 && l < N) ? (float)(cc * dt[l]) : 0.0f;
            }
            bf3_mma(F.a2[D::KSE32 + kv], bv, hi, lo);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) y[j] = (Real)(hi[j] + lo[j]);
    }
}

// Standalone apply in internal order: out = scale * K p (tiles of 64, one tile per block).
template <int P, typename Real, class Ops>
__global__ __launch_bounds__(kMxThreads) void k_apply_mx(const Ops* __restrict__ ops,
                                                         const MxTab<P>* __restrict__ tab,
                                                         const double4* __restrict__ geo,
                                                         const int4* __restrict__ nbr,
                                                         const int* __restrict__ halo_pad, int hmax,
                                                         int64_t ne, const Real* __restrict__ p,
                                                         Real* __restrict__ out) {
    using D = MxDims<P>;
    constexpr int N = D::N;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Real* sd = reinterpret_cast<Real*>(lds_raw);
    Real* se = sd + (size_t)(T + hmax) * N + (size_t)T * N;
    Real* sz = se + (size_t)(T + hmax) * D::R1;
    const int hs = hmax > 0 ? hmax : 1;
    MxFrag<P, Real> F;
    F.load(tab, threadIdx.x & 63);
    const int64_t tile = blockIdx.x;
    const int64_t i0 = tile * T;
    const int nown = (int)((ne - i0) < T ? (ne - i0) : T) * N;
    for (int f = threadIdx.x; f < T * N; f += kMxThreads) sd[f] = f < nown ? p[i0 * N + f] : Real(0);
    for (int e = threadIdx.x; e < hmax * N; e += kMxThreads) {
        const int h = halo_pad[tile * hs + e / N];
        sd[T * N + e] = h >= 0 ? p[(int64_t)h * N + (e - (e / N) * N)] : Real(0);
    }
    __syncthreads();
    Real y[4];
    mx_tile_op<P, Real, Ops>(*ops, F, geo, nbr, halo_pad + tile * hs, hmax, i0, ne, sd, se, sz, y);
    const int lane = threadIdx.x & 63;
    const int t = 16 * (threadIdx.x >> 6) + (lane & 15), g = lane >> 4;
    const int64_t i = i0 + t;
    if (i < ne) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = out_row<Real>(g, j);
            if (k < N) out[i * N + k] = y[j];
        }
    }
}

// One CG iteration (the k_cg_step recurrences of kernels_cg.hip) with the operator above:
// several tiles per block, in the per-XCD chunk order; x is the FP64 correction e (or the FP32
// correction of the mixed form).  kStream: x read and written non-temporally.
template <int P, typename Real, class Ops, bool kStream>
__global__ __launch_bounds__(kMxThreads) void k_cg_step_mx(const Ops* __restrict__ ops,
                                                           const MxTab<P>* __restrict__ tab,
                                                           const double4* __restrict__ geo,
                                                           const int4* __restrict__ nbr,
                                                           const int* __restrict__ halo_pad,
                                                           int hmax, int64_t ne,
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
    using D = MxDims<P>;
    using S = CgScalars;
    constexpr int N = D::N;
    constexpr int NT = kMxThreads;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Real* sd = reinterpret_cast<Real*>(lds_raw);
    Real* sr = sd + (size_t)(T + hmax) * N;
    Real* se = sr + (size_t)T * N;
    Real* sz = se + (size_t)(T + hmax) * D::R1;
    const int G = gridDim.x;
    const int hs = hmax > 0 ? hmax : 1;
    const int nhe = hmax * N;
    const int64_t ntiles = (ne + T - 1) / T;
    const int lb = (int)(blockIdx.x & 7) * (G >> 3) + (int)(blockIdx.x >> 3);
    const int64_t per = (ntiles + G - 1) / G;
    const int64_t t_begin = lb * per;
    const int64_t t_end = (lb + 1) * per < ntiles ? (lb + 1) * per : ntiles;

    const double done = scal[S::DONE];
    const double it = scal[S::ITER0 + parity];
    double alpha = 0.0, beta = 0.0;
    if (it > 0.0) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int b0 = threadIdx.x; b0 < G; b0 += NT) {
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] += part_in[c * G + b0];
        }
        block_sum_all<4, NT>(v);
        const double rr = v[0], dq = v[1], rq = v[2], qq = v[3];
        if (done != 0.0) return;
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
                scal[S::ITER] = it - 1.0;
            }
            return;
        }
        alpha = rr / dq;
        const double rr_next = fma(alpha * alpha, qq, fma(-2.0 * alpha, rq, rr));
        beta = rr_next / rr;
    } else if (done != 0.0) {
        return;
    }
    MxFrag<P, Real> F;
    F.load(tab, threadIdx.x & 63);
    const Real ra = (Real)alpha, rb = (Real)beta;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4;
    const int tq = 16 * wave + (lane & 15);
    for (int64_t tile = t_begin; tile < t_end; ++tile) {
        const int64_t i0 = tile * T;
        const int nown = (int)((ne - i0) < T ? (ne - i0) : T) * N;
        const int64_t base = i0 * N;
        // phase 1: the tile's state update (coalesced) and the directions of tile and halo
        for (int f = threadIdx.x; f < T * N; f += NT) {
            if (f < nown) {
                const int64_t o = base + f;
                const Real dprev = d_in[o];
                const Real rk = mad(-ra, q_in[o], r_in[o]);
                const Real dk = mad(rb, dprev, rk);
                if constexpr (kStream)
                    __builtin_nontemporal_store(mad(ra, dprev, __builtin_nontemporal_load(&x[o])), &x[o]);
                else
                    x[o] = mad(ra, dprev, x[o]);
                r_out[o] = rk;
                d_out[o] = dk;
                sd[f] = dk;
                sr[f] = rk;
                acc[0] = fma((double)rk, (double)rk, acc[0]);
            } else {
                sd[f] = Real(0);
                sr[f] = Real(0);
            }
        }
        for (int e0 = threadIdx.x; e0 < nhe; e0 += 2 * NT) {
            int id2[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = e0 + u * NT;
                id2[u] = e < nhe ? halo_pad[tile * hs + e / N] : -2;
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
            for (int u = 0; u < 2; ++u) {
                if (id2[u] >= 0) sd[T * N + e0 + u * NT] = mad(rb, hd[u], mad(-ra, hq[u], hr[u]));
                else if (id2[u] == -1) sd[T * N + e0 + u * NT] = Real(0);  // padding
            }
        }
        __syncthreads();
        Real y[4];
        mx_tile_op<P, Real, Ops>(*ops, F, geo, nbr, halo_pad + tile * hs, hmax, i0, ne, sd, se, sz, y);
        // phase 3: q_k = -K d_k from the output registers, and the dot products
        const int64_t i = i0 + tq;
        if (i < ne) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = out_row<Real>(g, j);
                if (k < N) {
                    const Real qk = -y[j];
                    q_out[i * N + k] = qk;
                    const double dk = sd[tq * N + k], rk = sr[tq * N + k], qd = qk;
                    acc[1] = fma(dk, qd, acc[1]);
                    acc[2] = fma(rk, qd, acc[2]);
                    acc[3] = fma(qd, qd, acc[3]);
                }
            }
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

// caller order <-> internal order (through perm), any word type
template <typename Real>
__global__ __launch_bounds__(kBlockFlat) void k_gather_mx(int64_t n, int nphi, const int* __restrict__ perm,
                                                          const Real* __restrict__ src,
                                                          Real* __restrict__ dst) {
    for (int64_t t = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlockFlat) {
        const int64_t i = t / nphi;
        dst[t] = src[(int64_t)perm[i] * nphi + (t - i * nphi)];
    }
}

template <typename Real>
__global__ __launch_bounds__(kBlockFlat) void k_scatter_mx(int64_t n, int nphi, const int* __restrict__ perm,
                                                           const Real* __restrict__ src,
                                                           Real* __restrict__ dst) {
    for (int64_t t = (int64_t)blockIdx.x * kBlockFlat + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlockFlat) {
        const int64_t i = t / nphi;
        dst[(int64_t)perm[i] * nphi + (t - i * nphi)] = src[t];
    }
}

// ---------------------------------------------------------------- host: tables
uint16_t bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

double bf16_value(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
}

// x = hi + mid + lo (bfloat16 terms, each the rounding of what the previous ones leave)
void split3_host(double x, uint16_t* out) {
    double r = x;
    for (int s = 0; s < 3; ++s) {
        out[s] = bf16_rne((float)r);
        r -= bf16_value(out[s]);
    }
}

template <int P>
const MxTab<P>* tab_of(const sld_disc_s* d) { return reinterpret_cast<const MxTab<P>*>(d->mx_dev); }
template <int P>
const RefOps<P>* ops64_of(const sld_disc_s* d) { return reinterpret_cast<const RefOps<P>*>(d->ops_dev); }
template <int P>
const RefOps32<P>* ops32x_of(const sld_disc_s* d) {
    return reinterpret_cast<const RefOps32<P>*>(d->ops32_dev);
}

#define SLD_MX_DISPATCH(p, CALL)                                \
    switch (p) {                                                \
        case 1: { constexpr int PP = 1; CALL; } break;          \
        case 2: { constexpr int PP = 2; CALL; } break;          \
        case 3: { constexpr int PP = 3; CALL; } break;          \
        case 4: { constexpr int PP = 4; CALL; } break;          \
        default: return hipErrorInvalidValue;                   \
    }

}  // namespace

template <int P>
int build_mxtab(const void* refops, MxTab<P>* out) {
    using D = MxDims<P>;
    constexpr int N = D::N, NE = D::NE, R1 = D::R1, KE = D::KE;
    const RefOps<P>& R = *static_cast<const RefOps<P>*>(refops);
    // dense E1 [R1][N] and W2 [N][K2] in the logical layouts of mx.h
    std::vector<double> E1((size_t)R1 * N, 0.0);
    for (int al = 0; al < 3; ++al)
        for (int c = 0; c < 2; ++c)
            for (int m = 0; m < NE; ++m)
                for (int l = 0; l < N; ++l) E1[(size_t)((al * 2 + c) * NE + m) * N + l] = R.E[al][c][m][l];
    // G2 columns: F64 layout (volume component stride NV) and BF3 layout (stride 16, edge part
    // padded to whole k-steps of 32)
    auto w2 = [&](int k, int kk, int vstride, int vbase) -> double {
        if (k >= N) return 0.0;
        if (kk < KE) {
            const int al = kk / (3 * NE), s = (kk - al * 3 * NE) / NE, m = kk - al * 3 * NE - s * NE;
            if (s == 0) {
                // line term: row edge_node(al, mm) takes M1[mm][m] tn_m
                for (int mm = 0; mm < NE; ++mm)
                    if (edge_node(P, al, mm) == k) return R.M1[mm][m];
                return 0.0;
            }
            return R.Pt[al][s - 1][k][m];
        }
        if (kk < vbase) return 0.0;
        const int c = (kk - vbase) / vstride, l = (kk - vbase) - c * vstride;
        if (c >= 3 || l >= N) return 0.0;
        return R.S[c][k][l];
    };
    for (int rb = 0; rb < 2; ++rb)
        for (int ks = 0; ks < D::KS1; ++ks)
            for (int lane = 0; lane < 64; ++lane) {
                const int row = 16 * rb + (lane & 15), col = 4 * ks + (lane >> 4);
                out->a1[rb][ks][lane] = (row < R1 && col < N) ? E1[(size_t)row * N + col] : 0.0;
            }
    for (int ks = 0; ks < D::KS2; ++ks)
        for (int lane = 0; lane < 64; ++lane)
            out->a2[ks][lane] = w2(lane & 15, 4 * ks + (lane >> 4), D::NV, 4 * D::KSE);
    for (int rb = 0; rb < 2; ++rb)
        for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 8; ++e) {
                const int row = 16 * rb + (lane & 15), col = 8 * (lane >> 4) + e;
                uint16_t sp[3];
                split3_host((row < R1 && col < N) ? E1[(size_t)row * N + col] : 0.0, sp);
                for (int s = 0; s < 3; ++s) out->b1[rb][s][lane][e] = sp[s];
            }
    for (int ks = 0; ks < D::KS232; ++ks)
        for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 8; ++e) {
                uint16_t sp[3];
                split3_host(w2(lane & 15, 32 * ks + 8 * (lane >> 4) + e, 16, 32 * D::KSE32), sp);
                for (int s = 0; s < 3; ++s) out->b2[ks][s][lane][e] = sp[s];
            }
    return 0;
}

template int build_mxtab<1>(const void*, MxTab<1>*);
template int build_mxtab<2>(const void*, MxTab<2>*);
template int build_mxtab<3>(const void*, MxTab<3>*);
template int build_mxtab<4>(const void*, MxTab<4>*);

size_t mx_tab_bytes(int p) {
    switch (p) {
        case 1: return sizeof(MxTab<1>);
        case 2: return sizeof(MxTab<2>);
        case 3: return sizeof(MxTab<3>);
        case 4: return sizeof(MxTab<4>);
    }
    return 0;
}

int build_mx_tables(int p, const void* refops, void* out) {
    switch (p) {
        case 1: return build_mxtab<1>(refops, static_cast<MxTab<1>*>(out));
        case 2: return build_mxtab<2>(refops, static_cast<MxTab<2>*>(out));
        case 3: return build_mxtab<3>(refops, static_cast<MxTab<3>*>(out));
        case 4: return build_mxtab<4>(refops, static_cast<MxTab<4>*>(out));
    }
    return -1;
}

size_t mx_lds_bytes(int p, int hmax, size_t word) {
    size_t w = 0;
    switch (p) {
        case 1: w = mx_lds_words<1>(hmax); break;
        case 2: w = mx_lds_words<2>(hmax); break;
        case 3: w = mx_lds_words<3>(hmax); break;
        case 4: w = mx_lds_words<4>(hmax); break;
    }
    return w * word;
}

hipError_t launch_apply_mx(const sld_disc_s* d, const void* p, void* out, bool f32, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    const int64_t n = m->ne * d->nphi;
    const unsigned tiles = (unsigned)((m->ne + T - 1) / T);
    const size_t lds = mx_lds_bytes(d->p, m->hmax, f32 ? sizeof(float) : sizeof(double));
    if (f32) {
        hipLaunchKernelGGL(k_gather_mx<float>, dim3(w.grid), dim3(kBlockFlat), 0, s, n, d->nphi,
                           m->perm, static_cast<const float*>(p), w.d32[1]);
        SLD_MX_DISPATCH(d->p, hipLaunchKernelGGL((k_apply_mx<PP, float, RefOps32<PP>>), dim3(tiles),
                                                 dim3(kMxThreads), lds, s, ops32x_of<PP>(d), tab_of<PP>(d),
                                                 m->geo_i, m->nbr_i, m->halo_pad, m->hmax, m->ne,
                                                 w.d32[1], w.q32[1]));
        hipLaunchKernelGGL(k_scatter_mx<float>, dim3(w.grid), dim3(kBlockFlat), 0, s, n, d->nphi,
                           m->perm, w.q32[1], static_cast<float*>(out));
    } else {
        hipLaunchKernelGGL(k_gather_mx<double>, dim3(w.grid), dim3(kBlockFlat), 0, s, n, d->nphi,
                           m->perm, static_cast<const double*>(p), w.d[1]);
        SLD_MX_DISPATCH(d->p, hipLaunchKernelGGL((k_apply_mx<PP, double, RefOps<PP>>), dim3(tiles),
                                                 dim3(kMxThreads), lds, s, ops64_of<PP>(d), tab_of<PP>(d),
                                                 m->geo_i, m->nbr_i, m->halo_pad, m->hmax, m->ne,
                                                 w.d[1], w.q[1]));
        hipLaunchKernelGGL(k_scatter_mx<double>, dim3(w.grid), dim3(kBlockFlat), 0, s, n, d->nphi,
                           m->perm, w.q[1], static_cast<double*>(out));
    }
    return hipGetLastError();
}

// one FP64 (x = e) or FP32 (mixed inner) CG iteration with the MFMA operator
hipError_t launch_cg_step_mx(const sld_disc_s* d, int parity, bool f32, bool stream_x, hipStream_t s) {
    const sld_mesh_s* m = d->mesh;
    const CgWork& w = d->cg;
    const int G = w.grid;
    const int o = 1 - parity;
    if (G & 7) return hipErrorInvalidValue;
    const size_t lds = mx_lds_bytes(d->p, m->hmax, f32 ? sizeof(float) : sizeof(double));
#define SLD_MXSTEP(R, OPS, ST, X, RB, QB, DB, PART, SC)                                             \
    SLD_MX_DISPATCH(d->p, hipLaunchKernelGGL((k_cg_step_mx<PP, R, OPS<PP>, ST>), dim3(G),          \
                                             dim3(kMxThreads), lds, s,                              \
                                             reinterpret_cast<const OPS<PP>*>(f32 ? d->ops32_dev : d->ops_dev), \
                                             tab_of<PP>(d), m->geo_i, m->nbr_i, m->halo_pad,        \
                                             m->hmax, m->ne, X, RB[parity], QB[parity], DB[parity], \
                                             RB[o], QB[o], DB[o], PART + parity * 4 * G,            \
                                             PART + o * 4 * G, SC, parity))
    if (f32) {
        if (stream_x) {
            SLD_MXSTEP(float, RefOps32, true, w.e32, w.r32, w.q32, w.d32, w.part32, w.scal_in);
        } else {
            SLD_MXSTEP(float, RefOps32, false, w.e32, w.r32, w.q32, w.d32, w.part32, w.scal_in);
        }
    } else {
        if (stream_x) {
            SLD_MXSTEP(double, RefOps, true, w.e, w.r, w.q, w.d, w.part, w.scal);
        } else {
            SLD_MXSTEP(double, RefOps, false, w.e, w.r, w.q, w.d, w.part, w.scal);
        }
    }
#undef SLD_MXSTEP
    return hipGetLastError();
}

// resident blocks of the MFMA CG kernel per CU (occupancy calculator), 0 on failure
int mx_blocks_per_cu(const sld_disc_s* d, bool f32) {
    const size_t lds = mx_lds_bytes(d->p, d->mesh->hmax, f32 ? sizeof(float) : sizeof(double));
    int nb = 0;
    hipError_t e = hipSuccess;
    switch (d->p) {
#define SLD_MX_OCC(PP)                                                                              \
    case PP:                                                                                        \
        e = f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                                     \
                      &nb, (k_cg_step_mx<PP, float, RefOps32<PP>, false>), kMxThreads, lds)         \
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(                                     \
                      &nb, (k_cg_step_mx<PP, double, RefOps<PP>, false>), kMxThreads, lds);         \
        break;
        SLD_MX_OCC(1)
        SLD_MX_OCC(2)
        SLD_MX_OCC(3)
        SLD_MX_OCC(4)
#undef SLD_MX_OCC
        default: return 0;
    }
    return e == hipSuccess ? nb : 0;
}
