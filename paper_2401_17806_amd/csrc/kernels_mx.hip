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
// Tuning constants (compile time): halo entries per thread whose ids are requested one tile
// ahead (larger halos take a plain loop for the rest); minimum waves per SIMD the CG kernel is
// compiled for (the register budget); whether the edge stage reads the neighbour's geometry from
// the per-edge copy (requested with the triangle's own) or through the neighbour's id.
// Measured per FP64 / FP32 iteration on the 512x512x2, p = 3 mesh (the software-pipelined tile
// loop below): two waves per SIMD and geometry through the id 134 / 120 us; with the per-edge
// copy 141 / 116 us; three waves per SIMD spill registers to scratch, 251 / 204 us.
#ifndef SLD_MX_HALO_PER
#define SLD_MX_HALO_PER 3
#endif
#ifndef SLD_MX_WAVES
#define SLD_MX_WAVES 2
#endif
#ifndef SLD_MX_GEONB
#define SLD_MX_GEONB 0
#endif
constexpr int kHaloPer = SLD_MX_HALO_PER;
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

// (G1's operands stay in registers for the whole launch; G2's, the larger set, are requested
// from the cache-resident table at the end of each tile's edge-node stage, so that they are not
// live during the state update and G1.)
template <int P>
struct MxFrag<P, double> {
    using D = MxDims<P>;
    const MxTab<P>* tab;
    double a1[2][D::KS1];
    __device__ __forceinline__ void load(const MxTab<P>* __restrict__ t, int lane) {
        tab = t;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int ks = 0; ks < D::KS1; ++ks) a1[rb][ks] = t->a1[rb][ks][lane];
    }
};

template <int P>
struct MxFrag<P, float> {
    using D = MxDims<P>;
    const MxTab<P>* tab;
    bf8v a1[2][3];
    __device__ __forceinline__ void load(const MxTab<P>* __restrict__ t, int lane) {
        tab = t;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int s = 0; s < 3; ++s) a1[rb][s] = load_bf8(&t->b1[rb][s][lane][0]);
    }
};

template <int P, typename Real>
struct MxFrag2;

template <int P>
struct MxFrag2<P, double> {
    double a2[MxDims<P>::KS2];
    __device__ __forceinline__ void load(const MxTab<P>* __restrict__ t, int lane) {
#pragma unroll
        for (int ks = 0; ks < MxDims<P>::KS2; ++ks) a2[ks] = t->a2[ks][lane];
    }
};

template <int P>
struct MxFrag2<P, float> {
    bf8v a2[MxDims<P>::KS232][3];
    __device__ __forceinline__ void load(const MxTab<P>* __restrict__ t, int lane) {
#pragma unroll
        for (int ks = 0; ks < MxDims<P>::KS232; ++ks)
#pragma unroll
            for (int s = 0; s < 3; ++s) a2[ks][s] = load_bf8(&t->b2[ks][s][lane][0]);
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

// LDS of one block, in words of Real, rows of odd stride (MxDims): sd [T + hmax][NS] directions
// of the tile then its halo; sr [T][NS] residuals (CG only); se [T + hmax][R1S] edge-node
// derivatives.
template <int P>
inline size_t mx_lds_words(int hmax) {
    using D = MxDims<P>;
    return (size_t)(T + hmax) * D::NS + (size_t)T * D::NS + (size_t)(T + hmax) * D::R1S;
}

// Per-thread geometry of one tile, requested before the tile's state so that its latency
// overlaps the state loads and G1: lane (t, g) of wave w needs triangle t = 16 w + lane % 16, its
// neighbour table and its neighbours' geometry (the per-edge copy, so no load waits for a
// neighbour's id).
struct MxPre {
    int4 nb4;
    double4 e, er[3];
};

__device__ __forceinline__ void mx_prefetch(const double4* __restrict__ geo,
                                            const double4* __restrict__ geo_nb,
                                            const int4* __restrict__ nbr, int64_t i0, int64_t ne,
                                            MxPre& pre) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = i0 + 16 * wave + (lane & 15);
    if (i < ne) {
        pre.nb4 = nbr[i];
        pre.e = geo[i];
#if SLD_MX_GEONB
#pragma unroll
        for (int al = 0; al < 3; ++al) pre.er[al] = geo_nb[i * 3 + al];
#else
        (void)geo_nb;
#pragma unroll
        for (int al = 0; al < 3; ++al) {
            const int nb = pick(pre.nb4, al);
            pre.er[al] = nb >= 0 ? geo[nb >> 2] : make_double4(0, 0, 0, 0);
        }
#endif
    }
}

// The operator on one tile whose directions (tile then halo, zero where padded) are in sd:
// returns in y four rows of (K d)_t for t = 16 wave + (lane & 15), g = lane / 16.
// (y[j] is row out_row<Real>(g, j).)  The caller separates the next tile's LDS writes from G2's
// reads with a barrier.  Requires every edge to have a neighbour (no walls).
template <int P, typename Real, class Ops>
__device__ __forceinline__ void mx_tile_op(const Ops& R, const MxFrag<P, Real>& F, const MxPre& pre,
                                           const int* __restrict__ halo_row, int hmax, int64_t i0,
                                           int64_t ne, const Real* sd, Real* se,
                                           Real (&y)[4]) {
    using D = MxDims<P>;
    constexpr int N = D::N, NE = D::NE, R1 = D::R1;
    constexpr int NS = D::NS, R1S = D::R1S;
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
                const double b = (sv && l < N) ? (double)sd[slot * NS + l] : 0.0;
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(F.a1[0][ks], b, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(F.a1[1][ks], b, acc1, 0, 0, 0);
            }
            if (sv) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r0 = out_row<double>(g, j), r1 = 16 + r0;
                    if (r0 < R1) se[slot * R1S + r0] = (Real)acc0[j];
                    if (r1 < R1) se[slot * R1S + r1] = (Real)acc1[j];
                }
            }
        } else {
            float bv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int l = 8 * g + e;
                bv[e] = (sv && l < N) ? (float)sd[slot * NS + l] : 0.0f;
            }
            f4v h0 = {0, 0, 0, 0}, l0 = {0, 0, 0, 0}, h1 = {0, 0, 0, 0}, l1 = {0, 0, 0, 0};
            bf3_mma(F.a1[0], bv, h0, l0);
            bf3_mma(F.a1[1], bv, h1, l1);
            if (sv) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r0 = out_row<float>(g, j), r1 = 16 + r0;
                    if (r0 < R1) se[slot * R1S + r0] = (Real)(h0[j] + l0[j]);
                    if (r1 < R1) se[slot * R1S + r1] = (Real)(h1[j] + l1[j]);
                }
            }
        }
    }
    __syncthreads();
    // ---- edge nodes, per wave and without a barrier before G2: lane (t, g) of wave w forms,
    // for tile triangle t = 16 w + lane % 16 and its nodes m = g + 4 q on each edge al, the
    // normal flux and the sub-triangle correction of the closed form of Mhat_j^{-1} (the same
    // algebra as the vector-unit operator core), which are exactly its B operands of G2
    const int t = 16 * wave + li;
    const int64_t i = i0 + t;
    constexpr int NQ = D::NQ;
    Real z[NQ][9];  // [q][al * 3 + s]: s = 0 normal flux, 1 / 2 the two reference components
    Real cf[3] = {Real(0), Real(0), Real(0)};  // -A m00, -A m01, -A m11 (volume term)
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int c = 0; c < 9; ++c) z[q][c] = Real(0);
    if (i < ne) {
        const double4 e = pre.e;
        const Geo gd = make_geo(e.x, e.y, e.z, e.w);
        const GeoR<Real> gg(gd);
        cf[0] = (Real)(-gd.A * (gd.G00 * gd.G00 + gd.G01 * gd.G01));
        cf[1] = (Real)(-gd.A * (gd.G00 * gd.G10 + gd.G01 * gd.G11));
        cf[2] = (Real)(-gd.A * (gd.G10 * gd.G10 + gd.G11 * gd.G11));
#pragma unroll
        for (int al = 0; al < 3; ++al) {
            const int nb = pick(pre.nb4, al);
            if (nb < 0) continue;  // (not reached: meshes without wall edges)
            const int slot = (pre.nb4.w >> (10 * al)) & 1023;
            const int ar = nb & 3;
            const double4 er = pre.er[al];
            const Geo grd = make_geo(er.x, er.y, er.z, er.w);
            const GeoR<Real> gr(grd);
            const Real wsum = (Real)(1.0 / (gd.A + grd.A));
            // |Gamma| n, outward: the edge vector v_{al+1} - v_al turned clockwise
            const double ex = al == 0 ? e.x : (al == 1 ? e.z - e.x : -e.z);
            const double ey = al == 0 ? e.y : (al == 1 ? e.w - e.y : -e.w);
            const Real snx = (Real)ey, sny = (Real)(-ex);
            // jump at the edge's nodes and C times it (C couples the nodes of the edge)
            Real delta[NE], cdv[NE];
#pragma unroll
            for (int mm = 0; mm < NE; ++mm)
                delta[mm] = sd[slot * NS + edge_node_rt<P>(ar, P - mm)] - sd[t * NS + edge_node(P, al, mm)];
#pragma unroll
            for (int mm = 0; mm < NE; ++mm) {
                Real cd = 0;
#pragma unroll
                for (int qq = 0; qq < NE; ++qq) cd = mad((Real)R.C[mm][qq], delta[qq], cd);
                cdv[mm] = cd;
            }
            const Real* dso = se + t * R1S + al * 2 * NE;
            const Real* dsn = se + slot * R1S + ar * 2 * NE;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int m = 4 * q + g;
                if (m >= NE) continue;
                Real cd = cdv[0];
#pragma unroll
                for (int mm = 1; mm < NE; ++mm) cd = m == mm ? cdv[mm] : cd;
                const Real ds0 = dso[m], ds1 = dso[NE + m];
                const Real dn0 = dsn[P - m], dn1 = dsn[NE + P - m];
                const Real gsx = gg.G00 * ds0 + gg.G10 * ds1, gsy = gg.G01 * ds0 + gg.G11 * ds1;
                const Real gnx = gr.G00 * dn0 + gr.G10 * dn1, gny = gr.G01 * dn0 + gr.G11 * dn1;
                const Real hx = (gg.A * gsx + gr.A * gnx + Real(3) * snx * cd) * wsum;
                const Real hy = (gg.A * gsy + gr.A * gny + Real(3) * sny * cd) * wsum;
                const Real dx = hx - gsx, dy = hy - gsy;
                z[q][al * 3 + 0] = snx * hx + sny * hy;
                z[q][al * 3 + 1] = -gg.A * (gg.G00 * dx + gg.G01 * dy);
                z[q][al * 3 + 2] = -gg.A * (gg.G10 * dx + gg.G11 * dy);
            }
        }
    }
    // ---- G2: rows of (K d)_t.  (The table address is laundered through an empty asm so the
    // compiler cannot hoist these loads to the top of the tile loop, where they would hold
    // registers through G1.)
    const MxTab<P>* tab2 = F.tab;
    __asm__ volatile("" : "+s"(tab2));
    MxFrag2<P, Real> F2;
    F2.load(tab2, lane);
    const Real* dt = sd + t * NS;
    if constexpr (sizeof(Real) == 8) {
        d4v acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < D::KSE; ++ks)  // ks = (al * 3 + s) * NQ + q
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(F2.a2[ks], (double)z[ks % NQ][ks / NQ], acc, 0, 0, 0);
#pragma unroll
        for (int kv = 0; kv < D::KSV; ++kv) {
            const int c = kv / D::KS1;                 // volume component (compile time)
            const int l = 4 * (kv - c * D::KS1) + g;
            const double b = l < N ? (double)(cf[c] * dt[l]) : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(F2.a2[D::KSE + kv], b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) y[j] = (Real)acc[j];
    } else {
        f4v hi = {0, 0, 0, 0}, lo = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < D::KSE32; ++ks) {  // ks = 2 q + h: elements e <-> al * 3 + s = 8 h + e
            float bv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int c = 8 * (ks & 1) + e;
                bv[e] = c < 9 ? (float)z[ks >> 1][c < 9 ? c : 0] : 0.0f;
            }
            bf3_mma(F2.a2[ks], bv, hi, lo);
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
        bf3_mma(F2.a2[D::KSE32 + kv], bv, hi, lo);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) y[j] = (Real)(hi[j] + lo[j]);
    }
}

// Standalone apply in internal order: out = scale * K p (tiles of 64, one tile per block).
template <int P, typename Real, class Ops>
__global__ __launch_bounds__(kMxThreads, 3) void k_apply_mx(const Ops* __restrict__ ops,
                                                         const MxTab<P>* __restrict__ tab,
                                                         const double4* __restrict__ geo,
                                                         const double4* __restrict__ geo_nb,
                                                         const int4* __restrict__ nbr,
                                                         const int* __restrict__ halo_pad, int hmax,
                                                         int64_t ne, const Real* __restrict__ p,
                                                         Real* __restrict__ out) {
    using D = MxDims<P>;
    constexpr int N = D::N;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Real* sd = reinterpret_cast<Real*>(lds_raw);
    Real* se = sd + (size_t)(T + hmax) * D::NS + (size_t)T * D::NS;
    const int hs = hmax > 0 ? hmax : 1;
    MxFrag<P, Real> F;
    F.load(tab, threadIdx.x & 63);
    const int64_t tile = blockIdx.x;
    const int64_t i0 = tile * T;
    const int nown = (int)((ne - i0) < T ? (ne - i0) : T) * N;
    MxPre pre;
    mx_prefetch(geo, geo_nb, nbr, i0, ne, pre);
    for (int f = threadIdx.x; f < T * N; f += kMxThreads)
        sd[(f / N) * D::NS + f % N] = f < nown ? p[i0 * N + f] : Real(0);
    for (int e = threadIdx.x; e < hmax * N; e += kMxThreads) {
        const int h = halo_pad[tile * hs + e / N];
        sd[(T + e / N) * D::NS + e % N] = h >= 0 ? p[(int64_t)h * N + e % N] : Real(0);
    }
    __syncthreads();
    Real y[4];
    mx_tile_op<P, Real, Ops>(*ops, F, pre, halo_pad + tile * hs, hmax, i0, ne, sd, se, y);
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
__global__ __launch_bounds__(kMxThreads, SLD_MX_WAVES) void k_cg_step_mx(const Ops* __restrict__ ops,
                                                           const MxTab<P>* __restrict__ tab,
                                                           const double4* __restrict__ geo,
                                                           const double4* __restrict__ geo_nb,
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
    constexpr int NS = D::NS;
    Real* sr = sd + (size_t)(T + hmax) * NS;
    Real* se = sr + (size_t)T * NS;
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
    // The tile loop is software-pipelined: the state of tile k + 1 (own entries and halo) is
    // requested right after tile k's state update, so it is in flight while tile k runs G1, the
    // edge-node stage and G2; the halo ids run one more tile ahead.
    // Own entry f = threadIdx.x + u NT (u < PER) and halo entry e = threadIdx.x + u NT
    // (u < kHaloPer) of a tile; hid: the entry's triangle id, -1 padding, -2 none.
    constexpr int PER = (T * N + NT - 1) / NT;
    Real sx[PER], srr[PER], sq[PER], sdd[PER];     // next tile: x, r, q, d of its own entries
    Real hd[kHaloPer], hq[kHaloPer], hr[kHaloPer];  // next tile: its halo's d, q, r
    int hid_n[kHaloPer], hid_nn[kHaloPer];         // halo ids of the next tile / the one after
    auto load_ids = [&](int64_t tile, int (&h)[kHaloPer]) {
#pragma unroll
        for (int u = 0; u < kHaloPer; ++u) {
            const int e = threadIdx.x + u * NT;
            h[u] = (tile < t_end && e < nhe) ? halo_pad[tile * hs + e / N] : -2;
        }
    };
    auto request = [&](int64_t tile) {  // state of `tile` (halo ids in hid_n)
        const int64_t i0 = tile * T;
        const int nown = tile < t_end ? (int)((ne - i0) < T ? (ne - i0) : T) * N : 0;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int f = threadIdx.x + u * NT;
            if (f < nown) {
                const int64_t o = i0 * N + f;
                sdd[u] = d_in[o];
                sq[u] = q_in[o];
                srr[u] = r_in[o];
                if constexpr (kStream) sx[u] = __builtin_nontemporal_load(&x[o]);
                else sx[u] = x[o];
            }
        }
#pragma unroll
        for (int u = 0; u < kHaloPer; ++u) {
            if (hid_n[u] >= 0) {
                const int e = threadIdx.x + u * NT;
                const int64_t o = (int64_t)hid_n[u] * N + e % N;
                hd[u] = d_in[o];
                hq[u] = q_in[o];
                hr[u] = r_in[o];
            }
        }
    };
    load_ids(t_begin, hid_n);
    request(t_begin);
    load_ids(t_begin + 1, hid_nn);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4;
    const int tq = 16 * wave + (lane & 15);
    for (int64_t tile = t_begin; tile < t_end; ++tile) {
        const int64_t i0 = tile * T;
        const int nown = (int)((ne - i0) < T ? (ne - i0) : T) * N;
        const int64_t base = i0 * N;
        MxPre pre;
        mx_prefetch(geo, geo_nb, nbr, i0, ne, pre);
        // phase 1: the tile's state update (coalesced) and the directions of tile and halo
        // into LDS, from the registers requested one tile earlier
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int f = threadIdx.x + u * NT;
            if (f < nown) {
                const int64_t o = base + f;
                const Real rk = mad(-ra, sq[u], srr[u]);
                const Real dk = mad(rb, sdd[u], rk);
                const Real xk = mad(ra, sdd[u], sx[u]);
                if constexpr (kStream) __builtin_nontemporal_store(xk, &x[o]);
                else x[o] = xk;
                r_out[o] = rk;
                d_out[o] = dk;
                sd[(f / N) * NS + f % N] = dk;
                sr[(f / N) * NS + f % N] = rk;
                acc[0] = fma((double)rk, (double)rk, acc[0]);
            } else if (f < T * N) {
                sd[(f / N) * NS + f % N] = Real(0);
                sr[(f / N) * NS + f % N] = Real(0);
            }
        }
#pragma unroll
        for (int u = 0; u < kHaloPer; ++u) {
            const int e = threadIdx.x + u * NT;
            if (hid_n[u] != -2) {
                Real* dst = sd + (T + e / N) * NS + e % N;
                *dst = hid_n[u] >= 0 ? mad(rb, hd[u], mad(-ra, hq[u], hr[u])) : Real(0);  // -1: padding
            }
        }
        // (halo entries beyond kHaloPer per thread: very large halos only)
        for (int e = threadIdx.x + kHaloPer * NT; e < nhe; e += NT) {
            const int h = halo_pad[tile * hs + e / N];
            const int64_t o = (int64_t)h * N + e % N;
            sd[(T + e / N) * NS + e % N] = h >= 0 ? mad(rb, d_in[o], mad(-ra, q_in[o], r_in[o])) : Real(0);
        }
        // the next tile's state goes out now; the halo ids one tile further
#pragma unroll
        for (int u = 0; u < kHaloPer; ++u) hid_n[u] = hid_nn[u];
        request(tile + 1);
        load_ids(tile + 2, hid_nn);
        __syncthreads();
        Real y[4];
        mx_tile_op<P, Real, Ops>(*ops, F, pre, halo_pad + tile * hs, hmax, i0, ne, sd, se, y);
        // phase 3: q_k = -K d_k from the output registers, and the dot products
        const int64_t i = i0 + tq;
        if (i < ne) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = out_row<Real>(g, j);
                if (k < N) {
                    const Real qk = -y[j];
                    q_out[i * N + k] = qk;
                    const double dk = sd[tq * NS + k], rk = sr[tq * NS + k], qd = qk;
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
    constexpr int N = D::N, NE = D::NE, R1 = D::R1;
    const RefOps<P>& R = *static_cast<const RefOps<P>*>(refops);
    // E1 [R1][N]: rows (al, c, m) -> (al * 2 + c) * NE + m
    std::vector<double> E1((size_t)R1 * N, 0.0);
    for (int al = 0; al < 3; ++al)
        for (int c = 0; c < 2; ++c)
            for (int m = 0; m < NE; ++m)
                for (int l = 0; l < N; ++l) E1[(size_t)((al * 2 + c) * NE + m) * N + l] = R.E[al][c][m][l];
    // entry (row k, edge al, quantity s, edge node m) of W2's edge part: s = 0 the normal flux
    // of node m, which enters the line term on the edge's nodes (row edge_node(al, mm) takes
    // M1[mm][m]); s = 1, 2 the correction's reference components (Pt)
    auto w2e = [&](int k, int al, int s, int m) -> double {
        if (k >= N || m >= NE) return 0.0;
        if (s == 0) {
            for (int mm = 0; mm < NE; ++mm)
                if (edge_node(P, al, mm) == k) return R.M1[mm][m];
            return 0.0;
        }
        return R.Pt[al][s - 1][k][m];
    };
    // entry (row k, component c, node l) of the volume part
    auto w2v = [&](int k, int c, int l) -> double {
        return (k < N && c < 3 && l < N) ? R.S[c][k][l] : 0.0;
    };
    for (int rb = 0; rb < 2; ++rb)
        for (int ks = 0; ks < D::KS1; ++ks)
            for (int lane = 0; lane < 64; ++lane) {
                const int row = 16 * rb + (lane & 15), col = 4 * ks + (lane >> 4);
                out->a1[rb][ks][lane] = (row < R1 && col < N) ? E1[(size_t)row * N + col] : 0.0;
            }
    // F64 G2: edge k-step (al * 3 + s) * NQ + q holds node m = g + 4 q in lane group g; volume
    // k-step KSE + c * KS1 + u holds node l = 4 u + g of component c
    for (int lane = 0; lane < 64; ++lane) {
        const int k = lane & 15, g = lane >> 4;
        for (int ks = 0; ks < D::KSE; ++ks) {
            const int c9 = ks / D::NQ, q = ks % D::NQ;
            out->a2[ks][lane] = w2e(k, c9 / 3, c9 % 3, 4 * q + g);
        }
        for (int kv = 0; kv < D::KSV; ++kv) {
            const int c = kv / D::KS1, u = kv % D::KS1;
            out->a2[D::KSE + kv][lane] = w2v(k, c, 4 * u + g);
        }
    }
    for (int rb = 0; rb < 2; ++rb)
        for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 8; ++e) {
                const int row = 16 * rb + (lane & 15), col = 8 * (lane >> 4) + e;
                uint16_t sp[3];
                split3_host((row < R1 && col < N) ? E1[(size_t)row * N + col] : 0.0, sp);
                for (int s = 0; s < 3; ++s) out->b1[rb][s][lane][e] = sp[s];
            }
    // BF3 G2: edge k-step 2 q + h, element e of lane group g: (al * 3 + s) = 8 h + e at node
    // m = g + 4 q; volume k-step KSE32 + kv, element e of lane group g: component 2 kv + g / 2,
    // node 8 (g % 2) + e
    for (int lane = 0; lane < 64; ++lane) {
        const int k = lane & 15, g = lane >> 4;
        for (int e = 0; e < 8; ++e) {
            for (int ks = 0; ks < D::KSE32; ++ks) {
                const int q = ks >> 1, c9 = 8 * (ks & 1) + e;
                uint16_t sp[3];
                split3_host(c9 < 9 ? w2e(k, c9 / 3, c9 % 3, 4 * q + g) : 0.0, sp);
                for (int s = 0; s < 3; ++s) out->b2[ks][s][lane][e] = sp[s];
            }
            for (int kv = 0; kv < D::KSV32; ++kv) {
                uint16_t sp[3];
                split3_host(w2v(k, 2 * kv + (g >> 1), 8 * (g & 1) + e), sp);
                for (int s = 0; s < 3; ++s) out->b2[D::KSE32 + kv][s][lane][e] = sp[s];
            }
        }
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
                                                 m->geo_i, m->geo_nb, m->nbr_i, m->halo_pad, m->hmax,
                                                 m->ne, w.d32[1], w.q32[1]));
        hipLaunchKernelGGL(k_scatter_mx<float>, dim3(w.grid), dim3(kBlockFlat), 0, s, n, d->nphi,
                           m->perm, w.q32[1], static_cast<float*>(out));
    } else {
        hipLaunchKernelGGL(k_gather_mx<double>, dim3(w.grid), dim3(kBlockFlat), 0, s, n, d->nphi,
                           m->perm, static_cast<const double*>(p), w.d[1]);
        SLD_MX_DISPATCH(d->p, hipLaunchKernelGGL((k_apply_mx<PP, double, RefOps<PP>>), dim3(tiles),
                                                 dim3(kMxThreads), lds, s, ops64_of<PP>(d), tab_of<PP>(d),
                                                 m->geo_i, m->geo_nb, m->nbr_i, m->halo_pad, m->hmax,
                                                 m->ne, w.d[1], w.q[1]));
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
                                             tab_of<PP>(d), m->geo_i, m->geo_nb, m->nbr_i,          \
                                             m->halo_pad,                                           \
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
