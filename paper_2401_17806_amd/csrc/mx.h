// Element-batched reference contractions on the matrix cores (MFMA), shared by the host table
// builder and the kernels.
//
// Every triangle's operator is the same reference matrices times its own geometry (Section
// 3.4.1: the "standard operators" of the reference element), so the reference products of a
// tile of triangles are two matrix products with the tile's triangles as columns:
//   G1: the reference derivatives of d at the edge nodes of all three edges,
//       E1 [6 NE x N] * [d_t ...]            rows (alpha, c, m) -> (alpha * 2 + c) * NE + m,
//   G2: the rows of (K d)_t from the per-triangle quantities z_t formed between the two,
//       W2 [N x K2] * [z_t ...],
//       z = (per edge alpha and edge node: the normal flux n.x_H, -A (G Delta)_0,
//            -A (G Delta)_1), then -A m00 d, -A m01 d, -A m11 d (volume term)
//       W2 = (per edge alpha: M1 placed on the edge's nodes, Pt[alpha][0], Pt[alpha][1]),
//            then S0, S1, S2 (the k-step order of the edge part is given in MxDims).
// Between the two products only pointwise work per edge node remains (the closed form of
// Mhat^{-1} on the edge nodes, which couples each edge's two sides).
//
// Two engines:
//   F64:  v_mfma_f64_16x16x4f64, 16 x 16 output blocks, k-steps of 4.
//   BF3:  v_mfma_f32_16x16x32_bf16 with each FP32 operand split into three bfloat16 terms
//         (hi + mid + lo carry 24 bits), the six products whose weight exceeds 2^-24 taken
//         (hi hi, hi mid, mid hi, hi lo, mid mid, lo hi) and accumulated in FP32: an FP32
//         contraction on the BF16 matrix cores.
// Lane layouts (one wave of 64 lanes, i = lane, g = i / 16):
//   F64  A[r][k]: lane r + 16 k (k < 4);      B[k][c]: lane c + 16 k;
//        D[r][c]: lane c + 16 (r % 4), element r / 4;
//   BF3  A[r][k]: lane r + 16 (k / 8), element k % 8 (k < 32); B[k][c] likewise;
//        D[r][c]: lane c + 16 (r / 4), element r % 4
// (measured on gfx950 with one-hot operands).
#pragma once

#include <cstdint>

template <int P>
struct MxDims {
    static constexpr int N = (P + 1) * (P + 2) / 2;  // main DOFs
    static constexpr int NE = P + 1;                 // nodes on an edge
    static constexpr int R1 = 6 * NE;                // rows of G1 (<= 32: two row blocks)
    static constexpr int KE = 9 * NE;                // edge part of G2's inner dimension
    // the nodes of an edge are dealt to the four lane groups of a 16-triangle block: node
    // m = g + 4 q to lane group g (q < NQ)
    static constexpr int NQ = (NE + 3) / 4;
    // F64: k-steps of 4; the edge part of G2 takes k-step (al * 3 + s) * NQ + q at node
    // m = g + 4 q (s: 0 the normal flux, 1 and 2 the two reference components of the correction)
    static constexpr int KS1 = (N + 3) / 4;
    static constexpr int KSE = 9 * NQ;
    static constexpr int NV = KS1 * 4;               // stride of one volume component
    static constexpr int KSV = 3 * KS1;
    static constexpr int KS2 = KSE + KSV;
    // BF3: k-steps of 32 (G1 needs one: N <= 15 < 32); the edge part of G2 takes k-step
    // 2 q + h, element e of lane group g being (al * 3 + s) = 8 h + e at node m = g + 4 q
    static constexpr int KSE32 = 2 * NQ;
    static constexpr int KSV32 = 2;                  // three volume components of 16
    static constexpr int KS232 = KSE32 + KSV32;
    // LDS row strides (words) of the per-triangle arrays: odd, so that lanes reading the same
    // entry of consecutive triangles fall in different banks
    static constexpr int NS = N | 1;
    static constexpr int R1S = R1 | 1;
};

// A operands of both engines, in lane order (each lane loads its own entries).
template <int P>
struct MxTab {
    using D = MxDims<P>;
    double a1[2][D::KS1][64];        // F64 G1: [row block][k-step][lane]
    double a2[D::KS2][64];           // F64 G2: [k-step][lane]
    uint16_t b1[2][3][64][8];        // BF3 G1: [row block][term hi/mid/lo][lane][element]
    uint16_t b2[D::KS232][3][64][8]; // BF3 G2: [k-step][term][lane][element]
};

// Fill the tables from the reference operators (refops.h).  Returns 0 on success.
template <int P>
int build_mxtab(const void* refops /* RefOps<P> */, MxTab<P>* out);
