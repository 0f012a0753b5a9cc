// Reference operators of degree P on the reference triangle (Section 3.4), in the
// triangle-centred form the kernels use.  Filled on the host in float64 by exact Gauss
// quadrature (refops.cpp), copied once to the device.
//
// Notation (reference triangle T_ref with vertices v0=(0,0), v1=(1,0), v2=(0,1), centroid c):
//   local edge alpha runs v_alpha -> v_{alpha+1}; its p+1 Lagrange nodes are numbered
//   m = 0..p from v_alpha.  The sub-triangle T^alpha = (c, v_alpha, v_{alpha+1}) is the image
//   of a triangle's half of the dual cell of edge alpha; its local coordinates zeta put
//   (0,0) at c, (1,0) at v_alpha, (0,1) at v_{alpha+1}, and its Lagrange nodes (a,b) use the
//   main numbering.  Nodes with a+b = p ("H", on the edge) are numbered by m = b; the others
//   are the interior set "I".
#pragma once

template <int P>
struct RefOps {
    static constexpr int NPHI = (P + 1) * (P + 2) / 2;
    static constexpr int NE = P + 1;          // nodes on one edge
    static constexpr int NI = NPHI - NE;      // sub-triangle nodes off the edge
    // int_{T_ref} d_d phi_k d_e phi_l: [0] = (xi,xi), [1] = (xi,eta)+(eta,xi), [2] = (eta,eta)
    double S[3][NPHI][NPHI];
    // the same integrals restricted to sub-triangle T^alpha (wall edges)
    double Sh[3][3][NPHI][NPHI];
    // E[alpha][d][m][l] = d_d phi_l at edge node m of edge alpha
    double E[3][2][NE][NPHI];
    // Pt[alpha][d][k][m] = int_{T^alpha} d_d phi_k chi_m, chi_m = sub-triangle polynomial equal
    // to 1 at edge node m, 0 at the other edge nodes and -Z[:,m] at the interior nodes
    double Pt[3][2][NPHI][NE];
    // Hn[alpha][d][n][l] = d_d phi_l at sub-triangle node n (main numbering in zeta) of T^alpha
    double Hn[3][2][NPHI][NPHI];
    // W[alpha][d][k][n] = int_{T^alpha} d_d phi_k phi_n(zeta)  (phi_n: sub-triangle Lagrange basis)
    double W[3][2][NPHI][NPHI];
    // Z = M_II^{-1} M_IH (sub-triangle mass matrix blocks), I in main order, H by m
    double Z[NI > 0 ? NI : 1][NE];
    // C = S0^{-1} M1, S0 = M_HH - M_HI Z (interface Schur complement), M1 = 1D edge mass
    double C[NE][NE];
    double M1[NE][NE];
    // int_{T_ref} phi_k
    double w[NPHI];
    // Tables of the grid transfers and the viscous operator (Section 4):
    // Mref = int_{T_ref} phi_k phi_l (the main mass matrix of triangle i is A_i Mref)
    double Mref[NPHI][NPHI];
    // Iv[n][l] = phi_l at sub-triangle node n (main numbering in zeta) of T^0
    double Iv[NPHI][NPHI];
    // Ldm[alpha][l][n] = (Mref^{-1} V_alpha)[l][n], V_alpha[k][n] = int_{T^alpha} phi_k phi_n(zeta):
    // the dual -> main projection of one triangle is sum_alpha Ldm[alpha] (its half of cell alpha)
    double Ldm[3][NPHI][NPHI];
};

// Float copy of the operators the Schur apply uses (mixed-precision inner solves).
template <int P>
struct RefOps32 {
    static constexpr int NPHI = RefOps<P>::NPHI;
    static constexpr int NE = P + 1;
    float S[3][NPHI][NPHI];
    float Sh[3][3][NPHI][NPHI];
    float E[3][2][NE][NPHI];
    float Pt[3][2][NPHI][NE];
    float C[NE][NE];
    float M1[NE][NE];
};

template <int P>
void round_refops(const RefOps<P>& in, RefOps32<P>* out) {
    constexpr int N = RefOps<P>::NPHI, NE = P + 1;
    for (int t = 0; t < 3; ++t)
        for (int k = 0; k < N; ++k)
            for (int l = 0; l < N; ++l) {
                out->S[t][k][l] = (float)in.S[t][k][l];
                for (int a = 0; a < 3; ++a) out->Sh[a][t][k][l] = (float)in.Sh[a][t][k][l];
            }
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 2; ++d) {
            for (int m = 0; m < NE; ++m)
                for (int l = 0; l < N; ++l) out->E[a][d][m][l] = (float)in.E[a][d][m][l];
            for (int k = 0; k < N; ++k)
                for (int m = 0; m < NE; ++m) out->Pt[a][d][k][m] = (float)in.Pt[a][d][k][m];
        }
    for (int m = 0; m < NE; ++m)
        for (int q = 0; q < NE; ++q) {
            out->C[m][q] = (float)in.C[m][q];
            out->M1[m][q] = (float)in.M1[m][q];
        }
}

// Semi-Lagrangian projection data (Section 3.5): the Gauss rule on T_ref (collapsed
// Gauss-Legendre, P + 1 points per direction, exact for the degree-2P projection integrand)
// and proj = M_ref^{-1} Phi^T diag(w), so that the projected coefficients of a field known at
// the Gauss points are proj * values.
template <int P>
struct SlOps {
    static constexpr int NPHI = (P + 1) * (P + 2) / 2;
    static constexpr int NG = (P + 1) * (P + 1);
    double pts[NG][2];
    double proj[NPHI][NG];
};

template <int P>
int build_slops(SlOps<P>* ops);

// Fill ops for degree P (1..4).  Returns 0 on success.
template <int P>
int build_refops(RefOps<P>* ops);

// Main node index of lattice node (a, b), b outer / a inner.
constexpr int main_idx(int P, int a, int b) { return b * (P + 1) - (b * (b - 1)) / 2 + a; }
// Main index of node m (0..P) on local edge alpha, counted from v_alpha.
constexpr int edge_node(int P, int alpha, int m) {
    return alpha == 0 ? main_idx(P, m, 0) : (alpha == 1 ? main_idx(P, P - m, m) : main_idx(P, 0, P - m));
}
