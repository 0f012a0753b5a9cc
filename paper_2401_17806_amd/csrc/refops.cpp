// Host construction of the reference operators (Section 3.4) for degree P.
//
// Basis: equispaced Lagrange polynomials on T_ref written in product form over the
// integer barycentric coordinates (a, b, c = P-a-b) of their node,
//   phi_(a,b)(xi,eta) = L_a(P xi) L_b(P eta) L_c(P (1-xi-eta)),
//   L_m(t) = prod_{q<m} (t - q)/(q + 1),
// which equals 1 at its node and 0 at every other lattice node.  Integrals use a collapsed
// Gauss-Legendre rule (nodes from Newton's iteration on P_n) exact for every integrand here.
// All arithmetic is long double; results are rounded once to double.
#include "refops.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace {

typedef long double ld;

struct GL {
    std::vector<ld> x, w;  // on [0, 1]
};

GL gauss_legendre(int n) {
    GL g;
    g.x.resize(n);
    g.w.resize(n);
    const ld pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        ld z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
        ld dp = 0;
        for (int it = 0; it < 100; ++it) {
            ld p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                ld pk = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            if (n == 1) { p1 = z; p0 = 1; }
            dp = n * (z * p1 - p0) / (z * z - 1);
            ld dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-30L) break;
        }
        // recompute derivative at the converged root
        ld p0 = 1, p1 = z;
        for (int k = 2; k <= n; ++k) {
            ld pk = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        dp = n * (z * p1 - p0) / (z * z - 1);
        g.x[i] = 0.5L * (1 - z);
        g.w[i] = 1.0L / ((1 - z * z) * dp * dp);  // 2/((1-z^2)P'^2) scaled by 1/2
    }
    return g;
}

struct TriRule {
    std::vector<ld> u, v, w;  // sum w = 1/2
};

TriRule triangle_rule(int n) {
    GL g = gauss_legendre(n);
    TriRule r;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            ld s = g.x[i], t = g.x[j];
            r.u.push_back(s);
            r.v.push_back((1 - s) * t);
            r.w.push_back(g.w[i] * g.w[j] * (1 - s));
        }
    return r;
}

ld lag(int m, ld t) {
    ld r = 1;
    for (int q = 0; q < m; ++q) r *= (t - q) / (q + 1);
    return r;
}

ld dlag(int m, ld t) {
    ld s = 0;
    for (int skip = 0; skip < m; ++skip) {
        ld r = 1;
        for (int q = 0; q < m; ++q) r *= (q == skip ? ld(1) : (t - q)) / (q + 1);
        s += r;
    }
    return s;
}

template <int P>
struct Basis {
    static constexpr int N = RefOps<P>::NPHI;
    int na[N], nb[N];
    Basis() {
        int k = 0;
        for (int b = 0; b <= P; ++b)
            for (int a = 0; a <= P - b; ++a) { na[k] = a; nb[k] = b; ++k; }
    }
    void eval(ld xi, ld eta, ld* val, ld* dxi, ld* deta) const {
        ld l0 = 1 - xi - eta;
        for (int k = 0; k < N; ++k) {
            int a = na[k], b = nb[k], c = P - a - b;
            ld A = lag(a, P * xi), B = lag(b, P * eta), Cc = lag(c, P * l0);
            ld dA = P * dlag(a, P * xi), dB = P * dlag(b, P * eta), dC = -P * dlag(c, P * l0);
            if (val) val[k] = A * B * Cc;
            if (dxi) dxi[k] = dA * B * Cc + A * B * dC;
            if (deta) deta[k] = A * dB * Cc + A * B * dC;
        }
    }
};

// Solve A X = B (A n x n, B n x m) in place by Gaussian elimination with partial pivoting.
bool solve_dense(int n, int m, std::vector<ld>& A, std::vector<ld>& B) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0) return false;
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
            for (int k = 0; k < m; ++k) std::swap(B[c * m + k], B[piv * m + k]);
        }
        for (int r = c + 1; r < n; ++r) {
            ld f = A[r * n + c] / A[c * n + c];
            if (f == 0) continue;
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            for (int k = 0; k < m; ++k) B[r * m + k] -= f * B[c * m + k];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        for (int k = 0; k < m; ++k) {
            ld s = B[c * m + k];
            for (int j = c + 1; j < n; ++j) s -= A[c * n + j] * B[j * m + k];
            B[c * m + k] = s / A[c * n + c];
        }
    }
    return true;
}

const ld VX[3] = {0, 1, 0};
const ld VY[3] = {0, 0, 1};
const ld CX = 1.0L / 3, CY = 1.0L / 3;

}  // namespace

template <int P>
int build_refops(RefOps<P>* ops) {
    typedef RefOps<P> R;
    constexpr int N = R::NPHI, NE = R::NE, NI = R::NI;
    std::memset(ops, 0, sizeof(R));
    Basis<P> B;
    TriRule q = triangle_rule(P + 3);
    const int nq = (int)q.w.size();
    ld val[N], dx[N], dy[N], sv[N];

    // stiffness, mass, weights on T_ref
    std::vector<ld> S(3 * N * N, 0), M(N * N, 0), w(N, 0);
    for (int iq = 0; iq < nq; ++iq) {
        B.eval(q.u[iq], q.v[iq], val, dx, dy);
        ld wq = q.w[iq];
        for (int k = 0; k < N; ++k) {
            w[k] += wq * val[k];
            for (int l = 0; l < N; ++l) {
                S[0 * N * N + k * N + l] += wq * dx[k] * dx[l];
                S[1 * N * N + k * N + l] += wq * (dx[k] * dy[l] + dy[k] * dx[l]);
                S[2 * N * N + k * N + l] += wq * dy[k] * dy[l];
                M[k * N + l] += wq * val[k] * val[l];
            }
        }
    }
    for (int t = 0; t < 3; ++t)
        for (int k = 0; k < N; ++k)
            for (int l = 0; l < N; ++l) ops->S[t][k][l] = (double)S[t * N * N + k * N + l];
    for (int k = 0; k < N; ++k) ops->w[k] = (double)w[k];
    for (int k = 0; k < N; ++k)
        for (int l = 0; l < N; ++l) ops->Mref[k][l] = (double)M[k * N + l];

    // interior / edge split of a sub-triangle's nodes
    int Iidx[N > 0 ? N : 1], Hidx[NE];
    {
        int ni = 0;
        for (int k = 0; k < N; ++k)
            if (B.na[k] + B.nb[k] < P) Iidx[ni++] = k;
        if (ni != NI) return 1;
        for (int m = 0; m < NE; ++m) Hidx[m] = main_idx(P, P - m, m);
    }
    // Z = M_II^{-1} M_IH
    std::vector<ld> Zl(NI * NE, 0);
    if (NI > 0) {
        std::vector<ld> A(NI * NI), Bm(NI * NE);
        for (int i = 0; i < NI; ++i) {
            for (int j = 0; j < NI; ++j) A[i * NI + j] = M[Iidx[i] * N + Iidx[j]];
            for (int m = 0; m < NE; ++m) Bm[i * NE + m] = M[Iidx[i] * N + Hidx[m]];
        }
        if (!solve_dense(NI, NE, A, Bm)) return 2;
        Zl = Bm;
        for (int i = 0; i < NI; ++i)
            for (int m = 0; m < NE; ++m) ops->Z[i][m] = (double)Zl[i * NE + m];
    }
    // S0 = M_HH - M_HI Z ; M1 ; C = S0^{-1} M1
    std::vector<ld> S0(NE * NE), M1(NE * NE, 0);
    for (int m = 0; m < NE; ++m)
        for (int n = 0; n < NE; ++n) {
            ld s = M[Hidx[m] * N + Hidx[n]];
            for (int i = 0; i < NI; ++i) s -= M[Hidx[m] * N + Iidx[i]] * Zl[i * NE + n];
            S0[m * NE + n] = s;
        }
    {
        GL g = gauss_legendre(P + 2);
        for (size_t iq = 0; iq < g.x.size(); ++iq) {
            ld t = g.x[iq];
            ld lv[NE];
            for (int m = 0; m < NE; ++m) {
                ld r = 1;
                for (int qn = 0; qn < NE; ++qn)
                    if (qn != m) r *= (P * t - qn) / ld(m - qn);
                lv[m] = r;
            }
            for (int m = 0; m < NE; ++m)
                for (int n = 0; n < NE; ++n) M1[m * NE + n] += g.w[iq] * lv[m] * lv[n];
        }
        std::vector<ld> A = S0, Bm = M1;
        if (!solve_dense(NE, NE, A, Bm)) return 3;
        for (int m = 0; m < NE; ++m)
            for (int n = 0; n < NE; ++n) {
                ops->C[m][n] = (double)Bm[m * NE + n];
                ops->M1[m][n] = (double)M1[m * NE + n];
            }
    }

    for (int al = 0; al < 3; ++al) {
        const int a1 = (al + 1) % 3;
        // derivatives at edge nodes
        for (int m = 0; m < NE; ++m) {
            ld t = ld(m) / P;
            ld xi = VX[al] + t * (VX[a1] - VX[al]);
            ld eta = VY[al] + t * (VY[a1] - VY[al]);
            B.eval(xi, eta, nullptr, dx, dy);
            for (int l = 0; l < N; ++l) {
                ops->E[al][0][m][l] = (double)dx[l];
                ops->E[al][1][m][l] = (double)dy[l];
            }
        }
        // sub-triangle map zeta -> xi
        auto map = [&](ld z1, ld z2, ld& xi, ld& eta) {
            xi = CX + z1 * (VX[al] - CX) + z2 * (VX[a1] - CX);
            eta = CY + z1 * (VY[al] - CY) + z2 * (VY[a1] - CY);
        };
        for (int n = 0; n < N; ++n) {
            ld xi, eta;
            map(ld(B.na[n]) / P, ld(B.nb[n]) / P, xi, eta);
            B.eval(xi, eta, val, dx, dy);
            for (int l = 0; l < N; ++l) {
                ops->Hn[al][0][n][l] = (double)dx[l];
                ops->Hn[al][1][n][l] = (double)dy[l];
                if (al == 0) ops->Iv[n][l] = (double)val[l];
            }
        }
        std::vector<ld> Wl(2 * N * N, 0), Sh(3 * N * N, 0), V(N * N, 0);
        const ld jac = 1.0L / 3;  // |det d xi / d zeta|
        for (int iq = 0; iq < nq; ++iq) {
            ld xi, eta;
            map(q.u[iq], q.v[iq], xi, eta);
            B.eval(xi, eta, val, dx, dy);
            B.eval(q.u[iq], q.v[iq], sv, nullptr, nullptr);
            ld wq = q.w[iq] * jac;
            for (int k = 0; k < N; ++k)
                for (int n = 0; n < N; ++n) {
                    V[k * N + n] += wq * val[k] * sv[n];
                    Wl[0 * N * N + k * N + n] += wq * dx[k] * sv[n];
                    Wl[1 * N * N + k * N + n] += wq * dy[k] * sv[n];
                    Sh[0 * N * N + k * N + n] += wq * dx[k] * dx[n];
                    Sh[1 * N * N + k * N + n] += wq * (dx[k] * dy[n] + dy[k] * dx[n]);
                    Sh[2 * N * N + k * N + n] += wq * dy[k] * dy[n];
                }
        }
        for (int d = 0; d < 2; ++d)
            for (int k = 0; k < N; ++k) {
                for (int n = 0; n < N; ++n) ops->W[al][d][k][n] = (double)Wl[d * N * N + k * N + n];
                for (int m = 0; m < NE; ++m) {
                    ld s = Wl[d * N * N + k * N + Hidx[m]];
                    for (int i = 0; i < NI; ++i) s -= Wl[d * N * N + k * N + Iidx[i]] * Zl[i * NE + m];
                    ops->Pt[al][d][k][m] = (double)s;
                }
            }
        for (int t = 0; t < 3; ++t)
            for (int k = 0; k < N; ++k)
                for (int n = 0; n < N; ++n) ops->Sh[al][t][k][n] = (double)Sh[t * N * N + k * N + n];
        // Ldm[al] = Mref^{-1} V_al
        std::vector<ld> Mc = M;
        if (!solve_dense(N, N, Mc, V)) return 4;
        for (int k = 0; k < N; ++k)
            for (int n = 0; n < N; ++n) ops->Ldm[al][k][n] = (double)V[k * N + n];
    }
    return 0;
}

template int build_refops<1>(RefOps<1>*);
template int build_refops<2>(RefOps<2>*);
template int build_refops<3>(RefOps<3>*);
template int build_refops<4>(RefOps<4>*);

template <int P>
int build_slops(SlOps<P>* ops) {
    constexpr int N = SlOps<P>::NPHI, NG = SlOps<P>::NG;
    const TriRule r = triangle_rule(P + 1);
    const Basis<P> B;
    std::vector<ld> phi(size_t(NG) * N);
    for (int g = 0; g < NG; ++g) B.eval(r.u[g], r.v[g], &phi[size_t(g) * N], nullptr, nullptr);
    // M_ref = Phi^T W Phi (exact: the integrand has degree 2P); rhs = Phi^T W
    std::vector<ld> M(size_t(N) * N, 0), R(size_t(N) * NG, 0);
    for (int g = 0; g < NG; ++g)
        for (int k = 0; k < N; ++k) {
            R[size_t(k) * NG + g] = r.w[g] * phi[size_t(g) * N + k];
            for (int l = 0; l < N; ++l)
                M[size_t(k) * N + l] += r.w[g] * phi[size_t(g) * N + k] * phi[size_t(g) * N + l];
        }
    if (!solve_dense(N, NG, M, R)) return 1;
    for (int g = 0; g < NG; ++g) {
        ops->pts[g][0] = (double)r.u[g];
        ops->pts[g][1] = (double)r.v[g];
    }
    for (int k = 0; k < N; ++k)
        for (int g = 0; g < NG; ++g) ops->proj[k][g] = (double)R[size_t(k) * NG + g];
    return 0;
}

template int build_slops<1>(SlOps<1>*);
template int build_slops<2>(SlOps<2>*);
template int build_slops<3>(SlOps<3>*);
template int build_slops<4>(SlOps<4>*);
