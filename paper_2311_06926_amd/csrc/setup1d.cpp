// Host-side univariate set-up: B-spline bases, the univariate matrices of
// App. B.3 / Sec. 3.3, and the generalised eigen-decompositions used by
// fast diagonalisation (App. A.3-A.4).  All O(n^3) with n <= E+p, run once.
#include "setup1d.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace hp {

// ---------------------------------------------------------------------------
// Gauss--Legendre rule on [-1, 1] by Newton iteration on P_n.
// ---------------------------------------------------------------------------
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute derivative at the converged root for the weight
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        if (n == 1) { p1 = z; p0 = 1.0; }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// ---------------------------------------------------------------------------
// B-spline evaluation: the degree-d functions that are non-zero on the knot
// span `s` (t[s] <= x < t[s+1]) and their first derivatives, by the
// triangular Cox--de Boor table; derivatives from the degree d-1 values.
// vals[j], ders[j] belong to function s-d+j.
// ---------------------------------------------------------------------------
static void span_basis(const std::vector<double>& t, int d, int s, double x,
                       std::vector<double>& vals, std::vector<double>& ders) {
    std::vector<std::vector<double>> tab(d + 1);
    tab[0] = {1.0};
    for (int deg = 1; deg <= d; ++deg) {
        std::vector<double> nv(deg + 1, 0.0);
        // functions s-deg .. s of degree deg
        for (int j = 0; j <= deg; ++j) {
            int i = s - deg + j;
            double v = 0.0;
            // left term uses N_{i,deg-1}, index j-1 in tab[deg-1] (functions s-deg+1..s)
            if (j >= 1) {
                double den = t[i + deg] - t[i];
                if (den > 0) v += (x - t[i]) / den * tab[deg - 1][j - 1];
            }
            if (j <= deg - 1) {
                double den = t[i + deg + 1] - t[i + 1];
                if (den > 0) v += (t[i + deg + 1] - x) / den * tab[deg - 1][j];
            }
            nv[j] = v;
        }
        tab[deg] = nv;
    }
    vals = tab[d];
    ders.assign(d + 1, 0.0);
    if (d == 0) return;
    for (int j = 0; j <= d; ++j) {
        int i = s - d + j;
        double v = 0.0;
        if (j >= 1) {
            double den = t[i + d] - t[i];
            if (den > 0) v += d / den * tab[d - 1][j - 1];
        }
        if (j <= d - 1) {
            double den = t[i + d + 1] - t[i + 1];
            if (den > 0) v -= d / den * tab[d - 1][j];
        }
        ders[j] = v;
    }
}

// knot span index for x in [0, 1] (x == 1 goes to the last non-empty span)
static int find_span(const std::vector<double>& t, int d, double x) {
    int m = (int)t.size() - 1;
    int last = m - d - 1;  // last span with non-zero length for open knots
    if (x >= t[last + 1]) return last;
    int s = d;
    while (s < last && !(x >= t[s] && x < t[s + 1])) ++s;
    return s;
}

// Evaluate all n functions (degree d on knots t) and derivatives at x.
static void eval_all(const std::vector<double>& t, int d, double x, std::vector<double>& v,
                     std::vector<double>& dv) {
    int n = (int)t.size() - d - 1;
    v.assign(n, 0.0);
    dv.assign(n, 0.0);
    int s = find_span(t, d, x);
    std::vector<double> a, b;
    span_basis(t, d, s, x, a, b);
    for (int j = 0; j <= d; ++j) {
        int i = s - d + j;
        if (i >= 0 && i < n) {
            v[i] = a[j];
            dv[i] = b[j];
        }
    }
}

// ---------------------------------------------------------------------------
// Dense linear algebra helpers (row-major n x n).
// ---------------------------------------------------------------------------
static void cholesky(std::vector<double>& A, int n) {  // in place, lower
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (s <= 0) throw std::runtime_error("cholesky: matrix not positive definite");
        double l = std::sqrt(s);
        A[j * n + j] = l;
        for (int i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int k = 0; k < j; ++k) v -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = v / l;
        }
        for (int k = j + 1; k < n; ++k) A[j * n + k] = 0.0;
    }
}

// cyclic Jacobi eigen-decomposition of a symmetric matrix: A = Q diag(lam) Q^T
static void jacobi_eig(std::vector<double> A, int n, std::vector<double>& lam,
                       std::vector<double>& Q) {
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                (i == j ? diag : off) += A[i * n + j] * A[i * n + j];
        if (off <= 1e-30 * diag) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                double app = A[p * n + p], aqq = A[q * n + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) /
                           (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // rotate columns p, q
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rotate rows p, q
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double qkp = Q[k * n + p], qkq = Q[k * n + q];
                    Q[k * n + p] = c * qkp - s * qkq;
                    Q[k * n + q] = s * qkp + c * qkq;
                }
            }
        }
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
}

// Generalised symmetric-definite problem K u = lam M u with U^T M U = I,
// via M = L L^T, C = L^{-1} K L^{-T} = Q Lam Q^T, U = L^{-T} Q (App. A.3).
void generalized_eig(const std::vector<double>& K, const std::vector<double>& M, int n,
                     std::vector<double>& lam, std::vector<double>& U) {
    std::vector<double> L = M;
    cholesky(L, n);
    // C = L^{-1} K L^{-T}: first W = L^{-1} K (forward substitution on columns)
    std::vector<double> W = K;
    for (int col = 0; col < n; ++col)
        for (int i = 0; i < n; ++i) {
            double v = W[i * n + col];
            for (int k = 0; k < i; ++k) v -= L[i * n + k] * W[k * n + col];
            W[i * n + col] = v / L[i * n + i];
        }
    // C = W L^{-T} = (L^{-1} W^T)^T
    std::vector<double> C((size_t)n * n);
    for (int row = 0; row < n; ++row)
        for (int i = 0; i < n; ++i) {
            double v = W[row * n + i];
            for (int k = 0; k < i; ++k) v -= L[i * n + k] * C[row * n + k];
            C[row * n + i] = v / L[i * n + i];
        }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double s = 0.5 * (C[i * n + j] + C[j * n + i]);
            C[i * n + j] = C[j * n + i] = s;
        }
    std::vector<double> Q;
    jacobi_eig(C, n, lam, Q);
    // sort ascending
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return lam[a] < lam[b]; });
    std::vector<double> lam2(n), Q2((size_t)n * n);
    for (int j = 0; j < n; ++j) {
        lam2[j] = lam[idx[j]];
        for (int i = 0; i < n; ++i) Q2[i * n + j] = Q[i * n + idx[j]];
    }
    lam = lam2;
    // U = L^{-T} Q: back substitution with L^T
    U.assign((size_t)n * n, 0.0);
    for (int col = 0; col < n; ++col)
        for (int i = n - 1; i >= 0; --i) {
            double v = Q2[i * n + col];
            for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * U[k * n + col];
            U[i * n + col] = v / L[i * n + i];
        }
}

void inverse_spd(const std::vector<double>& M, int n, std::vector<double>& Minv) {
    std::vector<double> L = M;
    cholesky(L, n);
    Minv.assign((size_t)n * n, 0.0);
    std::vector<double> y(n);
    for (int col = 0; col < n; ++col) {
        for (int i = 0; i < n; ++i) {
            double v = (i == col) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= L[i * n + k] * y[k];
            y[i] = v / L[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double v = y[i];
            for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * Minv[k * n + col];
            Minv[i * n + col] = v / L[i * n + i];
        }
    }
}

// ---------------------------------------------------------------------------
// Univariate tables
// ---------------------------------------------------------------------------
Tables1D build_tables(int E, int p, double c_pen) {
    if (E < 1 || p < 2) throw std::runtime_error("need E >= 1 and p >= 2");
    Tables1D T;
    T.E = E;
    T.p = p;
    T.n = E + p;
    T.nN = E + p - 2;
    T.nM = E + p - 1;
    T.h = 1.0 / E;
    T.alpha = c_pen / T.h;
    const int n = T.n, nm = T.nM;
    // knots: degree p open knots; degree p-1 functions on the same breakpoints
    std::vector<double> tp(n + p + 1), tm;
    for (int i = 0; i <= p; ++i) tp[i] = 0.0;
    for (int i = 1; i < E; ++i) tp[p + i] = (double)i / E;
    for (int i = 0; i <= p; ++i) tp[n + i] = 1.0;
    tm.assign(tp.begin() + 1, tp.end() - 1);
    // scale of the unit-integral M-splines: int N_{i,p-1} = (t_{i+p} - t_i) / p
    std::vector<double> mscale(nm);
    for (int i = 0; i < nm; ++i) mscale[i] = p / (tm[i + p] - tm[i]);

    std::vector<double> Mfull((size_t)n * n, 0.0), Kfull((size_t)n * n, 0.0);
    std::vector<double> Mc((size_t)nm * nm, 0.0), Kc((size_t)nm * nm, 0.0);
    std::vector<double> intN(n, 0.0), intM(nm, 0.0);
    std::vector<double> gx, gw;
    gauss_legendre(p + 1, gx, gw);
    std::vector<double> Nv, dNv, Mv, dMv;
    for (int e = 0; e < E; ++e) {
        double a = (double)e / E, b = (double)(e + 1) / E;
        for (size_t q = 0; q < gx.size(); ++q) {
            double x = 0.5 * (b - a) * gx[q] + 0.5 * (a + b);
            double w = 0.5 * (b - a) * gw[q];
            eval_all(tp, p, x, Nv, dNv);
            eval_all(tm, p - 1, x, Mv, dMv);
            for (int i = 0; i < nm; ++i) {
                Mv[i] *= mscale[i];
                dMv[i] *= mscale[i];
            }
            for (int i = 0; i < n; ++i) {
                if (Nv[i] == 0.0 && dNv[i] == 0.0) continue;
                intN[i] += w * Nv[i];
                for (int j = 0; j < n; ++j) {
                    Mfull[i * n + j] += w * Nv[i] * Nv[j];
                    Kfull[i * n + j] += w * dNv[i] * dNv[j];
                }
            }
            for (int i = 0; i < nm; ++i) {
                if (Mv[i] == 0.0 && dMv[i] == 0.0) continue;
                intM[i] += w * Mv[i];
                for (int j = 0; j < nm; ++j) {
                    Mc[i * nm + j] += w * Mv[i] * Mv[j];
                    Kc[i * nm + j] += w * dMv[i] * dMv[j];
                }
            }
        }
    }
    // boundary values of M and M' at 0 and 1
    std::vector<double> M0, dM0, M1, dM1;
    eval_all(tm, p - 1, 0.0, M0, dM0);
    eval_all(tm, p - 1, 1.0, M1, dM1);
    for (int i = 0; i < nm; ++i) {
        M0[i] *= mscale[i];
        dM0[i] *= mscale[i];
        M1[i] *= mscale[i];
        dM1[i] *= mscale[i];
    }
    // T^ = 1/2 (K^ + 2 alpha N^ - B^ - B^^T)   (Sec. 3.3)
    std::vector<double> Tc((size_t)nm * nm);
    for (int i = 0; i < nm; ++i)
        for (int j = 0; j < nm; ++j) {
            double Nc = M1[i] * M1[j] + M0[i] * M0[j];
            double Bij = M1[i] * dM1[j] - M0[i] * dM0[j];
            double Bji = M1[j] * dM1[i] - M0[j] * dM0[i];
            Tc[i * nm + j] = 0.5 * (Kc[i * nm + j] + 2.0 * T.alpha * Nc - Bij - Bji);
        }
    // interior degree-p functions (v.n = 0 strongly): indices 1..n-2
    const int nN = T.nN;
    T.M_int.resize((size_t)nN * nN);
    T.K_int.resize((size_t)nN * nN);
    for (int i = 0; i < nN; ++i)
        for (int j = 0; j < nN; ++j) {
            T.M_int[i * nN + j] = Mfull[(i + 1) * n + (j + 1)];
            T.K_int[i * nN + j] = Kfull[(i + 1) * n + (j + 1)];
        }
    T.Mc = Mc;
    T.Tc = Tc;
    T.int_N.assign(intN.begin() + 1, intN.end() - 1);
    T.int_M = intM;
    T.lid3.resize(nm);
    for (int i = 0; i < nm; ++i) T.lid3[i] = T.alpha * M1[i] - 0.5 * dM1[i];
    generalized_eig(T.K_int, T.M_int, nN, T.lamK, T.UK);
    generalized_eig(T.Tc, T.Mc, nm, T.lamT, T.UT);
    inverse_spd(T.Mc, nm, T.Mcinv);
    T.tp = tp;
    T.tm = tm;
    T.mscale = mscale;
    return T;
}

QuadTables1D build_quad_tables(const Tables1D& T) {
    const int E = T.E, p = T.p, nN = T.nN, nM = T.nM, n = T.n;
    QuadTables1D Q;
    Q.nq = E * (p + 1) + 2;
    const int nq = Q.nq;
    Q.NV.assign((size_t)nq * nN, 0.0);
    Q.ND.assign((size_t)nq * nN, 0.0);
    Q.MV.assign((size_t)nq * nM, 0.0);
    Q.MD.assign((size_t)nq * nM, 0.0);
    Q.w.assign(nq, 1.0);
    std::vector<double> gx, gw, Nv, dNv, Mv, dMv;
    gauss_legendre(p + 1, gx, gw);
    auto fill = [&](int r, double x) {
        eval_all(T.tp, p, x, Nv, dNv);
        eval_all(T.tm, p - 1, x, Mv, dMv);
        for (int i = 0; i < nN; ++i) {  // interior functions: full indices 1 .. n-2
            Q.NV[(size_t)r * nN + i] = Nv[i + 1];
            Q.ND[(size_t)r * nN + i] = dNv[i + 1];
        }
        for (int i = 0; i < nM; ++i) {
            Q.MV[(size_t)r * nM + i] = Mv[i] * T.mscale[i];
            Q.MD[(size_t)r * nM + i] = dMv[i] * T.mscale[i];
        }
    };
    (void)n;
    fill(0, 0.0);
    for (int e = 0; e < E; ++e) {
        double a = (double)e / E, b = (double)(e + 1) / E;
        for (int g = 0; g <= p; ++g) {
            const int r = 1 + e * (p + 1) + g;
            fill(r, 0.5 * (b - a) * gx[g] + 0.5 * (a + b));
            Q.w[r] = 0.5 * (b - a) * gw[g];
        }
    }
    fill(nq - 1, 1.0);
    return Q;
}

// Load vector of the separable mode sin(pi k x) against the interior degree-p
// functions (fam = 0) or all M-splines (fam = 1), by Gauss quadrature with
// p + 8 points per element.
std::vector<double> sine_load(const Tables1D& T, int fam, int k) {
    const double pi = 3.14159265358979323846;
    int p = T.p, E = T.E;
    int cnt = fam == 0 ? T.nN : T.nM;
    std::vector<double> out(cnt, 0.0);
    std::vector<double> gx, gw, v, dv;
    gauss_legendre(p + 8, gx, gw);
    for (int e = 0; e < E; ++e) {
        double a = (double)e / E, b = (double)(e + 1) / E;
        for (size_t q = 0; q < gx.size(); ++q) {
            double x = 0.5 * (b - a) * gx[q] + 0.5 * (a + b);
            double w = 0.5 * (b - a) * gw[q] * std::sin(pi * k * x);
            if (fam == 0) {
                eval_all(T.tp, p, x, v, dv);
                for (int i = 0; i < cnt; ++i) out[i] += w * v[i + 1];
            } else {
                eval_all(T.tm, p - 1, x, v, dv);
                for (int i = 0; i < cnt; ++i) out[i] += w * v[i] * T.mscale[i];
            }
        }
    }
    return out;
}

}  // namespace hp
