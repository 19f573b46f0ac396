// Host-side univariate tables (App. B.3, Sec. 3.3) and fast-diagonalisation
// eigenpairs (App. A.3-A.4).  Row-major dense matrices.
#pragma once
#include <vector>

namespace hp {

struct Tables1D {
    int E = 0, p = 0, n = 0, nN = 0, nM = 0;
    double h = 0, alpha = 0;
    // interior degree-p mass / stiffness (nN x nN)
    std::vector<double> M_int, K_int;
    // degree p-1 (unit-integral M-spline) mass and the Nitsche-augmented T^ (nM x nM)
    std::vector<double> Mc, Tc, Mcinv;
    // generalised eigenpairs: K_int U = M_int U diag(lamK), Tc U = Mc U diag(lamT)
    std::vector<double> lamK, UK, lamT, UT;
    // lid right-hand side pieces: int N_i (interior), int M_i, alpha M_i(1) - M_i'(1)/2
    std::vector<double> int_N, int_M, lid3;
    // knots and M-spline scales (for load vectors)
    std::vector<double> tp, tm, mscale;
};

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
void generalized_eig(const std::vector<double>& K, const std::vector<double>& M, int n,
                     std::vector<double>& lam, std::vector<double>& U);
void inverse_spd(const std::vector<double>& M, int n, std::vector<double>& Minv);
Tables1D build_tables(int E, int p, double c_pen);
std::vector<double> sine_load(const Tables1D& T, int fam, int k);

}  // namespace hp
