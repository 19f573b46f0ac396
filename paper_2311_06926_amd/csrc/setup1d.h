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

// Basis values at the points of the quadrature-based operator (Sec. 5.3:
// Gauss-Legendre with p+1 points per element, plus the two end points where
// the Nitsche face terms of Sec. 3.3 are evaluated).  Point 0 is x = 0,
// point 1 + e (p+1) + g is Gauss point g of element e, point nq - 1 is x = 1.
// Dense row-major nq x n matrices: values and first derivatives of the
// interior degree-p functions (n = nN) and of the unit-integral degree p-1
// functions (n = nM); w holds the Gauss weights (1 at the two end points).
struct QuadTables1D {
    int nq = 0;
    std::vector<double> NV, ND, MV, MD, w;
};
QuadTables1D build_quad_tables(const Tables1D& T);
std::vector<double> sine_load(const Tables1D& T, int fam, int k);

}  // namespace hp
