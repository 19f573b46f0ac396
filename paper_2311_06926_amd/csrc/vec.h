// Vector-kernel launchers (krylov.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace hp {

// out_r = a x_r + b y_r + g z_r over n entries (strides sx, sy, so per rhs);
// terms with a zero coefficient are not read; out may alias an input
hipError_t vec_axpbypcz(hipStream_t s, long long n, int nrhs, double a, const double* x,
                        long long sx, double b, const double* y, long long sy, double g,
                        const double* z, long long sz, double* out, long long so);
// y_r = sum_t dcoef[r*nt + t] * x[t]_r over n entries, rhs stride ld
hipError_t vec_lincomb(hipStream_t s, long long n, long long ld, int nrhs, int nt,
                       const double* const* x, const double* dcoef, double* y);
// dout[r*npair + q] = <X_q,r , Y_r>, X_q = X + q*xstride (deterministic order)
hipError_t vec_multidot_async(hipStream_t s, long long n, long long ld, const double* X,
                              long long xstride, int npair, const double* Y, int nrhs,
                              double* partial, double* dout);
size_t vec_partial_doubles(int npair, int nrhs);
// Y_r -= sum_q dh[r*hld + q] V_q,r
hipError_t vec_sub_combo(hipStream_t s, long long n, long long ld, const double* V,
                         long long vstride, int nq, const double* dh, int hld, int nrhs,
                         double* Y);
// Y_r += sum_q dh[r*hld + q] V_q,r
hipError_t vec_add_combo(hipStream_t s, long long n, long long ld, const double* V,
                         long long vstride, int nq, const double* dh, int hld, int nrhs,
                         double* Y);
// y += sum_m s1[m] (x) s2[m] (x) s3[m]  (direction 1 fastest)
hipError_t rank1_sum(hipStream_t s, int n1, int n2, int n3, int nm, const double* s1,
                     const double* s2, const double* s3, double* y);

// Per-right-hand-side state of device-side MINRES.
struct MinresScalars {
    double gamma, gamma_old, beta0, eta, c0, c1, s0, s1, delta, rel;
    int iters, done, status, pad;
};
// part_ref: partials of b . P^{-1} b for a warm start (else null): the
// monitored residual is then relative to ||b||_{P^{-1}}; a start that already
// meets tol ends the iteration at once
// (count: partials per right-hand side, vec_dot_partial_count of the length)
hipError_t minres_init(hipStream_t s, MinresScalars* sc, const double* part,
                       const double* part_ref, int count, double tol, int nrhs);
// A dot product handed over as partial sums: part[r * count + i], i < count,
// for right-hand side r (summed in a fixed order by the consumer).
struct Partials {
    const double* part;
    long long count;
};
// from the partials of (z_new.v_new) (the sum of two sets, b.part may be
// null): the rotation of sc_in, w_new = cw . (z, w_old, w), x += cx1 w_new;
// the new state goes to sc_out (not sc_in) and to mirror (device pointer of a
// host-mapped copy, or null)
hipError_t minres_w(hipStream_t s, long long n, long long ld, int nrhs, const double* z,
                    const double* wo, const double* w, double* wn, double* x,
                    const MinresScalars* sc_in, MinresScalars* sc_out, Partials a, Partials b,
                    double tol, double bd_tol, MinresScalars* mirror);
// the rotation and w/x update of iteration j-1 (as minres_w, when a.part is
// set; z, wo, w, wn, x its vectors) and the Lanczos step of iteration j in one
// launch: delta from the partials pkz of (Kz.z), v_new = cv . (Kz, v, v_old);
// reads the state of sc_in and writes the state after both to sc_out and
// mirror
hipError_t minres_wv(hipStream_t s, long long n, long long ld, int nrhs, const double* kz,
                     const double* v, const double* vo, double* vn, const double* z,
                     const double* wo, const double* w, double* wn, double* x,
                     const MinresScalars* sc_in, MinresScalars* sc_out, Partials pkz, Partials a,
                     Partials b, double tol, double bd_tol, MinresScalars* mirror);
// partial[r*count + b] of <X_r, Y_r>, count = vec_dot_partial_count(n)
// (finished by the MINRES, CG and FGMRES kernels)
hipError_t vec_dot_partials(hipStream_t s, long long n, long long ld, const double* X,
                            const double* Y, int nrhs, double* partial);
// partials per pair and right-hand side of a dot over n entries (at most
// vec_partial_doubles(1, 1); the chunks depend on n alone, so a batch and its
// right-hand sides one at a time give the same sums)
long long vec_dot_partial_count(long long n);

// Per-right-hand-side state of the inner preconditioned CG.
struct CgScalars {
    double rz, rz0;
    int done, pad;
};
// (count: partials per right-hand side, as for minres_init)
hipError_t cg_init(hipStream_t s, CgScalars* sc, const double* part, int count, int nrhs);
// cx = (1, alpha), cr = (1, -alpha) per rhs (2 doubles each)
hipError_t cg_alpha(hipStream_t s, CgScalars* sc, const double* part, int count, double* cx,
                    double* cr, int nrhs);
// cp = (1, beta) per rhs; freezes a rhs once sqrt(r.z) <= tol sqrt(r0.z0)
hipError_t cg_beta(hipStream_t s, CgScalars* sc, const double* part, int count, double* cp,
                   double tol, int nrhs);

// Per-right-hand-side state of device-side FGMRES.
struct FgScalars {
    double bnorm, rel;
    int done, active, jr, iters, status, pad;
};
// (count: partials per pair and right-hand side, as for minres_init)
hipError_t fg_init(hipStream_t s, FgScalars* sc, const double* part, int count, int nrhs);
hipError_t fg_begin(hipStream_t s, FgScalars* sc, const double* part, int count, double* g,
                    double* vscale, int m, int nrhs);
hipError_t fg_h(hipStream_t s, FgScalars* sc, const double* part, int count, double* H,
                double* hcoef, int j, int pass, int m, int nrhs);
// mirror: device pointer of a host-mapped copy of sc (or null), refreshed by the kernel
hipError_t fg_rot(hipStream_t s, FgScalars* sc, const double* part, int count, double* H,
                  double* cs, double* sn, double* g, double* vscale, double tol, double bd_tol,
                  int j, int m, int nrhs, FgScalars* mirror);
hipError_t fg_solve(hipStream_t s, const FgScalars* sc, const double* H, const double* g, double* y,
                    int m, int jmax, int nrhs);
hipError_t fg_check(hipStream_t s, FgScalars* sc, const double* part, int count, double tol,
                    int nrhs);
// partial[((r*npair + q)*count + b] of <X_q,r , Y_r>, count = vec_dot_partial_count(n)
hipError_t vec_multidot_partials(hipStream_t s, long long n, long long ld, const double* X,
                                 long long xstride, int npair, const double* Y, int nrhs,
                                 double* partial);

}  // namespace hp
