/*
 * hyperpower.h -- C ABI of the MI355X hyper-power preconditioned Stokes solver.
 *
 * Method: M.L. Mika, M.F.P. ten Eikelder, D. Schillinger, R.R. Hiemstra,
 * "Matrix-free polynomial preconditioning of saddle point systems using the
 * hyper-power method" (arXiv 2311.06926).
 *
 * Problem (Sec. 3.2, eq. systemmatrix): find u_h in V_h, p_h in Q_h with
 *
 *      [ A  B ] [u]   [f]
 *      [ B' 0 ] [p] = [0],
 *
 * the divergence-conforming tensor-product B-spline discretisation of the
 * Stokes equations on [0,1]^3 with E uniform elements per direction,
 * velocity degree p (component i has degree p in direction i and p-1 in the
 * others, App. B.2), pressure degree p-1, strong v.n = 0 and Nitsche
 * (weak) tangential conditions with alpha = c_pen * E (Sec. 3.1).
 *
 * VECTOR LAYOUT (all buffers): [u1 | u2 | u3 | p], each block a 3-tensor
 * stored with direction 1 fastest (vec ordering of App. A.2).  With
 * nN = E+p-2 and nM = E+p-1 the block shapes (n1, n2, n3) are
 *      u1: (nN, nM, nM)   u2: (nM, nN, nM)   u3: (nM, nM, nN)   p: (nM, nM, nM)
 * n_V = 3 nN nM^2, n_Q = nM^3, N = n_V + n_Q.  A batch of nrhs vectors is
 * stored back to back (the right-hand-side index is the slowest mode,
 * stride N).  Velocity-only buffers (apply_A/apply_B outputs) have stride
 * n_V, pressure-only buffers stride n_Q.
 *
 * MEMORY: every vector argument is a DEVICE pointer (FP64) on the device
 * that was current at hp_setup; the caller owns it.  The library owns only
 * the context and its tables/workspace.  Inputs and outputs must not
 * overlap unless stated.
 *
 * STREAMS: all work is enqueued on the stream given to hp_setup (0 = the
 * null stream).  hp_apply_* are asynchronous; hp_solve and hp_grad return
 * after the result is complete and fill their host-side info structs.
 *
 * ERRORS: functions return hp_status.  HP_EINVAL: a bad argument (nothing
 * is written).  HP_EHIP: a HIP runtime error.  HP_ENOMEM: device
 * allocation failed.  HP_ENOTSPD: a preconditioned inner product
 * r' P^{-1} r <= 0 was met (the preconditioner is not positive definite,
 * Sec. 2 Remark rmk:convergence_Pk), HP_EBREAKDOWN: Krylov breakdown,
 * HP_ENOCONV: maxit reached (x holds the last iterate), HP_ENAN: a NaN/Inf
 * appeared.  No C++ exception crosses this interface.
 */
#ifndef HYPERPOWER_H
#define HYPERPOWER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hp_ctx hp_ctx;

typedef enum {
    HP_OK = 0,
    HP_EINVAL = -1,
    HP_EHIP = -2,
    HP_ENOMEM = -3,
    HP_ENOTSPD = -4,
    HP_EBREAKDOWN = -5,
    HP_ENOCONV = -6,
    HP_ENAN = -7
} hp_status;

/* Precision of the preconditioner's fast-diagonalisation products (the
 * Krylov method always runs in FP64): FP64; FP32 (FP32 MFMA, FP32 storage of
 * the intermediates); split BF16 (each FP32 operand as hi + lo BF16 halves,
 * three BF16 MFMA products accumulated in FP32: about 16 significant bits,
 * products good to ~1e-5 relative).  Split BF16 runs in the 16-wave and
 * row-block plans (odd fd_plan codes, no 2x2 blocks); the 4-wave plans and
 * the mode-product GEMMs take FP32 products for it. */
enum { HP_PREC_FP64 = 0, HP_PREC_FP32 = 1, HP_PREC_BF16X3 = 2 };
/* Krylov method. MINRES needs an exactly symmetric preconditioner (FP64). */
enum { HP_MINRES = 0, HP_FGMRES = 1 };
/* Schur-complement sequence of Sec. 4.1: eq. Pcq1 (with inner updates),
 * eq. Pcq2 (without; B' P_{V,l}^{-1} B with l = schur_level), or eq. Pcq2 on
 * B' PCG(A, P_{V,l}) B, an inner preconditioned conjugate-gradient solve
 * (options (3), l = 0, and (4), l > 0; the operator is not linear, so the
 * solve needs HP_FGMRES). */
enum { HP_SCHUR_PCQ1 = 1, HP_SCHUR_PCQ2 = 2, HP_SCHUR_PCG = 3 };
/* Index l of P_{V,l} used by the k-th update of eq. Pcq1: LITERAL is the
 * schedule of Sec. 4.1 option (5), l = 0 for k = 1 and l = k for k > 1;
 * PREV uses l = k - 1. */
enum { HP_L_LITERAL = 0, HP_L_PREV = 1 };

typedef struct hp_opts {
    double c_pen;       /* Nitsche penalty constant, alpha = c_pen / h; 0 (default) =
                           max(12.5, 2.5 (degree + 1)) */
    int schur_variant;  /* HP_SCHUR_PCQ1 (default) or HP_SCHUR_PCQ2 */
    int l_schedule;     /* HP_L_LITERAL (default) or HP_L_PREV */
    int precision;      /* HP_PREC_* for P_k (default FP64) */
    int krylov;         /* HP_MINRES (default) or HP_FGMRES */
    int restart;        /* FGMRES restart length m (default 50, <= 128) */
    int maxit;          /* Krylov iteration limit (default 1000) */
    int order;          /* hyper-power order q >= 2 used by hp_solve (default 2) */
    int iters;          /* hyper-power updates k >= 0 used by hp_solve (default 1) */
    int max_rhs;        /* largest batch accepted (workspace size, default 1) */
    int poll_lag;       /* MINRES: the host reads the convergence flags of iteration j
                           once iteration j + poll_lag is enqueued (1..3, default 1), so
                           that it stays that far ahead of the device (with direct
                           launches it waits for the start of iteration j + 1, which
                           finishes iteration j; with graphs for the end of iteration
                           j); up to poll_lag iterations then run past convergence and
                           leave x unchanged */
    int use_graph;      /* solve: 0 = launch the kernels of each iteration directly
                           (default), 1 = replay each iteration (FGMRES: each Arnoldi
                           step) as one captured HIP graph; results are identical bit
                           for bit in both modes */
    int autotune;       /* time the launch shapes below at setup and keep the fastest
                           (default 1); results do not depend on the shapes */
    int op_kchunk;      /* operator kernels: i3-planes per workgroup, 0 = tuned/model */
    int op_order;       /* operator kernels: velocity workgroup order, -1 = tuned/model,
                           0 = tiles fastest, 1 = components fastest */
    int fd_plan;        /* P_0 kernels: -1 = tuned/default; 0..7 = the in-LDS kernels
                           (a whole direction, <= 128, in MFMA tiles): bit 0 = 16-wave
                           kernels, bit 1 = 1D matrices staged in LDS (if they fit),
                           bit 2 = 2x2 blocks of MFMA tiles per wave (16-wave plans,
                           FP64/FP32); 8 = every mode product as a batched GEMM over
                           HBM (FP64/FP32; the plan used whenever E + degree - 1 > 128,
                           where split BF16 falls back to FP32 products); 9 = the in-LDS
                           products with one 16-row block of a plane per 4-wave
                           workgroup and 16 z rows per workgroup (small meshes: several
                           times the workgroups of plans 0..7, the same result as the
                           16-wave plans) */
    int op_slabs;       /* operator: i3-slabs run one after the other (pressure chain
                           then velocity per slab), 0 = tuned/model */
    int schur_level;    /* eq. Pcq2 only: the fixed P_{V,l} inside B' P_{V,l}^{-1} B,
                           l = schur_level in [0, 6] (default 0 = P_{V,0}, option (1)
                           of Sec. 4.1; l > 0 is option (2), a fixed P_{V,k}, which for
                           large l approaches eq. Pcq_exact); for HP_SCHUR_PCG the
                           preconditioner P_{V,l} of the inner conjugate gradients */
    int schur_pcg_iters;   /* HP_SCHUR_PCG: inner CG steps, 1..1000 (default 20) */
    double schur_pcg_tol;  /* HP_SCHUR_PCG: a right-hand side stops once its
                              sqrt(r.P^{-1}r) has dropped by this factor (default 1e-2) */
    int op_fused;       /* operator K and A: -1 = tuned/model (default), 0 = the pressure
                           and velocity kernels, 1 = one single-pass kernel (degree <= 4) */
    int op_staged;      /* operator kernels: -1 = tuned/model (default), 0 = stream their
                           i3-planes, 1 = load all planes of a chunk at once where such a
                           kernel exists (velocity, modes K and A: degree <= 4 and op_kchunk
                           2, 4 or 8, 8 only to degree 3; pressure chain: degree <= 3 and
                           op_kchunk 2 or 4); same results bit for bit */
    int forward;        /* forward problem y = K x inside hp_solve: 0 = the Kronecker-
                           factored operator kernels (default), 1 = the quadrature-based
                           operator of hp_apply_K_quad (the same matrix up to rounding);
                           the reported true residual always uses hp_apply_K */
    int use_x0;         /* hp_solve: 0 = start from x_0 = 0 (default, Sec. 5), 1 = start
                           from the x passed in (warm start / resume); the stopping test
                           stays relative to b (see hp_solve) */
    int spectrum_gate;  /* hp_setup: 0 = off (default); n > 0 = run n Lanczos steps on each
                           block of P_0 (P_{V,0}^{-1} A and P_{Q,0}^{-1} B' P_{V,0}^{-1} B,
                           as hp_spectrum) and refuse the context with HP_ENOTSPD when an
                           estimated eigenvalue lies outside (0, 2), where the hyper-power
                           sequence diverges and P_k (k >= 1) loses definiteness (Sec. 2,
                           Lemma Sk_posdef, Remark rmk:convergence_Pk) */
    double p0_scale;    /* damping factor w of the base preconditioner: every
                           application of P_0^{-1} (both blocks, also inside P_k and
                           hp_spectrum) is w P_0^{-1}; 0 or 1 (default) = the plain P_0 of
                           Sec. 4.  The hyper-power sequence needs sigma(w P_0^{-1} A~) in
                           (0, 2) (Lemma Sk_posdef): a w that pushes the largest eigenvalue
                           past 2 makes P_k indefinite, which spectrum_gate and MINRES
                           report as HP_ENOTSPD */
    double breakdown_tol; /* Krylov breakdown threshold (default 0: exact breakdown only).
                           MINRES stops with HP_EBREAKDOWN when the rotated diagonal entry
                           a of the tridiagonal Lanczos matrix has |a| <= breakdown_tol *
                           (|delta| + gamma + gamma_next), its column's entries; FGMRES when
                           the rotated pivot of Hessenberg column j is <= breakdown_tol times
                           that column's 2-norm.  A value >= 1 forces the breakdown path at
                           the first iteration (used to test the error path) */
    int op_dma;         /* streaming velocity kernel (modes K, A, M_V): -1 = default (1),
                           1 = stage each plane's tile with direct-to-LDS loads into a ring
                           of three LDS planes (two planes in flight), 0 = stage through
                           registers (one plane in flight); same results bit for bit */
    int op_pres_wide;   /* streaming pressure kernel (modes K, A, B, B^T): -1 = tuned/model
                           (default), 0 = 16 x 8 tiles, 1 = 32 x 8 tiles (less halo per
                           point, larger workgroups); same results bit for bit */
} hp_opts;

/* Launch shapes in use (host struct, filled by hp_get_tuning). */
typedef struct hp_tuning {
    int op_kchunk;      /* operator i3-planes per workgroup for this nrhs */
    int op_order;       /* operator velocity workgroup order for this nrhs */
    int op_tuned;       /* 1 if the autotuner timed the operator shapes for this nrhs */
    int op_slabs;       /* operator i3-slabs for this nrhs */
    int fd_plan[3];     /* P_0 plan per precision (HP_PREC_*), -1 = default plan */
    double op_us;       /* tuned apply_K time (microseconds), 0 if not tuned */
    double fd_us[3];    /* tuned apply_P0 time per precision, 0 if not tuned */
    int op_staged;      /* 1 if the operator uses the all-planes velocity kernel */
    int op_pres_wide;   /* 1 if the streaming pressure kernel runs on 32 x 8 tiles */
} hp_tuning;

/* Per-solve report (host struct, filled by hp_solve / hp_grad). */
typedef struct hp_solve_info {
    int iterations;        /* max over the batch */
    int converged;         /* 1 if every right-hand side met tol */
    double relres;         /* max over the batch of the monitored relative residual */
    double true_relres;    /* max over the batch of ||b - K x||_2 / ||b||_2 (FP64) */
    double seconds;        /* wall time of the call */
    int iters_per_rhs[64]; /* iteration count of each right-hand side (first 64) */
} hp_solve_info;

/* Fill *o with the defaults listed above. */
void hp_default_opts(hp_opts* o);

/* The launch shapes used for batches of nrhs right-hand sides.  The
 * autotuner (hp_opts.autotune) times apply_K for nrhs = 1 and nrhs =
 * max_rhs over i3-chunk lengths, workgroup orders and i3-slab counts, and apply_P0 per
 * precision over the plans that fit in LDS (a batch size or precision the
 * tuner did not time uses the cost model / default plan).  Every shape and
 * plan computes the same result; only the time differs. */
hp_status hp_get_tuning(const hp_ctx* ctx, int nrhs, hp_tuning* out);

/* Build the univariate tables (App. B.3, Sec. 3.3), the generalised
 * eigen-decompositions for fast diagonalisation (App. A.3-A.4) and the
 * workspace.  elements >= 1, 2 <= degree <= 8, nu > 0.  Returns HP_ENOTSPD
 * when the Nitsche penalty opts.c_pen is too small for the degree and mesh
 * (the augmented T^ of Sec. 3.3 is then indefinite, e.g. degree 8 with
 * fewer than 6 elements at the default 12.5), or, with opts.spectrum_gate,
 * when P_0 leaves the convergence interval (0, 2).  opts may be NULL
 * (defaults).  stream: a hipStream_t or NULL.  *out receives the context.
 * Fast diagonalisation holds a whole direction in MFMA tiles while
 * E + degree - 1 <= 128 and runs its mode products as batched GEMMs beyond
 * (opts.fd_plan = 8), so every call serves any mesh that fits in memory. */
hp_status hp_setup(int elements, int degree, double nu, const hp_opts* opts,
                   void* stream, hp_ctx** out);

/* Change the viscosity (A, P_{V,0} scale with nu, P_{Q,0} with 1/nu,
 * Sec. 4; the tables are nu-free). */
hp_status hp_set_nu(hp_ctx* ctx, double nu);

/* Block shapes dims[b][d] (b = u1,u2,u3,p; d = direction) and offsets
 * (start of u1,u2,u3,p and N) of one vector.  Host arrays. */
hp_status hp_sizes(const hp_ctx* ctx, int64_t dims[4][3], int64_t offsets[5]);

/* y = K x for nrhs vectors (eq. systemmatrix): y_u = A u + B p, y_p = B' u. */
hp_status hp_apply_K(hp_ctx* ctx, const double* x, double* y, int nrhs);

/* y = K x by the quadrature-based, matrix-free route of Sec. 5.3: the
 * velocity gradients and the pressure are evaluated at the p+1 Gauss-Legendre
 * points per element and direction by global sum factorisation, the flux of
 * the weak form (Sec. 3.1; symmetric Nitsche face terms of Sec. 3.3 at the
 * face Gauss points) is formed at every point and integrated back.  Exact
 * quadrature: the same matrix as hp_apply_K, up to rounding.  x and y are
 * device arrays of nrhs vectors (stride N, layout of hp_apply_K), y must not
 * alias x.  The first call allocates the point tables and a scratch of
 * 7 (E(p+1)+2) n_M^2 + 10 (E(p+1)+2)^2 n_M + 10 (E(p+1)+2)^3 doubles
 * (one right-hand side at a time); HP_ENOMEM if that fails. */
hp_status hp_apply_K_quad(hp_ctx* ctx, const double* x, double* y, int nrhs);

/* y = A u (velocity only, stride n_V; Sec. 3.3). */
hp_status hp_apply_A(hp_ctx* ctx, const double* u, double* y, int nrhs);

/* y = B p (pressure in, stride n_Q; velocity out, stride n_V; Sec. 3.3). */
hp_status hp_apply_B(hp_ctx* ctx, const double* p, double* y, int nrhs);

/* y = B' u (velocity in, stride n_V; pressure out, stride n_Q). */
hp_status hp_apply_Bt(hp_ctx* ctx, const double* u, double* y, int nrhs);

/* y = P_0^{-1} x, the block-diagonal base preconditioner of Sec. 4
 * (eq. blockdiagprecond): the three diagonal blocks of A inverted by fast
 * diagonalisation (App. A.4) and P_{Q,0}^{-1} = 2 nu (M^^{-1})^{(x)3}. */
hp_status hp_apply_P0(hp_ctx* ctx, const double* x, double* y, int nrhs);

/* y = P_k^{-1} x, k = iters hyper-power updates of order q = order applied
 * block-wise to P_0 (eqs. hyperpowersequence, Pcv, Pcq1/Pcq2 per
 * opts.schur_variant and opts.l_schedule).  order >= 2, 0 <= iters <= 6. */
hp_status hp_apply_hyperpower(hp_ctx* ctx, int order, int iters, const double* x,
                              double* y, int nrhs);

/* y = P_{V,k}^{-1} u, the velocity block of P_k alone (eq. Pcv; its Neumann
 * form, eq. neumann: q^k applications of P_{V,0}^{-1} and q^k - 1 of A), the
 * operator timed in the paper's Sec. 5.1 cost study (eq. hyperpower_scaling).
 * u, y: velocity vectors (stride n_V), device, must not overlap.
 * order >= 2, 0 <= iters <= 6; opts.precision applies. */
hp_status hp_apply_PV(hp_ctx* ctx, int order, int iters, const double* u, double* y, int nrhs);

/* Blocks whose preconditioned spectrum hp_spectrum estimates. */
enum { HP_SPEC_VELOCITY = 0, HP_SPEC_SCHUR = 1 };

/* Lanczos estimate of the extreme eigenvalues of a preconditioned block
 * (Sec. 2, Lemma Sk_posdef and Corollary cor:Skform, which predict the
 * spectrum after k updates from that of P_0; the spectra of Sec. 5.2):
 *   HP_SPEC_VELOCITY: P_{V,k}^{-1} A,
 *   HP_SPEC_SCHUR:    P_{Q,k}^{-1} S~_l, S~_l = B' P_{V,l}^{-1} B with
 *                     l = s_level (large l approaches B' A^{-1} B),
 * with k = iters updates of order q = order (eqs. Pcv, Pcq1/Pcq2 per
 * opts.schur_variant, opts.l_schedule, opts.schur_level) in the context's
 * precision.  The Lanczos process runs in the inner product of P_{.,k}
 * from the residual r_0 = start (velocity) or r_0 = S~_l start (Schur;
 * every residual is projected orthogonally to the constant-pressure null
 * vector of B, so the smallest non-zero eigenvalue is estimated).
 * start: device vector of n_V (velocity) or n_Q (Schur) doubles, read only.
 * steps: 1 <= steps <= block dimension; the process stops early at an
 * invariant subspace.  alpha, beta: host arrays of `steps` doubles
 * receiving the tridiagonal matrix (beta[j] couples steps j and j+1), or
 * NULL.  *done: steps taken; *lmin, *lmax: extreme eigenvalues of the
 * tridiagonal matrix (Sturm bisection), inner estimates of the block's.
 * Synchronous; allocates and frees 5-6 block vectors of device memory.
 * Returns HP_ENOTSPD if r' P^{-1} r < 0 (the preconditioner is indefinite). */
hp_status hp_spectrum(hp_ctx* ctx, int block, int order, int iters, int s_level, int steps,
                      const double* start, double* alpha, double* beta, int* done,
                      double* lmin, double* lmax);

/* Solve K x = b to relative tolerance tol (Sec. 5: MINRES to 1e-8),
 * preconditioned by P_k (opts.order, opts.iters), from x_0 = 0, or from the
 * x passed in when opts.use_x0 = 1 (x is then read first; MINRES and FGMRES
 * run on the residual b - K x_0 and update x in place).  The stopping test
 * is relative to b in both cases: MINRES monitors the preconditioned norm
 * ||r_j||_{P^{-1}} / ||b||_{P^{-1}} (the norm its recurrence carries; a warm
 * start costs one extra P_k application for ||b||_{P^{-1}}), FGMRES the
 * 2-norm ||r_j||_2 / ||b||_2, confirmed with the true residual at the end of
 * each restart cycle.  info->true_relres is always the FP64 2-norm
 * ||b - K x||_2 / ||b||_2 of the returned x; for MINRES it can differ from
 * the monitored value by up to the condition number of P_k (converged = 1
 * refers to the monitored norm).  info may be NULL.  Returns HP_ENOCONV
 * (x = last iterate) if maxit is reached, HP_ENAN if b, x_0 or an iterate is
 * not finite, HP_ENOTSPD if MINRES meets r' P_k^{-1} r < 0, HP_EBREAKDOWN
 * (see opts.breakdown_tol; x = the last iterate). */
hp_status hp_solve(hp_ctx* ctx, const double* b, double* x, int nrhs, double tol,
                   hp_solve_info* info);

/* hp_solve without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the Krylov vectors live in a fixed 32 MiB device array of the
 * library (2^22 doubles per GPU, held from the library's load until the
 * process ends) instead of memory allocated on first use.  Same arguments,
 * results and errors as hp_solve, computed by the same kernels, with the
 * iteration launched directly (opts.use_graph is ignored).  Limits: the
 * solve must fit the array -- 10 N max_rhs doubles for MINRES,
 * (2 restart + 2) N max_rhs for FGMRES (e.g. MINRES at 32^3 elements, degree
 * 3, N = 153,748, up to max_rhs = 2) -- else HP_ENOMEM, nothing written;
 * nrhs <= 64; with opts.forward = 1 the quadrature operator must already be
 * set up (HP_EINVAL otherwise).  Every call on one GPU shares that GPU's
 * array and overwrites it (each call initialises what it reads): calls that
 * overlap in time on one GPU, from any context or stream, race. */
hp_status hp_solve_noalloc(hp_ctx* ctx, const double* b, double* x, int nrhs, double tol,
                           hp_solve_info* info);

/* Right-hand side of the lid-driven cavity (Sec. 5, Fig. liddrivencavity)
 * with a body force, b = [F_lid + F_modes + M_V beta; 0] (the linear form
 * l(v) of Sec. 3.1 plus the Nitsche lid data): for each rhs r, lid speed
 * lid[r] on x3 = 1, and for each velocity component c and mode m
 * F_c += amp[(r*3 + c)*nmodes + m] * prod_d sin(pi k_d x_d) with
 * k_d = waves[((r*3 + c)*nmodes + m)*3 + d] integrated against the basis,
 * and, when beta is not NULL, the body force whose coefficients in V_h are
 * beta (device, n_V per rhs, stride n_V), which contributes M_V beta.
 * Host arrays lid, amp, waves (lid may be NULL: no lid; amp/waves may be
 * NULL when nmodes == 0); device output b (N x nrhs, must not overlap beta). */
hp_status hp_build_rhs(hp_ctx* ctx, const double* lid, int nmodes, const double* amp,
                       const int* waves, const double* beta, double* b, int nrhs);

/* y = M_V u, the velocity mass matrix (block diagonal L2 Gram matrix of
 * V_h), stride n_V; used by the loss gradient of the differentiable solve. */
hp_status hp_apply_MV(hp_ctx* ctx, const double* u, double* y, int nrhs);

/* Adjoint pieces of the differentiable solve with K x = [F_lid(nu) + M_V beta; 0]:
 * given the forward solution x and the adjoint lambda (K lambda = [dL/du; 0]),
 *   dL_dbeta = M_V lambda_u                          (device, stride n_V)
 *   dL_dnu[r] = lambda_u' (F_lid/nu - A u / nu)       (host, one per rhs)
 * F_lid is rebuilt from lid[r] (host).  K is symmetric, so lambda comes
 * from hp_solve with the same preconditioner. */
hp_status hp_grad(hp_ctx* ctx, const double* x, const double* lambda, const double* lid,
                  double* dL_dbeta, double* dL_dnu, int nrhs);

/* Release the context and its device memory. */
void hp_destroy(hp_ctx* ctx);

/* Static string for a status code. */
const char* hp_status_string(hp_status s);

#ifdef __cplusplus
}
#endif

#endif /* HYPERPOWER_H */
