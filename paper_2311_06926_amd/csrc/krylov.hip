// Vector kernels for the Krylov solvers: fused linear combinations with
// per-right-hand-side coefficients and deterministic dot products (fixed
// grid, fixed reduction order: a wave64 shuffle tree, then an LDS tree, then
// one ordered pass over the per-block partials), plus the right-hand-side
// assembly of the cavity (Sec. 5).
#include "hp_internal.h"
#include "vec.h"

namespace hp {

namespace {

constexpr int VT = 256;
// partial sums per (pair, rhs), one per chunk of the vector: 480 chunks from
// 2^19 entries on (FGMRES at 64^3: 11.9 -> 11.0 ms, the FP32 preconditioner
// 10.6 -> 9.7 ms), 240 below (MINRES at 32^3 is 3% slower with 480)
constexpr int DOT_BLOCKS_MAX = 480;
inline int dot_blocks(long long n) { return n >= (1LL << 19) ? DOT_BLOCKS_MAX : DOT_BLOCKS_MAX / 2; }

__global__ void k_axpby(long long n, double a, const double* __restrict__ x, double b,
                        double* __restrict__ y) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

__global__ void k_copy(long long n, const double* __restrict__ x, double* __restrict__ y) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) y[i] = x[i];
}

__global__ void k_fill(long long n, double v, double* __restrict__ y) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) y[i] = v;
}

// out_r = a x_r + b y_r + g z_r for every right-hand side r (blockIdx.y); a
// term whose coefficient is zero is not read.  out may alias x, y or z.
__global__ void k_axpbypcz(long long n, double a, const double* x, long long sx, double b,
                           const double* y, long long sy, double g, const double* z, long long sz,
                           double* out, long long so) {
    const int r = blockIdx.y;
    x += (long long)r * sx;
    if (y) y += (long long)r * sy;
    if (z) z += (long long)r * sz;
    out += (long long)r * so;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) {
        double v = a * x[i];
        if (b != 0.0) v += b * y[i];
        if (g != 0.0) v += g * z[i];
        out[i] = v;
    }
}

// y_r = sum_t coef[r*nt + t] * x_t[r*ld + i]  (up to 4 terms; y may alias one x_t)
struct LinArgs {
    const double* x[4];
    double* y;
    const double* coef;
    int nt;
    long long n, ld;
};

__global__ void k_lincomb(LinArgs a) {
    const int r = blockIdx.y;
    const double* cf = a.coef + (long long)r * a.nt;
    double c0 = cf[0], c1 = a.nt > 1 ? cf[1] : 0.0, c2 = a.nt > 2 ? cf[2] : 0.0,
           c3 = a.nt > 3 ? cf[3] : 0.0;
    const long long off = (long long)r * a.ld;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < a.n; i += st) {
        double v = c0 * a.x[0][off + i];
        if (a.nt > 1) v += c1 * a.x[1][off + i];
        if (a.nt > 2) v += c2 * a.x[2][off + i];
        if (a.nt > 3) v += c3 * a.x[3][off + i];
        a.y[off + i] = v;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    }
    __syncthreads();
    return s;
}

// s + p[t] + p[t + VT] + p[t + 2 VT] + ... over the indices below count
// (t = threadIdx.x, a workgroup of VT threads), in that order; the first two
// are loaded together so that their latencies overlap.
__device__ __forceinline__ double strided_sum(const double* p, long long count, double s) {
    const long long t = threadIdx.x;
    const double a = p[t < count ? t : 0], b = p[t + VT < count ? t + VT : 0];
    if (t < count) s += a;
    if (t + VT < count) s += b;
    for (long long i = t + 2 * VT; i < count; i += VT) s += p[i];
    return s;
}

// partial[(r*npair + q)*nb + b] = sum over chunk b of x_q . y (x_q = X +
// q*xstride, one y per rhs; nb = dot_blocks(n) chunks of the vector).  A
// workgroup takes DOT_QB pairs of one chunk, so y is read once per DOT_QB
// pairs; each chunk's sum runs in the same order whatever the number of
// pairs or right-hand sides (a batch gives the same partials as its
// right-hand sides one at a time).
constexpr int DOT_QB = 8;
__global__ void k_dot_partial(long long n, long long ld, const double* X, long long xstride,
                              int npair, const double* Y, int nb, double* partial) {
    __shared__ double sh[VT / 64][DOT_QB];
    const int r = blockIdx.z, q0 = blockIdx.y * DOT_QB;
    const int nq = min(DOT_QB, npair - q0);
    const double* x = X + (long long)q0 * xstride + (long long)r * ld;
    const double* y = Y + (long long)r * ld;
    const long long chunk = (n + nb - 1) / nb;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = min(n, lo + chunk);
    double s[DOT_QB];
#pragma unroll
    for (int qq = 0; qq < DOT_QB; ++qq) s[qq] = 0.0;
    // thread t takes elements t, t + VT, ... of the chunk, DOT_U of them at
    // a time with all their loads issued before the first product (an index
    // past the chunk is clamped for the load and its product skipped)
    constexpr int DOT_U = 4;
    for (long long k0 = threadIdx.x; k0 < chunk; k0 += DOT_U * VT) {
        double yv[DOT_U], xv[DOT_U][DOT_QB];
#pragma unroll
        for (int u = 0; u < DOT_U; ++u) {
            const long long i = lo + k0 + u * VT;
            const long long ic = i < hi ? i : lo;
            yv[u] = y[ic];
#pragma unroll
            for (int qq = 0; qq < DOT_QB; ++qq)
                if (qq < nq) xv[u][qq] = x[qq * xstride + ic];
        }
#pragma unroll
        for (int u = 0; u < DOT_U; ++u)
            if (lo + k0 + u * VT < hi)
#pragma unroll
                for (int qq = 0; qq < DOT_QB; ++qq)
                    if (qq < nq) s[qq] += xv[u][qq] * yv[u];
    }
    // all sums of the workgroup in one reduction: wave trees, then thread v
    // adds the waves' results of sum v in wave order (as block_sum does)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int qq = 0; qq < DOT_QB; ++qq) {
        if (qq >= nq) break;  // uniform over the workgroup
        const double v = wave_sum(s[qq]);
        if (lane == 0) sh[wave][qq] = v;
    }
    __syncthreads();
    const int v = threadIdx.x;
    if (v < nq) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w][v];
        partial[((long long)r * npair + q0 + v) * nb + blockIdx.x] = t;
    }
}
// k_dot_partial over npair pairs and nrhs right-hand sides, one chunk per
// workgroup (two chunks per workgroup for batches, the same partials with
// half the workgroups, was measured slower: 48^3 x 32 FGMRES 102.5 -> 108 ms)
inline void dot_partial_launch(hipStream_t s, long long n, long long ld, const double* X,
                               long long xstride, int npair, const double* Y, int nrhs,
                               double* partial) {
    const unsigned groups = (unsigned)((npair + DOT_QB - 1) / DOT_QB);
    const int nb = dot_blocks(n);
    hipLaunchKernelGGL(k_dot_partial, dim3(nb, groups, nrhs), dim3(VT), 0, s, n, ld, X, xstride,
                       npair, Y, nb, partial);
}

__global__ void k_dot_final(const double* partial, int count, double* out) {
    __shared__ double sh[VT / 64];
    const long long base = (long long)blockIdx.x * count;
    double s = 0.0;
    s = strided_sum(partial + base, count, s);
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// y_r -= sum_{q<nq} h[r*hld + q] * V_q   (V_q = V + q*vstride)
__global__ void k_sub_combo(long long n, long long ld, const double* V, long long vstride, int nq,
                            const double* h, int hld, double* Y) {
    const int r = blockIdx.y;
    const double* hr = h + (long long)r * hld;
    double* y = Y + (long long)r * ld;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) {
        double s = 0.0;
        for (int q = 0; q < nq; ++q) s += hr[q] * V[(long long)q * vstride + (long long)r * ld + i];
        y[i] -= s;
    }
}

// y_r += sum_{q<nq} h[r*hld + q] * V_q
__global__ void k_add_combo(long long n, long long ld, const double* V, long long vstride, int nq,
                            const double* h, int hld, double* Y) {
    const int r = blockIdx.y;
    const double* hr = h + (long long)r * hld;
    double* y = Y + (long long)r * ld;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) {
        double s = 0.0;
        for (int q = 0; q < nq; ++q) s += hr[q] * V[(long long)q * vstride + (long long)r * ld + i];
        y[i] += s;
    }
}

// rank-one sums  y[i1 + n1 (i2 + n2 i3)] += sum_m s1[m][i1] s2[m][i2] s3[m][i3]
// (amplitudes folded into s3); one launch per (field, rhs)
__global__ void k_rank1_sum(int n1, int n2, int n3, int nm, const double* s1, const double* s2,
                            const double* s3, double* y) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long tot = (long long)n1 * n2 * n3;
    if (idx >= tot) return;
    int i1 = (int)(idx % n1);
    long long t = idx / n1;
    int i2 = (int)(t % n2);
    int i3 = (int)(t / n2);
    double s = 0.0;
    for (int m = 0; m < nm; ++m) s += s1[m * n1 + i1] * s2[m * n2 + i2] * s3[m * n3 + i3];
    y[idx] += s;
}

inline unsigned grid_for(long long n) {
    long long g = (n + VT - 1) / VT;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

hipError_t vec_axpby(hipStream_t s, long long n, double a, const double* x, double b, double* y) {
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(VT), 0, s, n, a, x, b, y);
    return hipGetLastError();
}

hipError_t vec_axpbypcz(hipStream_t s, long long n, int nrhs, double a, const double* x,
                        long long sx, double b, const double* y, long long sy, double g,
                        const double* z, long long sz, double* out, long long so) {
    hipLaunchKernelGGL(k_axpbypcz, dim3(grid_for(n), nrhs), dim3(VT), 0, s, n, a, x, sx, b, y, sy,
                       g, z, sz, out, so);
    return hipGetLastError();
}

hipError_t vec_copy(hipStream_t s, long long n, const double* x, double* y) {
    hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(VT), 0, s, n, x, y);
    return hipGetLastError();
}

hipError_t vec_zero(hipStream_t s, long long n, double* y) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(VT), 0, s, n, 0.0, y);
    return hipGetLastError();
}

hipError_t vec_lincomb(hipStream_t s, long long n, long long ld, int nrhs, int nt,
                       const double* const* x, const double* dcoef, double* y) {
    LinArgs a{};
    for (int t = 0; t < nt; ++t) a.x[t] = x[t];
    a.y = y;
    a.coef = dcoef;
    a.nt = nt;
    a.n = n;
    a.ld = ld;
    hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n), nrhs), dim3(VT), 0, s, a);
    return hipGetLastError();
}

hipError_t vec_multidot_async(hipStream_t s, long long n, long long ld, const double* X,
                              long long xstride, int npair, const double* Y, int nrhs,
                              double* partial, double* dout) {
    dot_partial_launch(s, n, ld, X, xstride, npair, Y, nrhs, partial);
    hipLaunchKernelGGL(k_dot_final, dim3(npair * nrhs), dim3(VT), 0, s, partial, dot_blocks(n),
                       dout);
    return hipGetLastError();
}

size_t vec_partial_doubles(int npair, int nrhs) { return (size_t)npair * nrhs * DOT_BLOCKS_MAX; }

hipError_t vec_sub_combo(hipStream_t s, long long n, long long ld, const double* V,
                         long long vstride, int nq, const double* dh, int hld, int nrhs,
                         double* Y) {
    hipLaunchKernelGGL(k_sub_combo, dim3(grid_for(n), nrhs), dim3(VT), 0, s, n, ld, V, vstride,
                       nq, dh, hld, Y);
    return hipGetLastError();
}

hipError_t vec_add_combo(hipStream_t s, long long n, long long ld, const double* V,
                         long long vstride, int nq, const double* dh, int hld, int nrhs,
                         double* Y) {
    hipLaunchKernelGGL(k_add_combo, dim3(grid_for(n), nrhs), dim3(VT), 0, s, n, ld, V, vstride,
                       nq, dh, hld, Y);
    return hipGetLastError();
}

hipError_t rank1_sum(hipStream_t s, int n1, int n2, int n3, int nm, const double* s1,
                     const double* s2, const double* s3, double* y) {
    long long tot = (long long)n1 * n2 * n3;
    hipLaunchKernelGGL(k_rank1_sum, dim3((unsigned)((tot + VT - 1) / VT)), dim3(VT), 0, s, n1, n2,
                       n3, nm, s1, s2, s3, y);
    return hipGetLastError();
}

hipError_t vec_dots(hp_ctx* c, long long n, long long ld, const double* x, const double* y,
                    int nrhs, double* out) {
    double* partial = c->d_red;
    double* dres = c->d_red + vec_partial_doubles(1, nrhs);
    hipError_t e = vec_multidot_async(c->stream, n, ld, x, 0, 1, y, nrhs, partial, dres);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(c->h_red, dres, sizeof(double) * nrhs, hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return e;
    for (int r = 0; r < nrhs; ++r) out[r] = c->h_red[r];
    return hipSuccess;
}

}  // namespace hp

// =====================================================================================
// MINRES with device-resident scalars (one thread per right-hand side).  The
// Lanczos/Givens recurrences of preconditioned MINRES run in these kernels,
// so an iteration needs no host round trip and can be replayed as a graph.
// Dot products are finished here from the fixed-order per-block partials.
namespace hp {
namespace {

// The scalar kernels below run one workgroup per right-hand side: the
// partials of its dot products are summed by the whole workgroup (strided
// over the threads, then the wave and workgroup trees: a fixed order), and
// thread 0 then takes the scalar step.  The result is valid in thread 0.
__device__ double sum_partials(const double* part, int count, int q, double* sh) {
    double s = 0.0;
    s = strided_sum(part + (long long)q * count, count, s);
    return block_sum(s, sh);
}

// after z = P^{-1} b:  gamma = sqrt(z.v), beta0 = eta = gamma, c = 1, s = 0
// part_ref (may be null): partials of b . P^{-1} b when the start residual
// is not b (warm start); the monitored residual is then relative to
// ||b||_{P^{-1}} instead of ||r_0||_{P^{-1}}.
__global__ void k_minres_init(MinresScalars* sc, const double* part_zv, const double* part_ref,
                              int count, double tol) {
    __shared__ double sh[VT / 64];
    const int r = blockIdx.x;
    const double zv = sum_partials(part_zv, count, r, sh);
    const double ref = part_ref ? sum_partials(part_ref, count, r, sh) : zv;
    if (threadIdx.x != 0) return;
    MinresScalars& m = sc[r];
    m = MinresScalars{};
    m.status = 0;
    if (!(zv >= 0.0) || !isfinite(zv) || !(ref >= 0.0) || !isfinite(ref)) {
        m.status = (zv < 0.0 || ref < 0.0) ? -4 : -7;
        m.done = 1;
        return;
    }
    m.gamma = sqrt(zv);
    m.gamma_old = 1.0;
    m.beta0 = ref > 0.0 ? sqrt(ref) : m.gamma;
    m.eta = m.gamma;
    m.c0 = m.c1 = 1.0;
    m.s0 = m.s1 = 0.0;
    m.rel = m.beta0 > 0.0 ? m.gamma / m.beta0 : 0.0;
    m.done = (m.gamma == 0.0) || (part_ref && m.rel <= tol);
    if (m.gamma == 0.0) m.rel = 0.0;
}

// after Kz = K z:  delta = (Kz.z)/gamma^2; coefficients of v_new = Kz/gamma - (delta/gamma) v - (gamma/gamma_old) v_old
__device__ void minres_a_core(MinresScalars& m, double kz, double* cv) {
    if (m.done) {
        cv[0] = cv[1] = cv[2] = 0.0;
        return;
    }
    const double g = m.gamma;
    m.delta = kz / (g * g);
    cv[0] = 1.0 / g;
    cv[1] = -m.delta / g;
    cv[2] = -g / m.gamma_old;
}

// after z_new = P^{-1} v_new: gamma_new, the Givens rotation, coefficients of
// w_new = (z/gamma - a3 w_old - a2 w)/a1 and x += c_new eta w_new, then shift.
__device__ void minres_b_core(MinresScalars& m, double zv, double* cw, double* cx, double tol,
                              double bd_tol) {
    cx[0] = 1.0;
    if (m.done) {
        cw[0] = cw[1] = cw[2] = 0.0;
        cx[1] = 0.0;
        return;
    }
    if (!isfinite(zv)) {
        m.status = -7;
        m.done = 1;
        cw[0] = cw[1] = cw[2] = 0.0;
        cx[1] = 0.0;
        return;
    }
    if (zv < 0.0) {
        m.status = -4;
        zv = 0.0;
    }
    const double gn = sqrt(zv), g = m.gamma;
    const double a0 = m.c1 * m.delta - m.c0 * m.s1 * g;
    const double a1 = hypot(a0, gn);
    const double a2 = m.s1 * m.delta + m.c0 * m.c1 * g;
    const double a3 = m.s0 * g;
    // breakdown: the rotated diagonal entry vanishes against its column
    // (delta, gamma, gamma_next) of the Lanczos matrix (bd_tol = 0: exactly)
    if (a1 <= bd_tol * (fabs(m.delta) + g + gn)) {
        m.status = -5;
        m.done = 1;
        cw[0] = cw[1] = cw[2] = 0.0;
        cx[1] = 0.0;
        return;
    }
    const double cn = a0 / a1, sn = gn / a1;
    cw[0] = 1.0 / (g * a1);
    cw[1] = -a3 / a1;
    cw[2] = -a2 / a1;
    cx[1] = cn * m.eta;
    m.eta = -sn * m.eta;
    m.gamma_old = g;
    m.gamma = gn;
    m.c0 = m.c1;
    m.c1 = cn;
    m.s0 = m.s1;
    m.s1 = sn;
    m.rel = fabs(m.eta) / m.beta0;
    m.iters += 1;
    if (m.rel <= tol || gn == 0.0 || m.status != 0) m.done = 1;
}

// ---- inner PCG for A y = b (Schur options (3)/(4) of Sec. 4.1) ------------------------
// Per rhs: rz = r.z; the step coefficients are written for vec_lincomb:
// cx = (1, alpha) for y += alpha p, cr = (1, -alpha) for r -= alpha A p,
// cp = (1, beta) for p = z + beta p.  A right-hand side whose preconditioned
// residual has dropped to tol of its start (or whose r.z is not positive)
// is frozen: alpha = 0 from then on.
__global__ void k_cg_init(CgScalars* sc, const double* part_rz, int count) {
    __shared__ double sh[VT / 64];
    const int r = blockIdx.x;
    const double rz = sum_partials(part_rz, count, r, sh);
    if (threadIdx.x != 0) return;
    sc[r].rz = rz;
    sc[r].rz0 = rz;
    sc[r].done = (rz > 0.0 && isfinite(rz)) ? 0 : 1;
}

__global__ void k_cg_alpha(CgScalars* sc, const double* part_pq, int count, double* cx,
                           double* cr) {
    __shared__ double sh[VT / 64];
    const int r = blockIdx.x;
    const double pq = sum_partials(part_pq, count, r, sh);
    if (threadIdx.x != 0) return;
    double a = 0.0;
    if (!sc[r].done && pq > 0.0 && isfinite(pq)) a = sc[r].rz / pq;
    else sc[r].done = 1;
    cx[2 * r] = 1.0;
    cx[2 * r + 1] = a;
    cr[2 * r] = 1.0;
    cr[2 * r + 1] = -a;
}

__global__ void k_cg_beta(CgScalars* sc, const double* part_rz, int count, double* cp,
                          double tol) {
    __shared__ double sh[VT / 64];
    const int r = blockIdx.x;
    const bool done = sc[r].done;  // the same in every thread of the workgroup
    if (threadIdx.x == 0) {
        cp[2 * r] = 1.0;
        cp[2 * r + 1] = 0.0;
    }
    if (done) return;
    const double rzn = sum_partials(part_rz, count, r, sh);
    if (threadIdx.x != 0) return;
    if (!(rzn > 0.0) || !isfinite(rzn)) {
        sc[r].done = 1;
        return;
    }
    cp[2 * r + 1] = rzn / sc[r].rz;
    sc[r].rz = rzn;
    if (sqrt(rzn) <= tol * sqrt(sc[r].rz0)) sc[r].done = 1;
}

// The MINRES vector updates, fused with the scalar steps that give their
// coefficients: every workgroup finishes the dot products from the
// per-block partials (the same fixed-order sum in each) and forms the
// coefficients itself, so no separate scalar launch is needed.
//   Lanczos step (minres_a_core): delta from (Kz.z); v_new = cv . (Kz, v, v_old).
//   Rotation step (minres_b_core): gamma_new, the Givens rotation and the
//               shift from (z_new.v_new); w_new = cw . (z, w_old, w) and
//               x += cx1 w_new.
// Each kernel applies its steps to a copy of the state read from sc_in;
// workgroup 0 writes the new state to sc_out (a second buffer, so no
// workgroup reads a half-updated state) and to the host mirror.
// Thread t sums partials t, t + VT, ... of set a, then of set b; the block
// sum of those is valid in thread 0.  The order depends only on the counts.
__device__ __forceinline__ double sum_block_partials(Partials a, Partials b, int r, double* sh) {
    double s = 0.0;
    s = strided_sum(a.part + r * a.count, a.count, s);
    if (b.part) s = strided_sum(b.part + r * b.count, b.count, s);
    return block_sum(s, sh);
}

__global__ void k_minres_w(long long n, long long ld, const double* z, const double* wo,
                           const double* w, double* wn, double* x, const MinresScalars* sc_in,
                           MinresScalars* sc_out, Partials pa, Partials pb, double tol,
                           double bd_tol, MinresScalars* mirror) {
    __shared__ double sh[VT / 64];
    __shared__ double cw[3], cx[2];
    const int r = blockIdx.y;
    const double d = sum_block_partials(pa, pb, r, sh);
    if (threadIdx.x == 0) {
        MinresScalars m = sc_in[r];
        minres_b_core(m, d, cw, cx, tol, bd_tol);
        if (blockIdx.x == 0) {
            sc_out[r] = m;
            if (mirror) mirror[r] = m;
        }
    }
    __syncthreads();
    const double c0 = cw[0], c1 = cw[1], c2 = cw[2], d0 = cx[0], d1 = cx[1];
    const long long off = (long long)r * ld;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) {
        const double v = c0 * z[off + i] + c1 * wo[off + i] + c2 * w[off + i];
        wn[off + i] = v;
        x[off + i] = d0 * x[off + i] + d1 * v;
    }
}

// Iteration j's v update and iteration j-1's rotation and w/x update (the
// work of k_minres_w) in one launch.  Both come after the partials they
// need (j-1's (z.v) from its P_k, j's (Kz.z) from its dot) and before
// iteration j's P_k, which overwrites j-1's z; so every workgroup applies
// the rotation of j-1 (when pa.part is set) and then the Lanczos step of j
// to its copy of the state, in that order, and updates its slice of w_new,
// x and v_new.  Workgroup 0 writes the state to sc_out and to the host
// mirror.
__global__ void k_minres_wv(long long n, long long ld, const double* kz, const double* v,
                            const double* vo, double* vn, const double* z, const double* wo,
                            const double* w, double* wn, double* x, const MinresScalars* sc_in,
                            MinresScalars* sc_out, Partials pkz, Partials pa, Partials pb,
                            double tol, double bd_tol, MinresScalars* mirror) {
    __shared__ double sh[2][VT / 64];
    __shared__ double cv[3], cw[3], cx[2];
    const int r = blockIdx.y;
    const bool prev = pa.part != nullptr;
    const long long off = (long long)r * ld;
    const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long st = (long long)gridDim.x * blockDim.x;
    // this thread's first element of every vector and the state are loaded
    // before the partial sums, so that their latencies overlap
    double e_kz = 0.0, e_v = 0.0, e_vo = 0.0, e_z = 0.0, e_wo = 0.0, e_w = 0.0, e_x = 0.0;
    if (i0 < n) {
        e_kz = kz[off + i0];
        e_v = v[off + i0];
        e_vo = vo[off + i0];
        if (prev) {
            e_z = z[off + i0];
            e_wo = wo[off + i0];
            e_w = w[off + i0];
            e_x = x[off + i0];
        }
    }
    MinresScalars m{};
    if (threadIdx.x == 0) m = sc_in[r];
    // both dot products in one reduction, each in the order of
    // sum_block_partials: this thread's strided partials (set a, then set
    // b), the wave tree, then the waves in order
    // (the first two strided partials of every set are loaded together
    // before any is added: a loop per set would wait for each in turn)
    double fa[2] = {0.0, 0.0}, fb[2] = {0.0, 0.0}, fk[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const long long q = threadIdx.x + u * VT;
        if (prev) {
            fa[u] = pa.part[r * pa.count + (q < pa.count ? q : 0)];
            if (pb.part) fb[u] = pb.part[r * pb.count + (q < pb.count ? q : 0)];
        }
        fk[u] = pkz.part[r * pkz.count + (q < pkz.count ? q : 0)];
    }
    double szv = 0.0, skz = 0.0;
    if (prev) {
#pragma unroll
        for (int u = 0; u < 2; ++u)
            if (threadIdx.x + u * VT < pa.count) szv += fa[u];
        for (long long q = threadIdx.x + 2 * VT; q < pa.count; q += VT) szv += pa.part[r * pa.count + q];
        if (pb.part) {
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (threadIdx.x + u * VT < pb.count) szv += fb[u];
            for (long long q = threadIdx.x + 2 * VT; q < pb.count; q += VT)
                szv += pb.part[r * pb.count + q];
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
        if (threadIdx.x + u * VT < pkz.count) skz += fk[u];
    for (long long q = threadIdx.x + 2 * VT; q < pkz.count; q += VT) skz += pkz.part[r * pkz.count + q];
    szv = wave_sum(szv);
    skz = wave_sum(skz);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][wave] = szv;
        sh[1][wave] = skz;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double dzv = 0.0, dkz = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) dzv += sh[0][k];
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) dkz += sh[1][k];
        if (prev) minres_b_core(m, dzv, cw, cx, tol, bd_tol);
        minres_a_core(m, dkz, cv);
        if (blockIdx.x == 0) {
            sc_out[r] = m;
            if (mirror) mirror[r] = m;
        }
    }
    __syncthreads();
    const double c0 = cv[0], c1 = cv[1], c2 = cv[2];
    if (prev) {
        const double f0 = cw[0], f1 = cw[1], f2 = cw[2], d0 = cx[0], d1 = cx[1];
        if (i0 < n) {
            const double t = f0 * e_z + f1 * e_wo + f2 * e_w;
            wn[off + i0] = t;
            x[off + i0] = d0 * e_x + d1 * t;
            vn[off + i0] = c0 * e_kz + c1 * e_v + c2 * e_vo;
        }
        for (long long i = i0 + st; i < n; i += st) {
            const double t = f0 * z[off + i] + f1 * wo[off + i] + f2 * w[off + i];
            wn[off + i] = t;
            x[off + i] = d0 * x[off + i] + d1 * t;
            vn[off + i] = c0 * kz[off + i] + c1 * v[off + i] + c2 * vo[off + i];
        }
    } else {
        if (i0 < n) vn[off + i0] = c0 * e_kz + c1 * e_v + c2 * e_vo;
        for (long long i = i0 + st; i < n; i += st)
            vn[off + i] = c0 * kz[off + i] + c1 * v[off + i] + c2 * vo[off + i];
    }
}

}  // namespace

hipError_t minres_init(hipStream_t s, MinresScalars* sc, const double* part,
                       const double* part_ref, int count, double tol, int nrhs) {
    hipLaunchKernelGGL(k_minres_init, dim3(nrhs), dim3(VT), 0, s, sc, part, part_ref, count, tol);
    return hipGetLastError();
}
hipError_t minres_w(hipStream_t s, long long n, long long ld, int nrhs, const double* z,
                    const double* wo, const double* w, double* wn, double* x,
                    const MinresScalars* sc_in, MinresScalars* sc_out, Partials a, Partials b,
                    double tol, double bd_tol, MinresScalars* mirror) {
    hipLaunchKernelGGL(k_minres_w, dim3(grid_for(n), nrhs), dim3(VT), 0,
                       s, n, ld, z, wo, w, wn, x, sc_in, sc_out, a, b, tol, bd_tol, mirror);
    return hipGetLastError();
}
hipError_t minres_wv(hipStream_t s, long long n, long long ld, int nrhs, const double* kz,
                     const double* v, const double* vo, double* vn, const double* z,
                     const double* wo, const double* w, double* wn, double* x,
                     const MinresScalars* sc_in, MinresScalars* sc_out, Partials pkz, Partials a,
                     Partials b, double tol, double bd_tol, MinresScalars* mirror) {
    hipLaunchKernelGGL(k_minres_wv, dim3(grid_for(n), nrhs), dim3(VT), 0, s, n, ld, kz, v, vo, vn,
                       z, wo, w, wn, x, sc_in, sc_out, pkz, a, b, tol, bd_tol, mirror);
    return hipGetLastError();
}
long long vec_dot_partial_count(long long n) { return dot_blocks(n); }
hipError_t cg_init(hipStream_t s, CgScalars* sc, const double* part, int count, int nrhs) {
    hipLaunchKernelGGL(k_cg_init, dim3(nrhs), dim3(VT), 0, s, sc, part, count);
    return hipGetLastError();
}
hipError_t cg_alpha(hipStream_t s, CgScalars* sc, const double* part, int count, double* cx,
                    double* cr, int nrhs) {
    hipLaunchKernelGGL(k_cg_alpha, dim3(nrhs), dim3(VT), 0, s, sc, part, count, cx, cr);
    return hipGetLastError();
}
hipError_t cg_beta(hipStream_t s, CgScalars* sc, const double* part, int count, double* cp,
                   double tol, int nrhs) {
    hipLaunchKernelGGL(k_cg_beta, dim3(nrhs), dim3(VT), 0, s, sc, part, count, cp, tol);
    return hipGetLastError();
}
hipError_t vec_dot_partials(hipStream_t s, long long n, long long ld, const double* X,
                            const double* Y, int nrhs, double* partial) {
    dot_partial_launch(s, n, ld, X, 0LL, 1, Y, nrhs, partial);
    return hipGetLastError();
}

}  // namespace hp

// =====================================================================================
// FGMRES(m) with device-resident Hessenberg matrix, Givens rotations and
// least-squares solve (one thread per right-hand side).  Iteration j of a
// restart cycle is a fixed launch sequence (its j is a kernel argument), so
// the m iterations are captured as m graphs and replayed.
namespace hp {
namespace {

__global__ void k_fg_init(FgScalars* sc, const double* part_bb, int count) {
    __shared__ double sh[VT / 64];
    const int r = blockIdx.x;
    const double bb = sum_partials(part_bb, count, r, sh);
    if (threadIdx.x != 0) return;
    FgScalars& s = sc[r];
    s = FgScalars{};
    s.bnorm = sqrt(bb);
    s.done = (s.bnorm == 0.0);
    s.rel = s.done ? 0.0 : 1.0;
    if (!isfinite(s.bnorm)) {
        s.status = -7;
        s.done = 1;
    }
}

// cycle start: w = b - K x;  beta = ||w||, g = beta e1, vscale = 1/beta
__global__ void k_fg_begin(FgScalars* sc, const double* part_ww, int count, double* g,
                           double* vscale, int m) {
    __shared__ double sh[VT / 64];
    const int r = blockIdx.x;
    const double ww = sum_partials(part_ww, count, r, sh);
    if (threadIdx.x != 0) return;
    FgScalars& s = sc[r];
    const double beta = sqrt(ww);
    double* gr = g + (long long)r * (m + 1);
    for (int i = 0; i <= m; ++i) gr[i] = 0.0;
    s.jr = 0;
    if (!s.done && !isfinite(beta)) {  // b - K x_0 not finite
        s.status = -7;
        s.done = 1;
    }
    s.active = !s.done && beta > 0.0;
    gr[0] = s.active ? beta : 0.0;
    vscale[r] = s.active ? 1.0 / beta : 0.0;
}

// Gram-Schmidt pass: h_i = <V_i, w> for i <= j; H[:, j] (+)= h.  One
// workgroup per (i, rhs) sums that pair's partials as a block reduction (a
// fixed order: the partials strided over the threads, then the wave and
// workgroup trees).
__global__ void k_fg_h(FgScalars* sc, const double* part, int count, double* H, double* hcoef,
                       int j, int pass, int m) {
    __shared__ double sh[VT / 64];
    const int i = blockIdx.x, r = blockIdx.y;
    const long long base = ((long long)r * (j + 1) + i) * count;
    double hs = 0.0;
    hs = strided_sum(part + base, count, hs);
    const double h = block_sum(hs, sh);
    if (threadIdx.x != 0) return;
    const bool active = sc[r].active;
    double* Hr = H + (long long)r * (m + 1) * m;
    if (active) Hr[i * m + j] = (pass == 0 ? 0.0 : Hr[i * m + j]) + h;
    hcoef[(long long)r * (m + 1) + i] = active ? h : 0.0;
}

// h_{j+1,j} = ||w||, previous rotations on column j, new rotation, residual estimate
__device__ void fg_rot_one(FgScalars* sc, double ww, double* H, double* cs, double* sn,
                           double* g, double* vscale, double tol, double bd_tol, int j, int m,
                           int r) {
    FgScalars& s = sc[r];
    if (!s.active) {
        vscale[r] = 0.0;
        return;
    }
    double* Hr = H + (long long)r * (m + 1) * m;
    double* cr = cs + (long long)r * m;
    double* sr = sn + (long long)r * m;
    double* gr = g + (long long)r * (m + 1);
    const double hn = sqrt(ww);
    Hr[(j + 1) * m + j] = hn;
    double col2 = ww;  // squared 2-norm of column j (the rotations keep it)
    for (int i = 0; i <= j; ++i) col2 += Hr[i * m + j] * Hr[i * m + j];
    for (int i = 0; i < j; ++i) {
        const double t = cr[i] * Hr[i * m + j] + sr[i] * Hr[(i + 1) * m + j];
        Hr[(i + 1) * m + j] = -sr[i] * Hr[i * m + j] + cr[i] * Hr[(i + 1) * m + j];
        Hr[i * m + j] = t;
    }
    const double d = hypot(Hr[j * m + j], Hr[(j + 1) * m + j]);
    if (!isfinite(col2) || !isfinite(d)) {
        s.status = -7;
        s.active = 0;
        s.done = 1;
        vscale[r] = 0.0;
        return;
    }
    // breakdown: the rotated pivot vanishes against its column (bd_tol = 0:
    // exactly zero, a singular least-squares problem)
    if (d <= bd_tol * sqrt(col2)) {
        s.status = -5;
        s.active = 0;
        s.done = 1;
        vscale[r] = 0.0;
        return;
    }
    cr[j] = Hr[j * m + j] / d;
    sr[j] = Hr[(j + 1) * m + j] / d;
    Hr[j * m + j] = d;
    Hr[(j + 1) * m + j] = 0.0;
    gr[j + 1] = -sr[j] * gr[j];
    gr[j] = cr[j] * gr[j];
    s.jr = j + 1;
    s.iters += 1;
    s.rel = fabs(gr[j + 1]) / s.bnorm;
    if (s.rel <= tol || hn == 0.0) s.active = 0;
    vscale[r] = s.active ? 1.0 / hn : 0.0;
}

// mirror: host-mapped copy of the scalars (may be null), refreshed after the step.
// One workgroup per rhs: ||w||^2 from its partials as a block reduction, then
// the rotations in thread 0.
__global__ void k_fg_rot(FgScalars* sc, const double* part_ww, int count, double* H, double* cs,
                         double* sn, double* g, double* vscale, double tol, double bd_tol, int j,
                         int m, FgScalars* mirror) {
    __shared__ double sh[VT / 64];
    const int r = blockIdx.x;
    double ws = 0.0;
    ws = strided_sum(part_ww + (long long)r * count, count, ws);
    const double ww = block_sum(ws, sh);
    if (threadIdx.x != 0) return;
    fg_rot_one(sc, ww, H, cs, sn, g, vscale, tol, bd_tol, j, m, r);
    if (mirror) mirror[r] = sc[r];
}

// y = H(1:jr,1:jr)^{-1} g(1:jr), zero beyond jr (padded to jmax)
__global__ void k_fg_solve(const FgScalars* sc, const double* H, const double* g, double* y, int m,
                           int jmax, int nrhs) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    const int jj = sc[r].jr;
    const double* Hr = H + (long long)r * (m + 1) * m;
    const double* gr = g + (long long)r * (m + 1);
    double* yr = y + (long long)r * m;
    for (int i = jj; i < jmax; ++i) yr[i] = 0.0;
    for (int i = jj - 1; i >= 0; --i) {
        double t = gr[i];
        for (int l = i + 1; l < jj; ++l) t -= Hr[i * m + l] * yr[l];
        yr[i] = t / Hr[i * m + i];
    }
}

// cycle end: relative true residual
__global__ void k_fg_check(FgScalars* sc, const double* part_rr, int count, double tol) {
    __shared__ double sh[VT / 64];
    const int r = blockIdx.x;
    if (sc[r].done) return;  // the same in every thread of the workgroup
    const double rr = sum_partials(part_rr, count, r, sh);
    if (threadIdx.x != 0) return;
    FgScalars& s = sc[r];
    s.rel = sqrt(rr) / s.bnorm;
    if (!isfinite(s.rel)) {
        s.status = -7;
        s.done = 1;
    }
    if (s.rel <= tol) s.done = 1;
}

inline dim3 rhs_block(int nrhs) { return dim3(64 * ((nrhs + 63) / 64)); }

}  // namespace

hipError_t fg_init(hipStream_t s, FgScalars* sc, const double* part, int count, int nrhs) {
    hipLaunchKernelGGL(k_fg_init, dim3(nrhs), dim3(VT), 0, s, sc, part, count);
    return hipGetLastError();
}
hipError_t fg_begin(hipStream_t s, FgScalars* sc, const double* part, int count, double* g,
                    double* vscale, int m, int nrhs) {
    hipLaunchKernelGGL(k_fg_begin, dim3(nrhs), dim3(VT), 0, s, sc, part, count, g, vscale, m);
    return hipGetLastError();
}
hipError_t fg_h(hipStream_t s, FgScalars* sc, const double* part, int count, double* H,
                double* hcoef, int j, int pass, int m, int nrhs) {
    hipLaunchKernelGGL(k_fg_h, dim3(j + 1, nrhs), dim3(VT), 0, s, sc, part, count, H, hcoef, j,
                       pass, m);
    return hipGetLastError();
}
hipError_t fg_rot(hipStream_t s, FgScalars* sc, const double* part, int count, double* H,
                  double* cs, double* sn, double* g, double* vscale, double tol, double bd_tol,
                  int j, int m, int nrhs, FgScalars* mirror) {
    hipLaunchKernelGGL(k_fg_rot, dim3(nrhs), dim3(VT), 0, s, sc, part, count, H, cs, sn, g, vscale,
                       tol, bd_tol, j, m, mirror);
    return hipGetLastError();
}
hipError_t fg_solve(hipStream_t s, const FgScalars* sc, const double* H, const double* g, double* y,
                    int m, int jmax, int nrhs) {
    hipLaunchKernelGGL(k_fg_solve, dim3(1), rhs_block(nrhs), 0, s, sc, H, g, y, m, jmax, nrhs);
    return hipGetLastError();
}
hipError_t fg_check(hipStream_t s, FgScalars* sc, const double* part, int count, double tol,
                    int nrhs) {
    hipLaunchKernelGGL(k_fg_check, dim3(nrhs), dim3(VT), 0, s, sc, part, count, tol);
    return hipGetLastError();
}
hipError_t vec_multidot_partials(hipStream_t s, long long n, long long ld, const double* X,
                                 long long xstride, int npair, const double* Y, int nrhs,
                                 double* partial) {
    dot_partial_launch(s, n, ld, X, xstride, npair, Y, nrhs, partial);
    return hipGetLastError();
}

}  // namespace hp
