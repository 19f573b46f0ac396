// Sum-factorised application of the Stokes saddle-point operator
// (Sec. 3.3, eq. systemmatrix) on gfx950.
//
// With the difference identity C^ = D^T M^ (App. B.1, eq. reduction) the
// blocks of Sec. 3.3 factor as
//     B = D^T M_q,   B^T = M_q D,   A = nu L + nu D^T M_q D,
//     L_1 = M^ (x) M^ (x) K + 2 M^ (x) T^ (x) M + 2 T^ (x) M^ (x) M   (dir 3 (x) dir 2 (x) dir 1)
// (L_2, L_3 by permuting directions), M_q = M^ (x) M^ (x) M^ and D the
// +-1 coefficient difference (the discrete divergence, App. B.2).  Hence
//     K [u; p] = [ nu L u + D^T M_q (nu D u + p) ;  M_q D u ].
// Every factor is banded (half-width p for the degree-p factors, p-1 for
// the degree p-1 ones), so one application costs O(N p) flops.
//
// Three kernels:
//   xy : per (row strip, i3-plane, field): directions 1 and 2 of every
//        Kronecker term, staged through LDS.  Velocity component c yields two
//        partial sums Ga, Gb grouped by their direction-3 factor; the pressure
//        field forms g = D u and z = nu g + p on the fly and yields M^ (x) M^ g,
//        M^ (x) M^ z.
//   zp : direction 3 for the pressure: y_p = M^_3 G_g, w = M^_3 G_z.
//   zv : direction 3 for the velocity and the coupling:
//        y_c = nu (A3a Ga + A3b Gb) + D_c^T w, with an axpby epilogue.
#include "hp_internal.h"

namespace hp {

namespace {

constexpr int XY_ROWS = 8;      // output rows (direction 2) per xy workgroup
constexpr int XY_THREADS = 256;
constexpr int Z_THREADS = 256;

struct OpArgs {
    BandTables bt;
    const double* u[3];  // velocity inputs (may be null)
    const double* p;     // pressure input (may be null)
    long long su, sp;    // per-rhs strides of the inputs (applied to all u blocks / p)
    double* ws;          // workspace base
    long long ws_stride;  // per-rhs workspace stride
    long long wsGa[3], wsGb[3], wsGg, wsGz, wsW;  // workspace offsets
    int dims[4][3];
    int nN, nM;
    double nu;
    int mode;
};

__device__ __forceinline__ double band_at(const double* tab, int w, int row, int t) {
    return tab[row * (2 * w + 1) + t];
}

// direction-1 banded product of one row held in LDS: out[i] = sum_t A[i][t] in[i+t-w]
__device__ __forceinline__ double dir1(const double* tab, int w, const double* row, int n1,
                                       int i) {
    double s = 0.0;
    for (int t = 0; t <= 2 * w; ++t) {
        int j = i + t - w;
        if (j >= 0 && j < n1) s += tab[i * (2 * w + 1) + t] * row[j];
    }
    return s;
}

template <int P>
__global__ __launch_bounds__(XY_THREADS) void k_xy(OpArgs a) {
    extern __shared__ double lds[];
    const int f = blockIdx.z & 3;
    const int r = blockIdx.z >> 2;
    const int k = blockIdx.y;
    const int j0 = blockIdx.x * XY_ROWS;
    const int WN = P, WM = P - 1;
    const int mode = a.mode;
    const BandTables& bt = a.bt;
    double* ws = a.ws + (long long)r * a.ws_stride;

    if (f < 3) {
        if (mode != OP_K && mode != OP_A && mode != OP_MV) return;
        const int c = f;
        const int n1 = a.dims[c][0], n2 = a.dims[c][1], n3 = a.dims[c][2];
        if (k >= n3 || j0 >= n2) return;
        const int w1 = (c == 0) ? WN : WM;
        const int w2 = (c == 1) ? WN : WM;
        const int R = XY_ROWS + 2 * w2;
        const int rows_out = min(XY_ROWS, n2 - j0);
        double* xs = lds;
        double* pa = xs + R * n1;
        double* pb = pa + R * n1;
        const double* x = a.u[c] + (long long)r * a.su + (long long)k * n1 * n2;
        for (int idx = threadIdx.x; idx < R * n1; idx += blockDim.x) {
            int jj = idx / n1, i = idx - jj * n1;
            int j = j0 - w2 + jj;
            xs[idx] = (j >= 0 && j < n2) ? x[(long long)j * n1 + i] : 0.0;
        }
        __syncthreads();
        const bool mv = (mode == OP_MV);
        const double* t1a = bt.ptr[c == 0 ? (mv ? BM_N : BK_N) : BM_C];
        const double* t1b = bt.ptr[c == 0 ? BM_N : BT_C];
        for (int idx = threadIdx.x; idx < R * n1; idx += blockDim.x) {
            int jj = idx / n1, i = idx - jj * n1;
            const double* row = xs + jj * n1;
            pa[idx] = dir1(t1a, w1, row, n1, i);
            if (!mv) pb[idx] = dir1(t1b, w1, row, n1, i);
        }
        __syncthreads();
        double* Ga = ws + a.wsGa[c] + (long long)k * n1 * n2;
        double* Gb = ws + a.wsGb[c] + (long long)k * n1 * n2;
        for (int idx = threadIdx.x; idx < rows_out * n1; idx += blockDim.x) {
            int jo = idx / n1, i = idx - jo * n1;
            int j = j0 + jo;
            double ga = 0.0, gb = 0.0;
            const int W = 2 * w2 + 1;
            for (int t = 0; t < W; ++t) {
                const int jj = jo + t;  // row j + t - w2 in strip coordinates
                const double xa = pa[jj * n1 + i];
                if (mv) {
                    ga += bt.ptr[c == 1 ? BM_N : BM_C][j * W + t] * xa;
                    continue;
                }
                const double xb = pb[jj * n1 + i];
                if (c == 0) {
                    const double m = bt.ptr[BM_C][j * W + t], tt = bt.ptr[BT_C][j * W + t];
                    ga += m * xa + 2.0 * tt * xb;
                    gb += 2.0 * m * xb;
                } else if (c == 1) {
                    const double kk = bt.ptr[BK_N][j * W + t], mm = bt.ptr[BM_N][j * W + t];
                    ga += kk * xa + 2.0 * mm * xb;
                    gb += 2.0 * mm * xa;
                } else {
                    const double m = bt.ptr[BM_C][j * W + t], tt = bt.ptr[BT_C][j * W + t];
                    ga += m * xa;
                    gb += 2.0 * (tt * xa + m * xb);
                }
            }
            Ga[(long long)j * n1 + i] = ga;
            if (!mv) Gb[(long long)j * n1 + i] = gb;
        }
    } else {
        // pressure field: g = D u, z = nu g + p, then M^ (x) M^ on both
        if (mode == OP_MV) return;
        const bool need_g = (mode == OP_K || mode == OP_BT);
        const bool need_z = (mode != OP_BT);
        const bool use_u = (mode != OP_B);
        const int nM = a.nM, nN = a.nN;
        if (k >= nM || j0 >= nM) return;
        const int w = WM;
        const int R = XY_ROWS + 2 * w;
        const int rows_out = min(XY_ROWS, nM - j0);
        double* gs = lds;
        double* zs = gs + R * nM;
        double* pg = zs + R * nM;
        double* pz = pg + R * nM;
        const double* u1 = use_u ? a.u[0] + (long long)r * a.su : nullptr;
        const double* u2 = use_u ? a.u[1] + (long long)r * a.su : nullptr;
        const double* u3 = use_u ? a.u[2] + (long long)r * a.su : nullptr;
        const double* pp = (mode == OP_K || mode == OP_B) ? a.p + (long long)r * a.sp : nullptr;
        for (int idx = threadIdx.x; idx < R * nM; idx += blockDim.x) {
            int jj = idx / nM, i = idx - jj * nM;
            int j = j0 - w + jj;
            double g = 0.0, z = 0.0;
            if (j >= 0 && j < nM) {
                if (use_u) {
                    // u1: (nN, nM, nM); u2: (nM, nN, nM); u3: (nM, nM, nN)
                    if (i < nN) g += u1[i + (long long)nN * (j + (long long)nM * k)];
                    if (i >= 1) g -= u1[(i - 1) + (long long)nN * (j + (long long)nM * k)];
                    if (j < nN) g += u2[i + (long long)nM * (j + (long long)nN * k)];
                    if (j >= 1) g -= u2[i + (long long)nM * ((j - 1) + (long long)nN * k)];
                    if (k < nN) g += u3[i + (long long)nM * (j + (long long)nM * k)];
                    if (k >= 1) g -= u3[i + (long long)nM * (j + (long long)nM * (k - 1))];
                }
                if (mode == OP_K) z = a.nu * g + pp[i + (long long)nM * (j + (long long)nM * k)];
                else if (mode == OP_A) z = a.nu * g;
                else if (mode == OP_B) z = pp[i + (long long)nM * (j + (long long)nM * k)];
            }
            gs[idx] = g;
            zs[idx] = z;
        }
        __syncthreads();
        const double* tm = bt.ptr[BM_C];
        for (int idx = threadIdx.x; idx < R * nM; idx += blockDim.x) {
            int jj = idx / nM, i = idx - jj * nM;
            if (need_g) pg[idx] = dir1(tm, w, gs + jj * nM, nM, i);
            if (need_z) pz[idx] = dir1(tm, w, zs + jj * nM, nM, i);
        }
        __syncthreads();
        double* Gg = ws + a.wsGg + (long long)k * nM * nM;
        double* Gz = ws + a.wsGz + (long long)k * nM * nM;
        const int W = 2 * w + 1;
        for (int idx = threadIdx.x; idx < rows_out * nM; idx += blockDim.x) {
            int jo = idx / nM, i = idx - jo * nM;
            int j = j0 + jo;
            double sg = 0.0, sz = 0.0;
            for (int t = 0; t < W; ++t) {
                const double m = tm[j * W + t];
                sg += m * pg[(jo + t) * nM + i];
                sz += m * pz[(jo + t) * nM + i];
            }
            if (need_g) Gg[(long long)j * nM + i] = sg;
            if (need_z) Gz[(long long)j * nM + i] = sz;
        }
    }
}

// direction 3 for the pressure: y_p = M^_3 G_g (modes K, BT), w = M^_3 G_z
template <int P>
__global__ __launch_bounds__(Z_THREADS) void k_zp(OpArgs a, double* yp, long long syp) {
    const int r = blockIdx.y;
    const int nM = a.nM;
    const long long nQ = (long long)nM * nM * nM;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nQ) return;
    const int w = P - 1, W = 2 * w + 1;
    const long long plane = (long long)nM * nM;
    const int k = (int)(idx / plane);
    const double* ws = a.ws + (long long)r * a.ws_stride;
    const double* tm = a.bt.ptr[BM_C];
    const bool need_g = (a.mode == OP_K || a.mode == OP_BT);
    const bool need_z = (a.mode != OP_BT);
    double sg = 0.0, sz = 0.0;
    for (int t = 0; t < W; ++t) {
        const int kk = k + t - w;
        if (kk < 0 || kk >= nM) continue;
        const double m = tm[k * W + t];
        const long long src = idx + (long long)(t - w) * plane;
        if (need_g) sg += m * ws[a.wsGg + src];
        if (need_z) sz += m * ws[a.wsGz + src];
    }
    if (need_g) yp[(long long)r * syp + idx] = sg;
    if (need_z) a.ws[(long long)r * a.ws_stride + a.wsW + idx] = sz;
}

// direction 3 for the velocity + D^T w; y = alpha * v + beta * src
template <int P>
__global__ __launch_bounds__(Z_THREADS) void k_zv(OpArgs a, Fields out, Fields src, double alpha,
                                                  double beta) {
    const int c = blockIdx.y;
    const int r = blockIdx.z;
    const int n1 = a.dims[c][0], n2 = a.dims[c][1], n3 = a.dims[c][2];
    const long long nc = (long long)n1 * n2 * n3;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nc) return;
    const long long plane = (long long)n1 * n2;
    const int k = (int)(idx / plane);
    const long long rem = idx - (long long)k * plane;
    const int j = (int)(rem / n1);
    const int i = (int)(rem - (long long)j * n1);
    const double* ws = a.ws + (long long)r * a.ws_stride;
    double v = 0.0;
    if (a.mode == OP_MV) {
        const int w3 = (c == 2) ? P : P - 1;
        const int W = 2 * w3 + 1;
        const double* ta = a.bt.ptr[c == 2 ? BM_N : BM_C];
        const double* Ga = ws + a.wsGa[c];
        double s = 0.0;
        for (int t = 0; t < W; ++t) {
            const int kk = k + t - w3;
            if (kk < 0 || kk >= n3) continue;
            s += ta[k * W + t] * Ga[idx + (long long)(t - w3) * plane];
        }
        v = s;
    } else if (a.mode == OP_K || a.mode == OP_A) {
        const int w3 = (c == 2) ? P : P - 1;
        const int W = 2 * w3 + 1;
        const double* ta = a.bt.ptr[c == 2 ? BK_N : BM_C];
        const double* tb = a.bt.ptr[c == 2 ? BM_N : BT_C];
        const double* Ga = ws + a.wsGa[c];
        const double* Gb = ws + a.wsGb[c];
        double s = 0.0;
        for (int t = 0; t < W; ++t) {
            const int kk = k + t - w3;
            if (kk < 0 || kk >= n3) continue;
            const long long sidx = idx + (long long)(t - w3) * plane;
            s += ta[k * W + t] * Ga[sidx] + tb[k * W + t] * Gb[sidx];
        }
        v = a.nu * s;
    }
    if (a.mode != OP_BT && a.mode != OP_MV) {
        // D_c^T w: (D^T w)[j] = w[j] - w[j+1] along direction c
        const int nM = a.nM;
        const double* wv = ws + a.wsW;
        const long long wi = i + (long long)nM * (j + (long long)nM * k);
        long long step = (c == 0) ? 1 : (c == 1) ? nM : (long long)nM * nM;
        v += wv[wi] - wv[wi + step];
    }
    double* y = out.f[c] + (long long)r * out.stride[c];
    double res = alpha * v;
    if (beta != 0.0) res += beta * src.f[c][(long long)r * src.stride[c] + idx];
    y[idx] = res;
}

}  // namespace

hipError_t ops_init_attributes() {
    const int bytes = 160 * 1024;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_xy<2>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_xy<3>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_xy<4>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t launch_operator(hp_ctx* c, OpMode mode, const Fields& in, const Fields& out,
                           double alpha, double beta, const Fields* src, int nrhs) {
    OpArgs a{};
    a.bt = c->band;
    for (int i = 0; i < 3; ++i) a.u[i] = in.f[i];
    a.p = in.f[3];
    a.su = in.stride[0];
    a.sp = in.stride[3];
    a.ws = c->ws;
    const long long nV = c->nV, nQ = c->nQ;
    a.ws_stride = 2 * nV + 3 * nQ;
    for (int i = 0; i < 3; ++i) {
        a.wsGa[i] = c->off[i];
        a.wsGb[i] = nV + c->off[i];
    }
    a.wsGg = 2 * nV;
    a.wsGz = 2 * nV + nQ;
    a.wsW = 2 * nV + 2 * nQ;
    for (int b = 0; b < 4; ++b)
        for (int d = 0; d < 3; ++d) a.dims[b][d] = (int)c->dims[b][d];
    a.nN = c->nN;
    a.nM = c->nM;
    a.nu = c->nu;
    a.mode = mode;
    const int nM = c->nM;
    const int P = c->p;
    // xy
    {
        int strips = (nM + XY_ROWS - 1) / XY_ROWS;
        dim3 grid(strips, nM, 4 * nrhs);
        int R = XY_ROWS + 2 * P;
        size_t shm = (size_t)4 * R * nM * sizeof(double);
        if (P == 2) hipLaunchKernelGGL(k_xy<2>, grid, dim3(XY_THREADS), shm, c->stream, a);
        else if (P == 3) hipLaunchKernelGGL(k_xy<3>, grid, dim3(XY_THREADS), shm, c->stream, a);
        else hipLaunchKernelGGL(k_xy<4>, grid, dim3(XY_THREADS), shm, c->stream, a);
    }
    // zp
    if (mode != OP_MV) {
        dim3 grid((unsigned)((nQ + Z_THREADS - 1) / Z_THREADS), nrhs);
        double* yp = out.f[3];
        long long syp = out.stride[3];
        if (P == 2) hipLaunchKernelGGL(k_zp<2>, grid, dim3(Z_THREADS), 0, c->stream, a, yp, syp);
        else if (P == 3) hipLaunchKernelGGL(k_zp<3>, grid, dim3(Z_THREADS), 0, c->stream, a, yp, syp);
        else hipLaunchKernelGGL(k_zp<4>, grid, dim3(Z_THREADS), 0, c->stream, a, yp, syp);
    }
    // zv
    if (mode != OP_BT) {
        long long maxc = 0;
        for (int b = 0; b < 3; ++b)
            maxc = std::max(maxc, c->dims[b][0] * c->dims[b][1] * c->dims[b][2]);
        dim3 grid((unsigned)((maxc + Z_THREADS - 1) / Z_THREADS), 3, nrhs);
        Fields s = src ? *src : out;
        if (!src) beta = 0.0;
        if (P == 2) hipLaunchKernelGGL(k_zv<2>, grid, dim3(Z_THREADS), 0, c->stream, a, out, s, alpha, beta);
        else if (P == 3) hipLaunchKernelGGL(k_zv<3>, grid, dim3(Z_THREADS), 0, c->stream, a, out, s, alpha, beta);
        else hipLaunchKernelGGL(k_zv<4>, grid, dim3(Z_THREADS), 0, c->stream, a, out, s, alpha, beta);
    }
    return hipGetLastError();
}

}  // namespace hp
