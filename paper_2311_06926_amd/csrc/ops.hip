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
//   xy : per (64-column x 16-row tile, i3-plane, field): directions 1 and 2
//        of every Kronecker term, the tile and its halo staged in LDS.  Velocity component c yields two partial sums Ga,
//        Gb grouped by their direction-3 factor; the pressure field forms
//        g = D u and z = nu g + p on the fly and yields M^ (x) M^ g, M^ (x) M^ z.
//   zp : direction 3 for the pressure: y_p = M^_3 G_g, w = M^_3 G_z.
//   zv : direction 3 for the velocity and the coupling:
//        y_c = nu (A3a Ga + A3b Gb) + D_c^T w, with an axpby epilogue.
//   Both z kernels give each thread one (i1, i2) point and 8 output planes;
//   the planes and their halo are loaded into registers up front, and the
//   band coefficients are uniform across the wave.
#include "hp_internal.h"

namespace hp {

namespace {

constexpr int XY_CHUNK = 16;    // output rows (direction 2) per xy workgroup
constexpr int ZCHUNK = 8;       // output planes (direction 3) per z thread
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

// ---- xy pass -----------------------------------------------------------------------
// A workgroup owns a tile of XY_T1 direction-1 columns x XY_CHUNK direction-2
// rows of one i3-plane.  The tile plus its halo (w1 columns, w2 rows on each
// side) is staged in LDS; thread (column c, row group g) applies the
// direction-1 band with its row of coefficients held in registers, then the
// direction-2 band whose row is the same for the whole wave (rows are dealt to
// waves), so its coefficients are scalar loads.  Two barriers per tile.
constexpr int XY_T1 = 64;                 // direction-1 columns per tile
constexpr int XY_THREADS = 256;           // 4 waves = 4 row groups
constexpr int XY_GROUPS = XY_THREADS / XY_T1;

template <int P, int C>
__device__ void xy_velocity(const OpArgs& a, int r, int k, int i0, int j0, double* lds) {
    constexpr int W1 = (C == 0) ? P : P - 1;
    constexpr int W2 = (C == 1) ? P : P - 1;
    constexpr int TW = XY_T1 + 2 * W1;        // staged columns
    constexpr int TR = XY_CHUNK + 2 * W2;     // staged rows
    const int n1 = a.dims[C][0], n2 = a.dims[C][1], n3 = a.dims[C][2];
    if (k >= n3 || j0 >= n2 || i0 >= n1) return;
    const bool mv = (a.mode == OP_MV);
    double* xs = lds;                 // TR x TW
    double* pa = xs + TR * TW;        // TR x XY_T1
    double* pb = pa + TR * XY_T1;
    const double* x = a.u[C] + (long long)r * a.su + (long long)k * n1 * n2;
    for (int idx = threadIdx.x; idx < TR * TW; idx += XY_THREADS) {
        const int rr = idx / TW, cc = idx - rr * TW;
        const int j = j0 - W2 + rr, i = i0 - W1 + cc;
        xs[idx] = (j >= 0 && j < n2 && i >= 0 && i < n1) ? x[(long long)j * n1 + i] : 0.0;
    }
    const int c = threadIdx.x % XY_T1, g = threadIdx.x / XY_T1;
    const int i = i0 + c;
    const bool act = i < n1;
    const double* t1a = a.bt.ptr[C == 0 ? (mv ? BM_N : BK_N) : BM_C];
    const double* t1b = a.bt.ptr[C == 0 ? BM_N : BT_C];
    double ca[2 * W1 + 1], cb[2 * W1 + 1];
#pragma unroll
    for (int t = 0; t <= 2 * W1; ++t) {
        ca[t] = act ? t1a[i * (2 * W1 + 1) + t] : 0.0;
        cb[t] = (act && !mv) ? t1b[i * (2 * W1 + 1) + t] : 0.0;
    }
    __syncthreads();
    for (int rr = g; rr < TR; rr += XY_GROUPS) {
        const double* row = xs + rr * TW + c;
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int t = 0; t <= 2 * W1; ++t) {
            sa += ca[t] * row[t];
            sb += cb[t] * row[t];
        }
        pa[rr * XY_T1 + c] = sa;
        pb[rr * XY_T1 + c] = sb;
    }
    __syncthreads();
    if (!act) return;
    const double* m2 = a.bt.ptr[C == 1 ? BM_N : BM_C];   // mass of direction 2
    const double* k2 = a.bt.ptr[C == 1 ? BK_N : BT_C];   // K (C==1) or T^ (C==0, 2)
    double* ws = a.ws + (long long)r * a.ws_stride;
    double* Ga = ws + a.wsGa[C] + (long long)k * n1 * n2;
    double* Gb = ws + a.wsGb[C] + (long long)k * n1 * n2;
    for (int o = g; o < XY_CHUNK; o += XY_GROUPS) {
        const int j = j0 + o;
        if (j >= n2) break;
        const double* rm = m2 + j * (2 * W2 + 1);
        const double* rk = k2 + j * (2 * W2 + 1);
        double am = 0.0, ak = 0.0, bm = 0.0, bk = 0.0;
#pragma unroll
        for (int t = 0; t <= 2 * W2; ++t) {
            const double va = pa[(o + t) * XY_T1 + c], vb = pb[(o + t) * XY_T1 + c];
            am += rm[t] * va;
            ak += rk[t] * va;
            bm += rm[t] * vb;
            bk += rk[t] * vb;
        }
        double ga, gb = 0.0;
        if (mv) {
            ga = am;
        } else if (C == 0) {          // M^2 K1 + 2 T^2 M1  |  2 M^2 M1
            ga = am + 2.0 * bk;
            gb = 2.0 * bm;
        } else if (C == 1) {          // K2 M^1 + 2 M2 T^1  |  2 M2 M^1
            ga = ak + 2.0 * bm;
            gb = 2.0 * am;
        } else {                      // M^2 M^1  |  2 (T^2 M^1 + M^2 T^1)
            ga = am;
            gb = 2.0 * (ak + bm);
        }
        Ga[(long long)j * n1 + i] = ga;
        if (!mv) Gb[(long long)j * n1 + i] = gb;
    }
}

// pressure: g = D u, z = nu g + p on the tile and halo, then M^ (x) M^ on both
template <int P>
__device__ void xy_pressure(const OpArgs& a, int r, int k, int i0, int j0, double* lds) {
    constexpr int W = P - 1;
    constexpr int TW = XY_T1 + 2 * W;
    constexpr int TR = XY_CHUNK + 2 * W;
    const int mode = a.mode;
    const bool need_g = (mode == OP_K || mode == OP_BT);
    const bool need_z = (mode != OP_BT);
    const bool use_u = (mode != OP_B);
    const bool use_p = (mode == OP_K || mode == OP_B);
    const int nM = a.nM, nN = a.nN;
    if (k >= nM || j0 >= nM || i0 >= nM) return;
    double* gs = lds;              // TR x TW
    double* zs = gs + TR * TW;
    double* pg = zs + TR * TW;     // TR x XY_T1
    double* pz = pg + TR * XY_T1;
    const double* u1 = use_u ? a.u[0] + (long long)r * a.su : nullptr;
    const double* u2 = use_u ? a.u[1] + (long long)r * a.su : nullptr;
    const double* u3 = use_u ? a.u[2] + (long long)r * a.su : nullptr;
    const double* pp = use_p ? a.p + (long long)r * a.sp : nullptr;
    for (int idx = threadIdx.x; idx < TR * TW; idx += XY_THREADS) {
        const int rr = idx / TW, cc = idx - rr * TW;
        const int j = j0 - W + rr, i = i0 - W + cc;
        double g = 0.0, z = 0.0;
        if (j >= 0 && j < nM && i >= 0 && i < nM) {
            if (use_u) {
                // u1: (nN, nM, nM); u2: (nM, nN, nM); u3: (nM, nM, nN)
                const long long b1 = (long long)nN * (j + (long long)nM * k);
                if (i < nN) g += u1[b1 + i];
                if (i >= 1) g -= u1[b1 + i - 1];
                if (j < nN) g += u2[i + (long long)nM * (j + (long long)nN * k)];
                if (j >= 1) g -= u2[i + (long long)nM * ((j - 1) + (long long)nN * k)];
                if (k < nN) g += u3[i + (long long)nM * (j + (long long)nM * k)];
                if (k >= 1) g -= u3[i + (long long)nM * (j + (long long)nM * (k - 1))];
            }
            const double pv = use_p ? pp[i + (long long)nM * (j + (long long)nM * k)] : 0.0;
            z = (mode == OP_B) ? pv : a.nu * g + pv;
        }
        gs[idx] = g;
        zs[idx] = z;
    }
    const int c = threadIdx.x % XY_T1, grp = threadIdx.x / XY_T1;
    const int i = i0 + c;
    const bool act = i < nM;
    const double* tm = a.bt.ptr[BM_C];
    double cm[2 * W + 1];
#pragma unroll
    for (int t = 0; t <= 2 * W; ++t) cm[t] = act ? tm[i * (2 * W + 1) + t] : 0.0;
    __syncthreads();
    for (int rr = grp; rr < TR; rr += XY_GROUPS) {
        const double* rg = gs + rr * TW + c;
        const double* rz = zs + rr * TW + c;
        double sg = 0.0, sz = 0.0;
#pragma unroll
        for (int t = 0; t <= 2 * W; ++t) {
            sg += cm[t] * rg[t];
            sz += cm[t] * rz[t];
        }
        pg[rr * XY_T1 + c] = sg;
        pz[rr * XY_T1 + c] = sz;
    }
    __syncthreads();
    if (!act) return;
    double* ws = a.ws + (long long)r * a.ws_stride;
    double* Gg = ws + a.wsGg + (long long)k * nM * nM;
    double* Gz = ws + a.wsGz + (long long)k * nM * nM;
    for (int o = grp; o < XY_CHUNK; o += XY_GROUPS) {
        const int j = j0 + o;
        if (j >= nM) break;
        const double* rm = tm + j * (2 * W + 1);
        double sg = 0.0, sz = 0.0;
#pragma unroll
        for (int t = 0; t <= 2 * W; ++t) {
            sg += rm[t] * pg[(o + t) * XY_T1 + c];
            sz += rm[t] * pz[(o + t) * XY_T1 + c];
        }
        if (need_g) Gg[(long long)j * nM + i] = sg;
        if (need_z) Gz[(long long)j * nM + i] = sz;
    }
}

template <int P>
__global__ __launch_bounds__(XY_THREADS) void k_xy(OpArgs a) {
    extern __shared__ double lds[];
    const int f = blockIdx.z & 3;
    const int r = blockIdx.z >> 2;
    const int k = blockIdx.y;
    const int ntile1 = (a.nM + XY_T1 - 1) / XY_T1;
    const int i0 = (blockIdx.x % ntile1) * XY_T1;
    const int j0 = (blockIdx.x / ntile1) * XY_CHUNK;
    const int mode = a.mode;
    if (f < 3) {
        if (mode != OP_K && mode != OP_A && mode != OP_MV) return;
        if (f == 0) xy_velocity<P, 0>(a, r, k, i0, j0, lds);
        else if (f == 1) xy_velocity<P, 1>(a, r, k, i0, j0, lds);
        else xy_velocity<P, 2>(a, r, k, i0, j0, lds);
    } else {
        if (mode == OP_MV) return;
        xy_pressure<P>(a, r, k, i0, j0, lds);
    }
}

// ---- direction 3, pressure: y_p = M^_3 G_g, w = M^_3 G_z --------------------------
// Thread = one (i1, i2) point; it loads the ZCHUNK planes it outputs plus a
// halo of W on each side into registers, then forms the band products.
template <int P>
__global__ __launch_bounds__(Z_THREADS) void k_zp(OpArgs a, double* yp, long long syp) {
    constexpr int W = P - 1;
    constexpr int R = ZCHUNK + 2 * W;
    const int r = blockIdx.z;
    const int nM = a.nM;
    const long long plane = (long long)nM * nM;
    const long long pidx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int k0 = blockIdx.y * ZCHUNK;
    if (k0 >= nM || pidx >= plane) return;
    double* ws = a.ws + (long long)r * a.ws_stride;
    const double* tm = a.bt.ptr[BM_C];
    const bool need_g = (a.mode == OP_K || a.mode == OP_BT);
    const bool need_z = (a.mode != OP_BT);
    double g[R], z[R];
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const int kk = k0 - W + s;
        const bool in = kk >= 0 && kk < nM;
        const long long src = pidx + (long long)kk * plane;
        g[s] = (need_g && in) ? ws[a.wsGg + src] : 0.0;
        z[s] = (need_z && in) ? ws[a.wsGz + src] : 0.0;
    }
#pragma unroll
    for (int o = 0; o < ZCHUNK; ++o) {
        const int k = k0 + o;
        if (k >= nM) break;
        const double* rm = tm + k * (2 * W + 1);
        double sg = 0.0, sz = 0.0;
#pragma unroll
        for (int t = 0; t <= 2 * W; ++t) {
            sg += rm[t] * g[o + t];
            sz += rm[t] * z[o + t];
        }
        const long long o3 = pidx + (long long)k * plane;
        if (need_g) yp[(long long)r * syp + o3] = sg;
        if (need_z) ws[a.wsW + o3] = sz;
    }
}

// ---- direction 3, velocity + D^T w; y = alpha v + beta src -------------------------
template <int P, int C>
__device__ void zv_component(const OpArgs& a, const Fields& out, const Fields& src, double alpha,
                             double beta, int r) {
    constexpr int W3 = (C == 2) ? P : P - 1;
    constexpr int R = ZCHUNK + 2 * W3;
    const int n1 = a.dims[C][0], n2 = a.dims[C][1], n3 = a.dims[C][2];
    const long long plane = (long long)n1 * n2;
    const long long pidx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int k0 = blockIdx.y * ZCHUNK;
    if (k0 >= n3 || pidx >= plane) return;
    const int i = (int)(pidx % n1);
    const int j = (int)(pidx / n1);
    const double* ws = a.ws + (long long)r * a.ws_stride;
    const bool mv = (a.mode == OP_MV);
    const bool lop = (a.mode == OP_K || a.mode == OP_A);
    const bool cpl = !mv && a.mode != OP_BT;
    const double* ta = a.bt.ptr[C == 2 ? (mv ? BM_N : BK_N) : BM_C];
    const double* tb = a.bt.ptr[C == 2 ? BM_N : BT_C];
    const double* Ga = ws + a.wsGa[C];
    const double* Gb = ws + a.wsGb[C];
    const double* wv = ws + a.wsW;
    const int nM = a.nM;
    const long long wstep = (C == 0) ? 1 : (C == 1) ? nM : (long long)nM * nM;
    double* y = out.f[C] + (long long)r * out.stride[C];
    const double* sv = (beta != 0.0) ? src.f[C] + (long long)r * src.stride[C] : nullptr;
    double ga[R], gb[R];
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const int kk = k0 - W3 + s;
        const bool in = (lop || mv) && kk >= 0 && kk < n3;
        const long long sidx = pidx + (long long)kk * plane;
        ga[s] = in ? Ga[sidx] : 0.0;
        gb[s] = (in && lop) ? Gb[sidx] : 0.0;
    }
#pragma unroll
    for (int o = 0; o < ZCHUNK; ++o) {
        const int k = k0 + o;
        if (k >= n3) break;
        double v = 0.0;
        if (lop || mv) {
            const double* ra = ta + k * (2 * W3 + 1);
            const double* rb = tb + k * (2 * W3 + 1);
            double sa = 0.0, sb = 0.0;
#pragma unroll
            for (int t = 0; t <= 2 * W3; ++t) {
                sa += ra[t] * ga[o + t];
                sb += rb[t] * gb[o + t];
            }
            v = mv ? sa : a.nu * (sa + sb);
        }
        if (cpl) {
            const long long wi = i + (long long)nM * (j + (long long)nM * k);
            v += wv[wi] - wv[wi + wstep];
        }
        const long long o3 = pidx + (long long)k * plane;
        double res = alpha * v;
        if (sv) res += beta * sv[o3];
        y[o3] = res;
    }
}

template <int P>
__global__ __launch_bounds__(Z_THREADS) void k_zv(OpArgs a, Fields out, Fields src, double alpha,
                                                  double beta) {
    const int c = blockIdx.z % 3;
    const int r = blockIdx.z / 3;
    if (c == 0) zv_component<P, 0>(a, out, src, alpha, beta, r);
    else if (c == 1) zv_component<P, 1>(a, out, src, alpha, beta, r);
    else zv_component<P, 2>(a, out, src, alpha, beta, r);
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
    // xy: tiles of 64 columns x 16 rows (+ halo)
    {
        const int ntile1 = (nM + XY_T1 - 1) / XY_T1;
        const int strips = (nM + XY_CHUNK - 1) / XY_CHUNK;
        dim3 grid(ntile1 * strips, nM, 4 * nrhs);
        const int TR = XY_CHUNK + 2 * P, TW = XY_T1 + 2 * P;
        size_t shm = (size_t)(2 * TR * TW + 2 * TR * XY_T1) * sizeof(double);
        if (P == 2) hipLaunchKernelGGL(k_xy<2>, grid, dim3(XY_THREADS), shm, c->stream, a);
        else if (P == 3) hipLaunchKernelGGL(k_xy<3>, grid, dim3(XY_THREADS), shm, c->stream, a);
        else hipLaunchKernelGGL(k_xy<4>, grid, dim3(XY_THREADS), shm, c->stream, a);
    }
    // zp
    if (mode != OP_MV) {
        const long long plane = (long long)nM * nM;
        dim3 grid((unsigned)((plane + Z_THREADS - 1) / Z_THREADS),
                  (unsigned)((nM + ZCHUNK - 1) / ZCHUNK), nrhs);
        double* yp = out.f[3];
        long long syp = out.stride[3];
        if (P == 2) hipLaunchKernelGGL(k_zp<2>, grid, dim3(Z_THREADS), 0, c->stream, a, yp, syp);
        else if (P == 3) hipLaunchKernelGGL(k_zp<3>, grid, dim3(Z_THREADS), 0, c->stream, a, yp, syp);
        else hipLaunchKernelGGL(k_zp<4>, grid, dim3(Z_THREADS), 0, c->stream, a, yp, syp);
    }
    // zv
    if (mode != OP_BT) {
        const long long plane = (long long)nM * nM;  // largest plane of the three components
        dim3 grid((unsigned)((plane + Z_THREADS - 1) / Z_THREADS),
                  (unsigned)((nM + ZCHUNK - 1) / ZCHUNK), 3 * nrhs);
        Fields s = src ? *src : out;
        if (!src) beta = 0.0;
        if (P == 2) hipLaunchKernelGGL(k_zv<2>, grid, dim3(Z_THREADS), 0, c->stream, a, out, s, alpha, beta);
        else if (P == 3) hipLaunchKernelGGL(k_zv<3>, grid, dim3(Z_THREADS), 0, c->stream, a, out, s, alpha, beta);
        else hipLaunchKernelGGL(k_zv<4>, grid, dim3(Z_THREADS), 0, c->stream, a, out, s, alpha, beta);
    }
    return hipGetLastError();
}

}  // namespace hp
