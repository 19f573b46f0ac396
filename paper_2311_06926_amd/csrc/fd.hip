// Base preconditioner P_0^{-1} (Sec. 4, eq. blockdiagprecond) on MFMA.
//
// Velocity block c: the diagonal block A_cc is a generalised Kronecker sum
// (Sec. 3.3, App. A.3) of (K_int, M_int) in direction c and (T^, M^) in the
// other two.  With the generalised eigenpairs U^T M U = I, U^T K U = Lambda,
// fast diagonalisation (App. A.4) gives
//     A_cc^{-1} = (U3 (x) U2 (x) U1) diag(1 / (2 nu (l1 + l2 + l3))) (U3 (x) U2 (x) U1)^T.
// Pressure: P_{Q,0}^{-1} = 2 nu (M^^{-1})^{(x)3} (dense 1D inverses).
//
// Each mode product is a dense contraction, run as 16x16x4 MFMA tiles
// (FP64 or FP32 operands, same-precision accumulation):
//   xy : one i3-plane (n1 x n2) staged in LDS: T = L X, Y = T R (modes 1, 2)
//   z  : 64 (i1,i2)-rows x n3 staged in LDS: Y = X U3, scale, Z = Y U3^T
//        (mode 3 both ways, fused with the eigenvalue scaling)
// Forward: L = U1^T, R = U2.  Inverse: L = U1, R = U2^T.
#include "hp_internal.h"

namespace hp {

namespace {

constexpr int FD_THREADS = 256;  // 4 waves
constexpr int MAXB = 8;          // up to 128 per direction (8 tiles of 16)

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// Operand layout of both 16x16x4 forms: lane l holds A[l%16][l/16] and
// B[l/16][l%16].  Result element i of lane l is D[row(l/16, i)][l%16]; the
// row map differs between the FP64 and FP32 instructions (measured).
template <>
struct Mfma<double> {
    using V = d4;
    static __device__ __forceinline__ V mma(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int i) { return lk + 4 * i; }
};
template <>
struct Mfma<float> {
    using V = f4;
    static __device__ __forceinline__ V mma(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int i) { return 4 * lk + i; }
};

struct XYArgs {
    const void* in[4];
    void* out[4];
    long long sin[4], sout[4];  // per-rhs strides
    int dims[4][3];
    int fields_lo, fields_hi;   // field range [lo, hi)
    int inverse;                // 0: forward (U^T), 1: inverse (U)
    int accumulate;             // final output: y += result
};

template <typename T>
__device__ __forceinline__ const T* xy_left(const FDTables<T>& t, int f, int inverse) {
    if (f == 3) return t.Mi;
    if (inverse) return f == 0 ? t.UK : t.UT;
    return f == 0 ? t.UKt : t.UTt;
}
template <typename T>
__device__ __forceinline__ const T* xy_right(const FDTables<T>& t, int f, int inverse) {
    if (f == 3) return t.Mi;
    if (inverse) return f == 1 ? t.UKt : t.UTt;
    return f == 1 ? t.UK : t.UT;
}

template <typename T, typename TI, typename TO>
__global__ __launch_bounds__(FD_THREADS) void k_fd_xy(XYArgs a, FDTables<T> t) {
    using M = Mfma<T>;
    using V = typename M::V;
    extern __shared__ unsigned char smem_raw[];
    T* S = reinterpret_cast<T*>(smem_raw);
    const int nf = a.fields_hi - a.fields_lo;
    const int f = a.fields_lo + (int)(blockIdx.y % nf);
    const int r = (int)(blockIdx.y / nf);
    const int k = blockIdx.x;
    const int n1 = a.dims[f][0], n2 = a.dims[f][1], n3 = a.dims[f][2];
    if (k >= n3) return;
    const int N1 = (n1 + 15) & ~15, N2 = (n2 + 15) & ~15;
    const int ld = N1 + 1;  // column-major plane, padded leading dimension
    const int nb1 = N1 >> 4, nb2 = N2 >> 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const TI* x = reinterpret_cast<const TI*>(a.in[f]) + (long long)r * a.sin[f] +
                  (long long)k * n1 * n2;
    // load plane (zero padded)
    for (int idx = threadIdx.x; idx < N1 * N2; idx += FD_THREADS) {
        int col = idx / N1, row = idx - col * N1;
        T v = 0;
        if (row < n1 && col < n2) v = (T)x[row + (long long)col * n1];
        S[col * ld + row] = v;
    }
    __syncthreads();
    const T* L = xy_left(t, f, a.inverse);
    const T* R = xy_right(t, f, a.inverse);
    const int ldL = (f == 0) ? t.NNp : t.NMp;
    const int ldR = (f == 1) ? t.NNp : t.NMp;
    // step 1: T = L X, in place by column blocks
    for (int cb = wave; cb < nb2; cb += 4) {
        V acc[MAXB];
#pragma unroll
        for (int b = 0; b < MAXB; ++b) acc[b] = V{0, 0, 0, 0};
        for (int kk = 0; kk < N1; kk += 4) {
            const T bv = S[(cb * 16 + lr) * ld + kk + lk];
#pragma unroll
            for (int b = 0; b < MAXB; ++b)
                if (b < nb1) {
                    const T av = L[(b * 16 + lr) * ldL + kk + lk];
                    acc[b] = M::mma(av, bv, acc[b]);
                }
        }
#pragma unroll
        for (int b = 0; b < MAXB; ++b)
            if (b < nb1) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    S[(cb * 16 + lr) * ld + b * 16 + M::row(lk, i)] = acc[b][i];
            }
    }
    __syncthreads();
    // step 2: Y = T R by row blocks; result back into own rows of S
    for (int rb = wave; rb < nb1; rb += 4) {
        V acc[MAXB];
#pragma unroll
        for (int b = 0; b < MAXB; ++b) acc[b] = V{0, 0, 0, 0};
        for (int kk = 0; kk < N2; kk += 4) {
            const T av = S[(kk + lk) * ld + rb * 16 + lr];
#pragma unroll
            for (int b = 0; b < MAXB; ++b)
                if (b < nb2) {
                    const T bv = R[(kk + lk) * ldR + b * 16 + lr];
                    acc[b] = M::mma(av, bv, acc[b]);
                }
        }
#pragma unroll
        for (int b = 0; b < MAXB; ++b)
            if (b < nb2) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    S[(b * 16 + lr) * ld + rb * 16 + M::row(lk, i)] = acc[b][i];
            }
    }
    __syncthreads();
    TO* y = reinterpret_cast<TO*>(a.out[f]) + (long long)r * a.sout[f] + (long long)k * n1 * n2;
    for (int idx = threadIdx.x; idx < n1 * n2; idx += FD_THREADS) {
        int col = idx / n1, row = idx - col * n1;
        TO v = (TO)S[col * ld + row];
        if (a.accumulate) y[idx] += v;
        else y[idx] = v;
    }
}

struct ZArgs {
    const void* in[4];
    void* out[4];
    long long sin[4], sout[4];
    int dims[4][3];
    int fields_lo, fields_hi;
    int accumulate;
    double two_nu;
};

constexpr int ZROWS = 64;

template <typename T, typename TI, typename TO>
__global__ __launch_bounds__(FD_THREADS) void k_fd_z(ZArgs a, FDTables<T> t) {
    using M = Mfma<T>;
    using V = typename M::V;
    extern __shared__ unsigned char smem_raw[];
    T* S = reinterpret_cast<T*>(smem_raw);
    const int nf = a.fields_hi - a.fields_lo;
    const int f = a.fields_lo + (int)(blockIdx.y % nf);
    const int r = (int)(blockIdx.y / nf);
    const int n1 = a.dims[f][0], n2 = a.dims[f][1], n3 = a.dims[f][2];
    const long long plane = (long long)n1 * n2;
    const long long r0 = (long long)blockIdx.x * ZROWS;
    if (r0 >= plane) return;
    const int N3 = (n3 + 15) & ~15;
    const int ld = N3 + 1;  // row-major [row][k]
    const int nb3 = N3 >> 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const TI* x = reinterpret_cast<const TI*>(a.in[f]) + (long long)r * a.sin[f];
    for (int idx = threadIdx.x; idx < ZROWS * N3; idx += FD_THREADS) {
        int kk = idx / ZROWS, row = idx - kk * ZROWS;
        T v = 0;
        if (kk < n3 && r0 + row < plane) v = (T)x[r0 + row + (long long)kk * plane];
        S[row * ld + kk] = v;
    }
    __syncthreads();
    const bool pres = (f == 3);
    const T* U3 = pres ? t.Mi : (f == 2 ? t.UK : t.UT);
    const int ldU = (f == 2) ? t.NNp : t.NMp;
    T* Sw = S + wave * 16 * ld;  // this wave's 16 rows
    // Y = X U3
    V acc[MAXB];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) acc[b] = V{0, 0, 0, 0};
    for (int kk = 0; kk < N3; kk += 4) {
        const T av = Sw[lr * ld + kk + lk];
#pragma unroll
        for (int b = 0; b < MAXB; ++b)
            if (b < nb3) {
                const T bv = U3[(kk + lk) * ldU + b * 16 + lr];
                acc[b] = M::mma(av, bv, acc[b]);
            }
    }
    if (pres) {
#pragma unroll
        for (int b = 0; b < MAXB; ++b)
            if (b < nb3)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    Sw[(M::row(lk, i)) * ld + b * 16 + lr] = (T)(a.two_nu * (double)acc[b][i]);
    } else {
        // scale by 1 / (2 nu (l1 + l2 + l3)) and transform back: Z = Y U3^T
        const double* l1 = (f == 0) ? t.lamK : t.lamT;
        const double* l2 = (f == 1) ? t.lamK : t.lamT;
        const double* l3 = (f == 2) ? t.lamK : t.lamT;
#pragma unroll
        for (int b = 0; b < MAXB; ++b)
            if (b < nb3)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = M::row(lk, i);
                    const long long rr = r0 + wave * 16 + row;
                    const int col = b * 16 + lr;
                    double s = 0.0;
                    if (rr < plane && col < n3) {
                        const int i1 = (int)(rr % n1), i2 = (int)(rr / n1);
                        s = 1.0 / (a.two_nu * (l1[i1] + l2[i2] + l3[col]));
                    }
                    Sw[row * ld + col] = (T)(s * (double)acc[b][i]);
                }
        const T* U3t = (f == 2) ? t.UKt : t.UTt;
#pragma unroll
        for (int b = 0; b < MAXB; ++b) acc[b] = V{0, 0, 0, 0};
        for (int kk = 0; kk < N3; kk += 4) {
            const T av = Sw[lr * ld + kk + lk];
#pragma unroll
            for (int b = 0; b < MAXB; ++b)
                if (b < nb3) {
                    const T bv = U3t[(kk + lk) * ldU + b * 16 + lr];
                    acc[b] = M::mma(av, bv, acc[b]);
                }
        }
#pragma unroll
        for (int b = 0; b < MAXB; ++b)
            if (b < nb3)
#pragma unroll
                for (int i = 0; i < 4; ++i) Sw[(M::row(lk, i)) * ld + b * 16 + lr] = acc[b][i];
    }
    __syncthreads();
    TO* y = reinterpret_cast<TO*>(a.out[f]) + (long long)r * a.sout[f];
    for (int idx = threadIdx.x; idx < ZROWS * n3; idx += FD_THREADS) {
        int kk = idx / ZROWS, row = idx - kk * ZROWS;
        if (r0 + row >= plane) continue;
        TO v = (TO)S[row * ld + kk];
        long long o = r0 + row + (long long)kk * plane;
        if (a.accumulate) y[o] += v;
        else y[o] = v;
    }
}

template <typename T>
hipError_t run_P0(hp_ctx* c, const FDTables<T>& t, const Fields& in, const Fields& out, bool vel,
                  bool pres, bool accumulate, int nrhs) {
    // scratch for the two intermediate tensors (precision T), per rhs N values each
    const long long N = c->N;
    T* tmp1 = reinterpret_cast<T*>(c->ws + (2 * c->nV + 3 * c->nQ) * (long long)c->opts.max_rhs);
    T* tmp2 = tmp1 + N * (long long)c->opts.max_rhs;
    const int lo = vel ? 0 : 3, hi = pres ? 4 : 3;
    if (lo >= hi) return hipSuccess;
    const int nf = hi - lo;
    const int nM = c->nM;
    const int NMp = (nM + 15) & ~15;
    XYArgs xa{};
    for (int f = 0; f < 4; ++f) {
        for (int d = 0; d < 3; ++d) xa.dims[f][d] = (int)c->dims[f][d];
        xa.in[f] = in.f[f];
        xa.sin[f] = in.stride[f];
        xa.out[f] = tmp1 + c->off[f];
        xa.sout[f] = N;
    }
    xa.fields_lo = lo;
    xa.fields_hi = hi;
    xa.inverse = 0;
    xa.accumulate = 0;
    size_t shm_xy = (size_t)NMp * (NMp + 1) * sizeof(T);
    dim3 gxy(nM, nf * nrhs);
    hipLaunchKernelGGL((k_fd_xy<T, double, T>), gxy, dim3(FD_THREADS), shm_xy, c->stream, xa, t);
    ZArgs za{};
    for (int f = 0; f < 4; ++f) {
        for (int d = 0; d < 3; ++d) za.dims[f][d] = (int)c->dims[f][d];
        za.in[f] = tmp1 + c->off[f];
        za.sin[f] = N;
        za.out[f] = tmp2 + c->off[f];
        za.sout[f] = N;
    }
    za.fields_lo = lo;
    za.fields_hi = hi;
    za.accumulate = 0;
    za.two_nu = 2.0 * c->nu;
    size_t shm_z = (size_t)ZROWS * (NMp + 1) * sizeof(T);
    long long maxplane = (long long)nM * nM;
    if (vel) {
        ZArgs zv = za;
        zv.fields_lo = 0;
        zv.fields_hi = 3;
        dim3 g((unsigned)((maxplane + ZROWS - 1) / ZROWS), 3 * nrhs);
        hipLaunchKernelGGL((k_fd_z<T, T, T>), g, dim3(FD_THREADS), shm_z, c->stream, zv, t);
    }
    if (pres) {
        ZArgs zp = za;
        zp.fields_lo = 3;
        zp.fields_hi = 4;
        zp.out[3] = out.f[3];
        zp.sout[3] = out.stride[3];
        zp.accumulate = accumulate ? 1 : 0;
        dim3 g((unsigned)((maxplane + ZROWS - 1) / ZROWS), nrhs);
        hipLaunchKernelGGL((k_fd_z<T, T, double>), g, dim3(FD_THREADS), shm_z, c->stream, zp, t);
    }
    if (vel) {
        XYArgs xi = xa;
        for (int f = 0; f < 3; ++f) {
            xi.in[f] = tmp2 + c->off[f];
            xi.sin[f] = N;
            xi.out[f] = out.f[f];
            xi.sout[f] = out.stride[f];
        }
        xi.fields_lo = 0;
        xi.fields_hi = 3;
        xi.inverse = 1;
        xi.accumulate = accumulate ? 1 : 0;
        dim3 g(nM, 3 * nrhs);
        hipLaunchKernelGGL((k_fd_xy<T, T, double>), g, dim3(FD_THREADS), shm_xy, c->stream, xi, t);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t set_fd_attrs() {
    const int bytes = 160 * 1024;
    hipError_t e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fd_xy<T, double, T>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fd_xy<T, T, double>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fd_z<T, T, T>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fd_z<T, T, double>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace

hipError_t fd_init_attributes() {
    hipError_t e = set_fd_attrs<double>();
    if (e != hipSuccess) return e;
    return set_fd_attrs<float>();
}

hipError_t launch_P0(hp_ctx* c, const Fields& in, const Fields& out, bool vel, bool pres,
                     bool accumulate, int precision, int nrhs) {
    if (precision == HP_PREC_FP64) return run_P0<double>(c, c->fd64, in, out, vel, pres, accumulate, nrhs);
    return run_P0<float>(c, c->fd32, in, out, vel, pres, accumulate, nrhs);
}

}  // namespace hp
