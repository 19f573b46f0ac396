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
//        (16 rows per wave)
//        (mode 3 both ways, fused with the eigenvalue scaling)
// Forward: L = U1^T, R = U2.  Inverse: L = U1, R = U2^T.
#include <type_traits>

#include "hp_internal.h"
#include "vec.h"

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

// acc[b] += sum over k of the 16x16 tile product for output tiles b < nb:
// one operand (`s`, this lane's value at k-step base kk) is shared by all
// tiles, the other (`v(b, kk)`) differs per tile.  SHARED_A selects which of
// the two is the MFMA A operand.  Operands are fetched 16 k-values (4 MFMA
// k-steps) at a time and the next chunk is fetched while the current one
// is multiplied, so the L2 latency of the matrix operand overlaps compute.
template <typename T, bool SHARED_A, typename FS, typename FV>
__device__ __forceinline__ void mfma_row(typename Mfma<T>::V (&acc)[MAXB], int nb, int K, FS s,
                                         FV v) {
    using M = Mfma<T>;
    T sc[4], vc[4][MAXB];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        sc[u] = s(4 * u);
#pragma unroll
        for (int b = 0; b < MAXB; ++b) vc[u][b] = (b < nb) ? v(b, 4 * u) : T(0);
    }
    for (int k0 = 0; k0 < K; k0 += 16) {
        T sn[4], vn[4][MAXB];
        const bool more = k0 + 16 < K;
        if (more) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                sn[u] = s(k0 + 16 + 4 * u);
#pragma unroll
                for (int b = 0; b < MAXB; ++b) vn[u][b] = (b < nb) ? v(b, k0 + 16 + 4 * u) : T(0);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int b = 0; b < MAXB; ++b)
                if (b < nb) {
                    if (SHARED_A) acc[b] = M::mma(sc[u], vc[u][b], acc[b]);
                    else acc[b] = M::mma(vc[u][b], sc[u], acc[b]);
                }
        if (more) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                sc[u] = sn[u];
#pragma unroll
                for (int b = 0; b < MAXB; ++b) vc[u][b] = vn[u][b];
            }
        }
    }
}

struct XYArgs {
    const void* in[4];
    void* out[4];
    long long sin[4], sout[4];  // per-rhs strides
    int dims[4][3];
    int fields_lo, fields_hi;   // field range [lo, hi)
    int inverse;                // 0: forward (U^T), 1: inverse (U)
    int accumulate;             // final output: y += result
    // FP64 output only: partial sums of (stored output) . dw per (field,
    // plane) to dpart[r * dp_stride + f * dp_planes + k] (dpart null: none)
    const double* dw[4];        // same layout and rhs stride as out
    double* dpart;
    long long dp_stride;
    int dp_planes;
    // row-block kernel (k_fd_xy_s) only: row blocks per plane in its grid
    // order, and the partial of row block b goes to slot + b dp_rb
    int nrb;
    long long dp_rb;
    // FP64 input only: for a field with inb[f] set, the input is
    // ca in + cb inb + cc inc (the same layout as in, rhs strides sinb, sinc)
    const double* inb[4];
    const double* inc[4];
    long long sinb[4], sinc[4];
    double ca, cb, cc;
};

// Global-to-LDS staging and the write-outs run in batches: a thread issues
// the loads of FD_BATCH elements before it uses any of them, so that their
// latencies overlap (a load, its wait and the LDS write per element in turn
// would add them up).  Indices past the end are clamped for the load and
// their values dropped, so no load leaves the array.
constexpr int FD_BATCH = 8;

// Plane k of field f (n1 x n2 at x) into S, column-major with leading
// dimension ld, zero padded to N1 x N2.  The forward input is x itself or,
// when inb[f] is set, the combination ca x + cb inb + cc inc (the same
// layout; terms with a zero coefficient are not read), formed in the
// operation order of the vector kernel k_axpbypcz so that it equals reading
// a materialised result.
template <typename T, typename TI, int NTH>
__device__ __forceinline__ void xy_stage(const XYArgs& a, int f, const TI* x, int r,
                                         long long kofs, T* S, int ld, int n1, int n2, int N1,
                                         int N2) {
    const int n = n1 * n2;
    // the combination's three loads are issued before its arithmetic
    const double* xb = nullptr;
    const double* xc = nullptr;
    if constexpr (std::is_same<TI, double>::value) {
        if (a.inb[f]) {
            if (a.cb != 0.0) xb = a.inb[f] + (long long)r * a.sinb[f] + kofs;
            if (a.cc != 0.0) xc = a.inc[f] + (long long)r * a.sinc[f] + kofs;
        }
    }
    const bool comb = std::is_same<TI, double>::value && a.inb[f] != nullptr;
    for (int base = 0; base < n; base += FD_BATCH * NTH) {
        TI vx[FD_BATCH];
        double vb[FD_BATCH], vc[FD_BATCH];
#pragma unroll
        for (int u = 0; u < FD_BATCH; ++u) vx[u] = x[min(base + u * NTH + (int)threadIdx.x, n - 1)];
        if (xb)
#pragma unroll
            for (int u = 0; u < FD_BATCH; ++u)
                vb[u] = xb[min(base + u * NTH + (int)threadIdx.x, n - 1)];
        if (xc)
#pragma unroll
            for (int u = 0; u < FD_BATCH; ++u)
                vc[u] = xc[min(base + u * NTH + (int)threadIdx.x, n - 1)];
#pragma unroll
        for (int u = 0; u < FD_BATCH; ++u) {
            const int idx = base + u * NTH + (int)threadIdx.x;
            if (idx < n) {
                T v;
                if (comb) {
                    double c = a.ca * (double)vx[u];
                    if (xb) c += a.cb * vb[u];
                    if (xc) c += a.cc * vc[u];
                    v = (T)c;
                } else {
                    v = (T)vx[u];
                }
                const int col = idx / n1;
                S[col * ld + (idx - col * n1)] = v;
            }
        }
    }
    const int pr = N1 - n1;
    for (int idx = threadIdx.x; idx < pr * N2; idx += NTH) {
        const int col = idx / pr;
        S[col * ld + n1 + (idx - col * pr)] = T(0);
    }
    for (int idx = threadIdx.x; idx < n1 * (N2 - n2); idx += NTH) {
        const int c = idx / n1;
        S[(n2 + c) * ld + (idx - c * n1)] = T(0);
    }
}

// Rows [r0, r0 + ZR) of field f (rows of length n3 at stride `plane` in x,
// none at or past `plane`) into S, row-major with leading dimension ld, zero
// padded to N3 columns and for the missing rows.
template <typename T, typename TI, int NTH, int ZR>
__device__ __forceinline__ void z_stage(const TI* x, long long r0, long long plane, int n3,
                                        int N3, T* S, int ld) {
    const int n = ZR * n3;
    for (int base = 0; base < n; base += FD_BATCH * NTH) {
        T v[FD_BATCH];
#pragma unroll
        for (int u = 0; u < FD_BATCH; ++u) {
            const int idx = base + u * NTH + (int)threadIdx.x;
            const int kk = idx / ZR, row = idx - kk * ZR;
            const bool ok = idx < n && r0 + row < plane;
            const T e = (T)x[ok ? r0 + row + (long long)kk * plane : r0];
            v[u] = ok ? e : T(0);
        }
#pragma unroll
        for (int u = 0; u < FD_BATCH; ++u) {
            const int idx = base + u * NTH + (int)threadIdx.x;
            if (idx < n) {
                const int kk = idx / ZR, row = idx - kk * ZR;
                S[row * ld + kk] = v[u];
            }
        }
    }
    for (int idx = threadIdx.x; idx < ZR * (N3 - n3); idx += NTH) {
        const int kk = idx / ZR, row = idx - kk * ZR;
        S[row * ld + n3 + kk] = T(0);
    }
}

// The final write-out of plane k of field f from the column-major plane S
// (leading dimension ld): y = S, or y += S.  With a dot the workgroup also
// sums (stored value) x dw over the plane, a fixed-order reduction whose
// scratch reuses S once every read of it is done.
template <typename T, typename TO, int NTH>
__device__ __forceinline__ void xy_store(const XYArgs& a, T* S, int ld, int f, int r, int k,
                                         int n1, int n2) {
    TO* y = reinterpret_cast<TO*>(a.out[f]) + (long long)r * a.sout[f] + (long long)k * n1 * n2;
    const int n = n1 * n2;
    if constexpr (std::is_same<TO, double>::value) {
        if (a.dpart) {
            const double* w = a.dw[f] + (long long)r * a.sout[f] + (long long)k * n1 * n2;
            double s = 0.0;
            for (int base = 0; base < n; base += FD_BATCH * NTH) {
                double yv[FD_BATCH], wv[FD_BATCH];
#pragma unroll
                for (int u = 0; u < FD_BATCH; ++u) {
                    const int e = min(base + u * NTH + (int)threadIdx.x, n - 1);
                    yv[u] = a.accumulate ? y[e] : 0.0;
                    wv[u] = w[e];
                }
#pragma unroll
                for (int u = 0; u < FD_BATCH; ++u) {
                    const int idx = base + u * NTH + (int)threadIdx.x;
                    if (idx < n) {
                        const int col = idx / n1, row = idx - col * n1;
                        double v = (double)S[col * ld + row];
                        if (a.accumulate) v += yv[u];
                        y[idx] = v;
                        s += v * wv[u];
                    }
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
            __syncthreads();
            double* red = reinterpret_cast<double*>(S);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
            __syncthreads();
            if (threadIdx.x == 0) {
                double t = 0.0;
                for (int wv = 0; wv < NTH / 64; ++wv) t += red[wv];
                a.dpart[(long long)r * a.dp_stride + (long long)f * a.dp_planes + k] = t;
            }
            return;
        }
    }
    if (a.accumulate) {
        for (int base = 0; base < n; base += FD_BATCH * NTH) {
            TO yv[FD_BATCH];
#pragma unroll
            for (int u = 0; u < FD_BATCH; ++u) yv[u] = y[min(base + u * NTH + (int)threadIdx.x, n - 1)];
#pragma unroll
            for (int u = 0; u < FD_BATCH; ++u) {
                const int idx = base + u * NTH + (int)threadIdx.x;
                if (idx < n) {
                    const int col = idx / n1, row = idx - col * n1;
                    y[idx] = yv[u] + (TO)S[col * ld + row];
                }
            }
        }
        return;
    }
    for (int idx = threadIdx.x; idx < n; idx += NTH) {
        int col = idx / n1, row = idx - col * n1;
        y[idx] = (TO)S[col * ld + row];
    }
}

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
// the transpose of xy_right (M^^{-1} is symmetric)
template <typename T>
__device__ __forceinline__ const T* xy_right_t(const FDTables<T>& t, int f, int inverse) {
    if (f == 3) return t.Mi;
    if (inverse) return f == 1 ? t.UK : t.UT;
    return f == 1 ? t.UKt : t.UTt;
}

template <typename T, typename TI, typename TO, bool STAGE>
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
    const long long kofs = (long long)k * n1 * n2;
    const TI* x = reinterpret_cast<const TI*>(a.in[f]) + (long long)r * a.sin[f] + kofs;
    // load plane (zero padded)
    xy_stage<T, TI, FD_THREADS>(a, f, x, r, kofs, S, ld, n1, n2, N1, N2);
    __syncthreads();
    const T* L = xy_left(t, f, a.inverse);
    const T* R = xy_right(t, f, a.inverse);
    const int ldL = (f == 0) ? t.NNp : t.NMp;
    const int ldR = (f == 1) ? t.NNp : t.NMp;
    if (STAGE) {
        // small directions: the two dense 1D matrices move to LDS once
        T* Ls = S + N2 * ld;
        T* Rs = Ls + N1 * N1;
        for (int idx = threadIdx.x; idx < N1 * N1; idx += FD_THREADS) Ls[idx] = L[idx];
        for (int idx = threadIdx.x; idx < N2 * N2; idx += FD_THREADS) Rs[idx] = R[idx];
        L = Ls;
        R = Rs;
        __syncthreads();
    }
    // step 1: T = L X, in place by column blocks
    for (int cb = wave; cb < nb2; cb += 4) {
        V acc[MAXB];
#pragma unroll
        for (int b = 0; b < MAXB; ++b) acc[b] = V{0, 0, 0, 0};
        mfma_row<T, false>(
            acc, nb1, N1, [&](int kk) { return S[(cb * 16 + lr) * ld + kk + lk]; },
            [&](int b, int kk) { return L[(b * 16 + lr) * ldL + kk + lk]; });
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
        mfma_row<T, true>(
            acc, nb2, N2, [&](int kk) { return S[(kk + lk) * ld + rb * 16 + lr]; },
            [&](int b, int kk) { return R[(kk + lk) * ldR + b * 16 + lr]; });
#pragma unroll
        for (int b = 0; b < MAXB; ++b)
            if (b < nb2) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    S[(b * 16 + lr) * ld + rb * 16 + M::row(lk, i)] = acc[b][i];
            }
    }
    __syncthreads();
    xy_store<T, TO, FD_THREADS>(a, S, ld, f, r, k, n1, n2);
}

constexpr int ZROWS = 64;      // (i1,i2)-rows per z workgroup: 16 per wave

struct ZArgs {
    const void* in[4];
    void* out[4];
    long long sin[4], sout[4];
    int dims[4][3];
    int fields_lo, fields_hi;
    int accumulate;   // bit f set: field f is added to its output
    double two_nu;
    double omega;     // damping factor of P_0^{-1} (1: the plain base preconditioner)
    // FP64 output, launches of one field only: partial sums of (stored
    // output) . dw per workgroup to dpart[r * dp_stride + blockIdx.x]
    const double* dw;  // same layout and rhs stride as the output
    double* dpart;
    long long dp_stride;
};

// The final write-out of z rows [r0, r0 + ZR) of field f from the
// row-major buffer Out (leading dimension ld): y = Out or y += Out; with a
// dot also the workgroup's fixed-order sum of (stored value) x dw, whose
// scratch reuses S once every read of the LDS buffers is done.
template <typename T, typename TO, int NTH, int ZR = ZROWS>
__device__ __forceinline__ void z_store(const ZArgs& a, const T* Out, T* S, int ld, int f, int r,
                                        long long r0, long long plane, int n3) {
    TO* y = reinterpret_cast<TO*>(a.out[f]) + (long long)r * a.sout[f];
    const int n = ZR * n3;
    const bool acc = (a.accumulate >> f) & 1;
    if constexpr (std::is_same<TO, double>::value) {
        if (a.dpart) {
            const double* w = a.dw + (long long)r * a.sout[f];
            double s = 0.0;
            for (int base = 0; base < n; base += FD_BATCH * NTH) {
                double yv[FD_BATCH], wv[FD_BATCH];
#pragma unroll
                for (int u = 0; u < FD_BATCH; ++u) {
                    const int idx = base + u * NTH + (int)threadIdx.x;
                    const int kk = idx / ZR, row = idx - kk * ZR;
                    const long long o =
                        idx < n && r0 + row < plane ? r0 + row + (long long)kk * plane : r0;
                    yv[u] = acc ? y[o] : 0.0;
                    wv[u] = w[o];
                }
#pragma unroll
                for (int u = 0; u < FD_BATCH; ++u) {
                    const int idx = base + u * NTH + (int)threadIdx.x;
                    const int kk = idx / ZR, row = idx - kk * ZR;
                    if (idx < n && r0 + row < plane) {
                        const long long o = r0 + row + (long long)kk * plane;
                        double v = (double)Out[row * ld + kk];
                        if (acc) v += yv[u];
                        y[o] = v;
                        s += v * wv[u];
                    }
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
            __syncthreads();
            double* red = reinterpret_cast<double*>(S);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
            __syncthreads();
            if (threadIdx.x == 0) {
                double t = 0.0;
                for (int wv = 0; wv < NTH / 64; ++wv) t += red[wv];
                a.dpart[(long long)r * a.dp_stride + blockIdx.x] = t;
            }
            return;
        }
    }
    if (acc) {
        for (int base = 0; base < n; base += FD_BATCH * NTH) {
            TO yv[FD_BATCH];
#pragma unroll
            for (int u = 0; u < FD_BATCH; ++u) {
                const int idx = base + u * NTH + (int)threadIdx.x;
                const int kk = idx / ZR, row = idx - kk * ZR;
                yv[u] = y[idx < n && r0 + row < plane ? r0 + row + (long long)kk * plane : r0];
            }
#pragma unroll
            for (int u = 0; u < FD_BATCH; ++u) {
                const int idx = base + u * NTH + (int)threadIdx.x;
                const int kk = idx / ZR, row = idx - kk * ZR;
                if (idx < n && r0 + row < plane)
                    y[r0 + row + (long long)kk * plane] = yv[u] + (TO)Out[row * ld + kk];
            }
        }
        return;
    }
    for (int idx = threadIdx.x; idx < n; idx += NTH) {
        int kk = idx / ZR, row = idx - kk * ZR;
        if (r0 + row >= plane) continue;
        y[r0 + row + (long long)kk * plane] = (TO)Out[row * ld + kk];
    }
}


template <typename T, typename TI, typename TO, bool STAGE>
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
    z_stage<T, TI, FD_THREADS, ZROWS>(x, r0, plane, n3, N3, S, ld);
    const bool pres = (f == 3);
    const T* U3 = pres ? t.Mi : (f == 2 ? t.UK : t.UT);
    const T* U3t = pres ? t.Mi : (f == 2 ? t.UKt : t.UTt);
    const int ldU = (f == 2) ? t.NNp : t.NMp;
    if (STAGE) {
        T* Us = S + ZROWS * ld;
        T* Uts = Us + N3 * N3;
        for (int idx = threadIdx.x; idx < N3 * N3; idx += FD_THREADS) {
            Us[idx] = U3[idx];
            if (!pres) Uts[idx] = U3t[idx];
        }
        U3 = Us;
        U3t = pres ? Us : Uts;  // M^^{-1} is symmetric: one staged copy serves both
    }
    __syncthreads();
    T* Sw = S + wave * 16 * ld;  // this wave's 16 rows
    const long long w0 = r0 + wave * 16;
    // Y = X U3
    V acc[MAXB];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) acc[b] = V{0, 0, 0, 0};
    if (w0 < plane)
        mfma_row<T, true>(
            acc, nb3, N3, [&](int kk) { return Sw[lr * ld + kk + lk]; },
            [&](int b, int kk) { return U3[(kk + lk) * ldU + b * 16 + lr]; });
    if (pres) {
#pragma unroll
        for (int b = 0; b < MAXB; ++b)
            if (b < nb3)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    Sw[M::row(lk, i) * ld + b * 16 + lr] =
                        (T)(a.omega * a.two_nu * (double)acc[b][i]);
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
                    const long long rr = w0 + row;
                    const int col = b * 16 + lr;
                    double sc = 0.0;
                    if (rr < plane && col < n3) {
                        const int i1 = (int)(rr % n1), i2 = (int)(rr / n1);
                        sc = a.omega / (a.two_nu * (l1[i1] + l2[i2] + l3[col]));
                    }
                    Sw[row * ld + col] = (T)(sc * (double)acc[b][i]);
                }
#pragma unroll
        for (int b = 0; b < MAXB; ++b) acc[b] = V{0, 0, 0, 0};
        if (w0 < plane)
            mfma_row<T, true>(
                acc, nb3, N3, [&](int kk) { return Sw[lr * ld + kk + lk]; },
                [&](int b, int kk) { return U3t[(kk + lk) * ldU + b * 16 + lr]; });
#pragma unroll
        for (int b = 0; b < MAXB; ++b)
            if (b < nb3)
#pragma unroll
                for (int i = 0; i < 4; ++i) Sw[M::row(lk, i) * ld + b * 16 + lr] = acc[b][i];
    }
    __syncthreads();
    z_store<T, TO, FD_THREADS>(a, S, S, ld, f, r, r0, plane, n3);
}

// ---- tile-per-wave variants ----------------------------------------------------------
// Each wave owns one 16x16 output tile at a time (16 waves per workgroup), so
// every dependency chain is one tile's k-loop; the two GEMM steps use
// separate LDS buffers.  Used when both buffers (and, when small enough,
// the two dense 1D matrices) fit in LDS.
constexpr int FD_WIDE = 1024;   // 16 waves

// D = A B on one 16x16 tile, K <= 128 (a multiple of 16).  One operand, G,
// is stored with contiguous k: G(idx, k) = G[idx*ldg + k] (global memory or
// an LDS copy); the other, H, is in LDS: H(k, idx) = H[k*h_k + idx*h_i].
// GA: G is the A operand (rows of D), else the B operand (columns of D).
// The contraction order over k is free as long as both operands use the same
// one: in k-chunk c (16 wide), MFMA step s, lane (lr, lk) supplies
// k = 16c + 4 lk + s, so its four G values of a chunk are contiguous and
// arrive in one vector load, issued one chunk ahead of their products.
template <typename T>
struct Vec4T;
template <>
struct Vec4T<double> {
    typedef double V __attribute__((ext_vector_type(4)));
};
template <>
struct Vec4T<float> {
    typedef float V __attribute__((ext_vector_type(4)));
};

// K (the contraction length) is a multiple of 4: the full 16-wide chunks
// as above, then the remaining 4, 8 or 12 values with step s taking
// k = K16 + 4 s + lk (any assignment of k to (step, lane group) that both
// operands share gives the same sum), so that no MFMA step multiplies only
// zero padding.  Up to two chunks (K <= 44) all G values are loaded before
// the first product, the same products in the same order (at 32^3 this
// saves the waits of the second chunk and the tail: P_0 21.2 -> 21.0 us,
// 2-4 % per MINRES iteration).
template <typename T, bool GA>
__device__ __forceinline__ typename Mfma<T>::V tile_gemm(const T* G, int ldg, const T* H, int h_k,
                                                         int h_i, int K, int lr, int lk) {
    using M = Mfma<T>;
    using V4 = typename Vec4T<T>::V;
    const int K16 = K & ~15;
    const T* gp = G + lr * ldg + 4 * lk;
    const T* hp = H + lr * h_i + 4 * lk * h_k;
    typename M::V acc = {0, 0, 0, 0};
    if (K16 <= 32) {
        V4 g0 = *reinterpret_cast<const V4*>(gp), g1 = g0;
        if (K16 > 16) g1 = *reinterpret_cast<const V4*>(gp + 16);
        const T* gt = G + lr * ldg + K16 + lk;
        T tv[3];
#pragma unroll
        for (int s = 0; s < 3; ++s) tv[s] = (K16 + 4 * s < K) ? gt[4 * s] : T(0);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (16 * c >= K16) break;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const T h = hp[(16 * c + s) * h_k];
                const T gv = c ? g1[s] : g0[s];
                acc = GA ? M::mma(gv, h, acc) : M::mma(h, gv, acc);
            }
        }
        const T* ht = H + lr * h_i + (K16 + lk) * h_k;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            if (K16 + 4 * s >= K) break;
            const T h = ht[4 * s * h_k];
            acc = GA ? M::mma(tv[s], h, acc) : M::mma(h, tv[s], acc);
        }
        return acc;
    }
    V4 g[2];
    g[0] = *reinterpret_cast<const V4*>(gp);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (16 * c >= K16) break;
        if (16 * (c + 1) < K16) g[(c + 1) & 1] = *reinterpret_cast<const V4*>(gp + 16 * (c + 1));
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const T h = hp[(16 * c + s) * h_k];
            const T gv = g[c & 1][s];
            acc = GA ? M::mma(gv, h, acc) : M::mma(h, gv, acc);
        }
    }
    const T* gt = G + lr * ldg + K16 + lk;
    const T* ht = H + lr * h_i + (K16 + lk) * h_k;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        if (K16 + 4 * s >= K) break;
        const T h = ht[4 * s * h_k];
        const T gv = gt[4 * s];
        acc = GA ? M::mma(gv, h, acc) : M::mma(h, gv, acc);
    }
    return acc;
}

// A 2x2 block of tile products: row tiles G0, G1 (G1 used when g1) and column
// tiles H0, H1 (when h1), each operand fragment loaded once for two MFMAs.
template <typename T, bool GA>
__device__ __forceinline__ void tile_gemm_2x2(const T* G0, const T* G1, int ldg, const T* H0,
                                              const T* H1, int h_k, int h_i, int K, int lr, int lk,
                                              bool g1, bool h1,
                                              typename Mfma<T>::V (&acc)[2][2]) {
    using M = Mfma<T>;
    using V4 = typename Vec4T<T>::V;
    const T* gp0 = G0 + lr * ldg + 4 * lk;
    const T* gp1 = G1 + lr * ldg + 4 * lk;
    const T* hp0 = H0 + lr * h_i + 4 * lk * h_k;
    const T* hp1 = H1 + lr * h_i + 4 * lk * h_k;
    V4 ga[2], gb[2];
    ga[0] = *reinterpret_cast<const V4*>(gp0);
    gb[0] = g1 ? *reinterpret_cast<const V4*>(gp1) : ga[0];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = typename M::V{0, 0, 0, 0};
    const int K16 = K & ~15;  // K: a multiple of 4, the tail as in tile_gemm
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (16 * c >= K16) break;
        if (16 * (c + 1) < K16) {
            ga[(c + 1) & 1] = *reinterpret_cast<const V4*>(gp0 + 16 * (c + 1));
            gb[(c + 1) & 1] = g1 ? *reinterpret_cast<const V4*>(gp1 + 16 * (c + 1)) : ga[(c + 1) & 1];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const T x0 = hp0[(16 * c + s) * h_k];
            const T x1 = h1 ? hp1[(16 * c + s) * h_k] : x0;
            const T a0 = ga[c & 1][s], a1 = gb[c & 1][s];
            acc[0][0] = GA ? M::mma(a0, x0, acc[0][0]) : M::mma(x0, a0, acc[0][0]);
            acc[0][1] = GA ? M::mma(a0, x1, acc[0][1]) : M::mma(x1, a0, acc[0][1]);
            acc[1][0] = GA ? M::mma(a1, x0, acc[1][0]) : M::mma(x0, a1, acc[1][0]);
            acc[1][1] = GA ? M::mma(a1, x1, acc[1][1]) : M::mma(x1, a1, acc[1][1]);
        }
    }
    const T* gt0 = G0 + lr * ldg + K16 + lk;
    const T* gt1 = G1 + lr * ldg + K16 + lk;
    const T* ht0 = H0 + lr * h_i + (K16 + lk) * h_k;
    const T* ht1 = H1 + lr * h_i + (K16 + lk) * h_k;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        if (K16 + 4 * s >= K) break;
        const T x0 = ht0[4 * s * h_k];
        const T x1 = h1 ? ht1[4 * s * h_k] : x0;
        const T a0 = gt0[4 * s];
        const T a1 = g1 ? gt1[4 * s] : a0;
        acc[0][0] = GA ? M::mma(a0, x0, acc[0][0]) : M::mma(x0, a0, acc[0][0]);
        acc[0][1] = GA ? M::mma(a0, x1, acc[0][1]) : M::mma(x1, a0, acc[0][1]);
        acc[1][0] = GA ? M::mma(a1, x0, acc[1][0]) : M::mma(x0, a1, acc[1][0]);
        acc[1][1] = GA ? M::mma(a1, x1, acc[1][1]) : M::mma(x1, a1, acc[1][1]);
    }
}

// Split-BF16 ("bf16x3") product for FP32 data: each operand is written as
// hi + lo with hi = bf16(x), lo = bf16(x - hi) (round to nearest even), and
// A B ~= A_hi B_hi + A_hi B_lo + A_lo B_hi, three 16x16x16 BF16 MFMAs per
// 16-wide k step accumulated in FP32.  hi + lo keeps 16 significant bits of
// each operand (relative error up to 2^-17), so a product is good to about
// 1e-5 relative, not to FP32 rounding; the dropped lo*lo term is of the
// same order.  A lane supplies the four values
// k = 16c + 4 lk + j, j < 4, of both operands (the instruction only needs
// the same k for both); result rows are 4 (l/16) + i as for FP32.  Operand
// roles and layouts as in tile_gemm.
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

template <bool GA>
__device__ __forceinline__ f4 tile_gemm_bf16x3(const float* G, int ldg, const float* H, int h_k,
                                               int h_i, int K, int lr, int lk) {
    const float* gp = G + lr * ldg + 4 * lk;
    const float* hp = H + lr * h_i + 4 * lk * h_k;
    f4 g[2];
    g[0] = *reinterpret_cast<const f4*>(gp);
    f4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (16 * c >= K) break;
        if (16 * (c + 1) < K) g[(c + 1) & 1] = *reinterpret_cast<const f4*>(gp + 16 * (c + 1));
        bf4 ghi, glo, hhi, hlo;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float gv = g[c & 1][j];
            const float hv = hp[(16 * c + j) * h_k];
            const __bf16 gh = (__bf16)gv, hh = (__bf16)hv;
            ghi[j] = gh;
            hhi[j] = hh;
            glo[j] = (__bf16)(gv - (float)gh);
            hlo[j] = (__bf16)(hv - (float)hh);
        }
        if (GA) {
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ghi, hhi, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ghi, hlo, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(glo, hhi, acc, 0, 0, 0);
        } else {
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(hhi, ghi, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(hhi, glo, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(hlo, ghi, acc, 0, 0, 0);
        }
    }
    return acc;
}

// dispatch of a 16x16 tile product: native MFMA of T, or split BF16 (T = float)
template <typename T, bool SPLIT, bool GA>
__device__ __forceinline__ typename Mfma<T>::V tile_mm(const T* G, int ldg, const T* H, int h_k,
                                                       int h_i, int n, int lr, int lk) {
    // n: the contraction's true length; the operands are zero from n to the
    // next multiple of 16
    if constexpr (SPLIT) {
        return tile_gemm_bf16x3<GA>(G, ldg, H, h_k, h_i, (n + 15) & ~15, lr, lk);
    } else {
        return tile_gemm<T, GA>(G, ldg, H, h_k, h_i, (n + 3) & ~3, lr, lk);
    }
}

// One i3-plane per workgroup, one buffer: the plane is transformed in place.
// Each wave computes its (at most XY_MT) output tiles into registers, the
// workgroup synchronises, and only then are the tiles written back, so the
// two steps need a single plane of LDS (which leaves room to stage the two
// dense 1D matrices, or lets FP64 planes up to 128 x 128 use 16 waves).
constexpr int XY_MT = 4;        // tiles per wave: 8 x 8 tiles over 16 waves

template <typename T, typename TI, typename TO, bool STAGE, bool SPLIT = false, bool BLK = false>
__global__ __launch_bounds__(FD_WIDE) void k_fd_xy_w(XYArgs a, FDTables<T> t) {
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
    const int ld = N1 + 1;  // column-major plane
    const int nb1 = N1 >> 4, nb2 = N2 >> 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = FD_WIDE / 64;
    const int lr = lane & 15, lk = lane >> 4;
    const long long kofs = (long long)k * n1 * n2;
    const TI* x = reinterpret_cast<const TI*>(a.in[f]) + (long long)r * a.sin[f] + kofs;
    xy_stage<T, TI, FD_WIDE>(a, f, x, r, kofs, S, ld, n1, n2, N1, N2);
    // L (rows contiguous) for step 1 and R^T (rows of R^T = columns of R) for step 2
    const T* L = xy_left(t, f, a.inverse);
    const T* Rt = xy_right_t(t, f, a.inverse);
    const int ldL = (f == 0) ? t.NNp : t.NMp;
    const int ldR = (f == 1) ? t.NNp : t.NMp;
    if (STAGE) {
        T* Ls = S + N2 * ld;
        T* Rs = Ls + N1 * N1;
        for (int idx = threadIdx.x; idx < N1 * N1; idx += FD_WIDE) Ls[idx] = L[idx];
        for (int idx = threadIdx.x; idx < N2 * N2; idx += FD_WIDE) Rs[idx] = Rt[idx];
        L = Ls;
        Rt = Rs;
    }
    __syncthreads();
    if constexpr (!SPLIT && BLK) {
        {
            // 2x2 blocks of tiles per wave: each operand fragment feeds two MFMAs
            const int nbb1 = (nb1 + 1) >> 1, nbb2 = (nb2 + 1) >> 1;
            const int nblk = nbb1 * nbb2;
            V bacc[2][2];
            const bool mine = wave < nblk;  // 16 waves cover up to 4 x 4 blocks
            const int RB = mine ? wave % nbb1 : 0, CB = mine ? wave / nbb1 : 0;
            const bool g1 = 2 * RB + 1 < nb1, h1 = 2 * CB + 1 < nb2;
            if (mine)
                tile_gemm_2x2<T, true>(L + 2 * RB * 16 * ldL, L + (2 * RB + 1) * 16 * ldL, ldL,
                                       S + 2 * CB * 16 * ld, S + (2 * CB + 1) * 16 * ld, 1, ld,
                                       (n1 + 3) & ~3, lr, lk, g1, h1, bacc);
            __syncthreads();
            if (mine)
#pragma unroll
                for (int ii = 0; ii < 2; ++ii)
#pragma unroll
                    for (int jj = 0; jj < 2; ++jj) {
                        if ((ii && !g1) || (jj && !h1)) continue;
                        const int rb = 2 * RB + ii, cb = 2 * CB + jj;
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            S[(cb * 16 + lr) * ld + rb * 16 + M::row(lk, i)] = bacc[ii][jj][i];
                    }
            __syncthreads();
            // step 2: Y = T R; block (RB2, CB2): G from R^T rows cb, H from T rows rb
            const int nbr = (nb1 + 1) >> 1, nbc = (nb2 + 1) >> 1;
            const bool mine2 = wave < nbr * nbc;
            const int RB2 = mine2 ? wave % nbr : 0, CB2 = mine2 ? wave / nbr : 0;
            const bool gc1 = 2 * CB2 + 1 < nb2, hr1 = 2 * RB2 + 1 < nb1;
            if (mine2)
                tile_gemm_2x2<T, false>(Rt + 2 * CB2 * 16 * ldR, Rt + (2 * CB2 + 1) * 16 * ldR, ldR,
                                        S + 2 * RB2 * 16, S + (2 * RB2 + 1) * 16, ld, 1,
                                        (n2 + 3) & ~3, lr, lk, gc1, hr1, bacc);
            __syncthreads();
            if (mine2)
#pragma unroll
                for (int ii = 0; ii < 2; ++ii)
#pragma unroll
                    for (int jj = 0; jj < 2; ++jj) {
                        if ((ii && !gc1) || (jj && !hr1)) continue;
                        const int cb = 2 * CB2 + ii, rb = 2 * RB2 + jj;
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            S[(cb * 16 + lr) * ld + rb * 16 + M::row(lk, i)] = bacc[ii][jj][i];
                    }
            __syncthreads();
            xy_store<T, TO, FD_WIDE>(a, S, ld, f, r, k, n1, n2);
            return;
        }
    }
    const int ntile = nb1 * nb2;
    V acc[XY_MT];
    // step 1: T = L X  (tile (rb, cb): rows of L, columns of X)
#pragma unroll
    for (int m = 0; m < XY_MT; ++m) {
        const int tt = wave + m * nw;
        if (tt < ntile) {
            const int rb = tt % nb1, cb = tt / nb1;
            acc[m] = tile_mm<T, SPLIT, true>(L + rb * 16 * ldL, ldL, S + cb * 16 * ld, 1, ld, n1,
                                             lr, lk);
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < XY_MT; ++m) {
        const int tt = wave + m * nw;
        if (tt < ntile) {
            const int rb = tt % nb1, cb = tt / nb1;
#pragma unroll
            for (int i = 0; i < 4; ++i) S[(cb * 16 + lr) * ld + rb * 16 + M::row(lk, i)] = acc[m][i];
        }
    }
    __syncthreads();
    // step 2: Y = T R
#pragma unroll
    for (int m = 0; m < XY_MT; ++m) {
        const int tt = wave + m * nw;
        if (tt < ntile) {
            const int rb = tt % nb1, cb = tt / nb1;
            acc[m] = tile_mm<T, SPLIT, false>(Rt + cb * 16 * ldR, ldR, S + rb * 16, ld, 1, n2, lr,
                                              lk);
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < XY_MT; ++m) {
        const int tt = wave + m * nw;
        if (tt < ntile) {
            const int rb = tt % nb1, cb = tt / nb1;
#pragma unroll
            for (int i = 0; i < 4; ++i) S[(cb * 16 + lr) * ld + rb * 16 + M::row(lk, i)] = acc[m][i];
        }
    }
    __syncthreads();
    xy_store<T, TO, FD_WIDE>(a, S, ld, f, r, k, n1, n2);
}

// One 16-row block of one i3-plane per 4-wave workgroup, for meshes whose
// planes alone leave most compute units idle: the nb1 row blocks of a plane
// run as nb1 workgroups.  Step 1's row block T_b = L_b X needs the whole
// plane X, which every workgroup of the plane stages; T_b stays in LDS
// (column-major, pitch 17) and Y_b = T_b R follows.  The dense 1D matrices
// are read from L2.  Per output tile the contraction is tile_mm's, with the
// operands of the wide kernel, so the result equals it bit for bit.
// Grid order: workgroup g runs on XCD g mod 8 (round-robin dispatch), and the
// row blocks of plane k take consecutive slots of XCD k mod 8, so that the
// workgroups staging one plane share that XCD's L2.
constexpr int FD_SPLIT = 256;   // 4 waves
constexpr int TBP = 17;         // pitch of the row block T_b in LDS

template <typename T, typename TI, typename TO, bool SPLIT = false>
__global__ __launch_bounds__(FD_SPLIT) void k_fd_xy_s(XYArgs a, FDTables<T> t) {
    using M = Mfma<T>;
    extern __shared__ unsigned char smem_raw[];
    T* S = reinterpret_cast<T*>(smem_raw);
    const int nf = a.fields_hi - a.fields_lo;
    const int f = a.fields_lo + (int)(blockIdx.y % nf);
    const int r = (int)(blockIdx.y / nf);
    const int xcd = (int)(blockIdx.x & 7), slot = (int)(blockIdx.x >> 3);
    const int k = (slot / a.nrb) * 8 + xcd, rb = slot % a.nrb;
    const int n1 = a.dims[f][0], n2 = a.dims[f][1], n3 = a.dims[f][2];
    const int N1 = (n1 + 15) & ~15, N2 = (n2 + 15) & ~15;
    if (k >= n3 || 16 * rb >= N1) return;
    const int ld = N1 + 1;  // column-major plane
    const int nb2 = N2 >> 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const long long kofs = (long long)k * n1 * n2;
    const TI* x = reinterpret_cast<const TI*>(a.in[f]) + (long long)r * a.sin[f] + kofs;
    xy_stage<T, TI, FD_SPLIT>(a, f, x, r, kofs, S, ld, n1, n2, N1, N2);
    T* Tb = S + N2 * ld;  // Tb[col * TBP + i]: row 16 rb + i of T (and later of Y)
    const T* L = xy_left(t, f, a.inverse);
    const T* Rt = xy_right_t(t, f, a.inverse);
    const int ldL = (f == 0) ? t.NNp : t.NMp;
    const int ldR = (f == 1) ? t.NNp : t.NMp;
    __syncthreads();
    typename M::V acc[2];
    // step 1: T_b = L_b X, tiles (rb, cb), cb = wave, wave + 4 (nb2 <= 8)
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int cb = wave + 4 * m;
        if (cb < nb2)
            acc[m] = tile_mm<T, SPLIT, true>(L + rb * 16 * ldL, ldL, S + cb * 16 * ld, 1, ld, n1,
                                             lr, lk);
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int cb = wave + 4 * m;
        if (cb < nb2)
#pragma unroll
            for (int i = 0; i < 4; ++i) Tb[(cb * 16 + lr) * TBP + M::row(lk, i)] = acc[m][i];
    }
    __syncthreads();
    // step 2: Y_b = T_b R, tiles (rb, cb)
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int cb = wave + 4 * m;
        if (cb < nb2)
            acc[m] = tile_mm<T, SPLIT, false>(Rt + cb * 16 * ldR, ldR, Tb, TBP, 1, n2, lr, lk);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int cb = wave + 4 * m;
        if (cb < nb2)
#pragma unroll
            for (int i = 0; i < 4; ++i) Tb[(cb * 16 + lr) * TBP + M::row(lk, i)] = acc[m][i];
    }
    __syncthreads();
    // write-out of rows [16 rb, min(n1, 16 rb + 16)), as xy_store for one row block
    const int rows = min(16, n1 - 16 * rb), n = 16 * n2;
    TO* y = reinterpret_cast<TO*>(a.out[f]) + (long long)r * a.sout[f] + kofs + 16 * rb;
    if constexpr (std::is_same<TO, double>::value) {
        if (a.dpart) {
            const double* w = a.dw[f] + (long long)r * a.sout[f] + kofs + 16 * rb;
            double s = 0.0;
            for (int base = 0; base < n; base += FD_BATCH * FD_SPLIT) {
                double yv[FD_BATCH], wv[FD_BATCH];
#pragma unroll
                for (int u = 0; u < FD_BATCH; ++u) {
                    const int idx = base + u * FD_SPLIT + (int)threadIdx.x;
                    const int col = idx >> 4, i = idx & 15;
                    const long long o = idx < n && i < rows ? i + (long long)col * n1 : 0;
                    yv[u] = a.accumulate ? y[o] : 0.0;
                    wv[u] = w[o];
                }
#pragma unroll
                for (int u = 0; u < FD_BATCH; ++u) {
                    const int idx = base + u * FD_SPLIT + (int)threadIdx.x;
                    const int col = idx >> 4, i = idx & 15;
                    if (idx < n && i < rows) {
                        double v = (double)Tb[col * TBP + i];
                        if (a.accumulate) v += yv[u];
                        y[i + (long long)col * n1] = v;
                        s += v * wv[u];
                    }
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
            __syncthreads();
            double* red = reinterpret_cast<double*>(S);
            if (lane == 0) red[wave] = s;
            __syncthreads();
            if (threadIdx.x == 0)
                a.dpart[(long long)r * a.dp_stride + (long long)f * a.dp_planes + k +
                        rb * a.dp_rb] = red[0] + red[1] + red[2] + red[3];
            return;
        }
    }
    if (a.accumulate) {
        for (int base = 0; base < n; base += FD_BATCH * FD_SPLIT) {
            TO yv[FD_BATCH];
#pragma unroll
            for (int u = 0; u < FD_BATCH; ++u) {
                const int idx = base + u * FD_SPLIT + (int)threadIdx.x;
                const int col = idx >> 4, i = idx & 15;
                yv[u] = y[idx < n && i < rows ? i + (long long)col * n1 : 0];
            }
#pragma unroll
            for (int u = 0; u < FD_BATCH; ++u) {
                const int idx = base + u * FD_SPLIT + (int)threadIdx.x;
                const int col = idx >> 4, i = idx & 15;
                if (idx < n && i < rows) y[i + (long long)col * n1] = yv[u] + (TO)Tb[col * TBP + i];
            }
        }
        return;
    }
    for (int idx = threadIdx.x; idx < n; idx += FD_SPLIT) {
        const int col = idx >> 4, i = idx & 15;
        if (i >= rows) continue;
        y[i + (long long)col * n1] = (TO)Tb[col * TBP + i];
    }
}

// z: ZR (i1,i2)-rows x n3 per workgroup of NTH threads (64 rows and 16
// waves, or 16 rows and 4 waves for small meshes), tiles of Y = X U3 and
// Z = Y U3^T dealt to the waves; the scaling by 1/(2 nu (l1 + l2 + l3)) is
// applied to Y.
template <typename T, typename TI, typename TO, bool STAGE, bool SPLIT = false, int ZR = ZROWS,
          int NTH = FD_WIDE>
__global__ __launch_bounds__(NTH) void k_fd_z_w(ZArgs a, FDTables<T> t) {
    using M = Mfma<T>;
    extern __shared__ unsigned char smem_raw[];
    T* S = reinterpret_cast<T*>(smem_raw);
    const int nf = a.fields_hi - a.fields_lo;
    const int f = a.fields_lo + (int)(blockIdx.y % nf);
    const int r = (int)(blockIdx.y / nf);
    const int n1 = a.dims[f][0], n2 = a.dims[f][1], n3 = a.dims[f][2];
    const long long plane = (long long)n1 * n2;
    const long long r0 = (long long)blockIdx.x * ZR;
    if (r0 >= plane) return;
    const int N3 = (n3 + 15) & ~15;
    const int ld = N3 + 1;  // row-major [row][k]
    const int nb3 = N3 >> 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = NTH / 64;
    const int lr = lane & 15, lk = lane >> 4;
    T* Y = S + ZR * ld;
    const TI* x = reinterpret_cast<const TI*>(a.in[f]) + (long long)r * a.sin[f];
    z_stage<T, TI, NTH, ZR>(x, r0, plane, n3, N3, S, ld);
    const bool pres = (f == 3);
    const T* U3 = pres ? t.Mi : (f == 2 ? t.UK : t.UT);
    const T* U3t = pres ? t.Mi : (f == 2 ? t.UKt : t.UTt);
    const int ldU = (f == 2) ? t.NNp : t.NMp;
    if (STAGE) {
        T* Us = Y + ZR * ld;
        T* Uts = Us + N3 * N3;
        for (int idx = threadIdx.x; idx < N3 * N3; idx += NTH) {
            Us[idx] = U3[idx];
            if (!pres) Uts[idx] = U3t[idx];
        }
        U3 = Us;
        U3t = pres ? Us : Uts;  // M^^{-1} is symmetric: one staged copy serves both
    }
    __syncthreads();
    const int ntile = (ZR / 16) * nb3;
    const double* l1 = (f == 0) ? t.lamK : t.lamT;
    const double* l2 = (f == 1) ? t.lamK : t.lamT;
    const double* l3 = (f == 2) ? t.lamK : t.lamT;
    for (int tt = wave; tt < ntile; tt += nw) {
        const int rb = tt % (ZR / 16), cb = tt / (ZR / 16);
        auto acc = tile_mm<T, SPLIT, false>(U3t + cb * 16 * ldU, ldU, S + rb * 16 * ld, 1, ld, n3, lr, lk);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = rb * 16 + M::row(lk, i);
            const int col = cb * 16 + lr;
            double sc;
            if (pres) {
                sc = a.omega * a.two_nu;
            } else {
                sc = 0.0;
                const long long rr = r0 + row;
                if (rr < plane && col < n3) {
                    const int i1 = (int)(rr % n1), i2 = (int)(rr / n1);
                    sc = a.omega / (a.two_nu * (l1[i1] + l2[i2] + l3[col]));
                }
            }
            Y[row * ld + col] = (T)(sc * (double)acc[i]);
        }
    }
    __syncthreads();
    T* Out = Y;
    if (!pres) {
        for (int tt = wave; tt < ntile; tt += nw) {
            const int rb = tt % (ZR / 16), cb = tt / (ZR / 16);
            auto acc = tile_mm<T, SPLIT, false>(U3 + cb * 16 * ldU, ldU, Y + rb * 16 * ld, 1, ld, n3, lr, lk);
#pragma unroll
            for (int i = 0; i < 4; ++i) S[(rb * 16 + M::row(lk, i)) * ld + cb * 16 + lr] = acc[i];
        }
        __syncthreads();
        Out = S;
    }
    z_store<T, TO, NTH, ZR>(a, Out, S, ld, f, r, r0, plane, n3);
}

// LDS plan for a direction of padded size np: wide (two buffers) or in place,
// and whether the dense 1D matrices are staged in LDS as well.
struct FDPlan {
    bool wide, stage_xy, stage_z, block;
    bool split;  // row-block xy kernel and 16-row z kernel (FD_PLAN_SPLIT)
    size_t shm_xy, shm_z;
};

// The plan of plan code `code` (bit 0: wide kernels, bit 1: stage the 1D
// matrices in LDS when they fit, bit 2: 2x2 blocks of MFMA tiles per wave in
// the wide xy kernel); code < 0 gives the default plan: wide when two planes
// fit in LDS, staging when it leaves room for a second workgroup.
template <typename T>
FDPlan fd_plan(int np, int code) {
    // wide kernels: the xy kernel transforms one plane in place (one plane of
    // LDS), the z kernel keeps its input and intermediate rows (two buffers)
    const size_t lim = 160 * 1024, e = sizeof(T);
    FDPlan pl{};
    if (code == FD_PLAN_SPLIT) {
        pl.wide = true;
        pl.split = true;
        pl.shm_xy = (size_t)np * (np + 1 + TBP) * e;
        pl.shm_z = (size_t)2 * 16 * (np + 1) * e;
        return pl;
    }
    const size_t plane = (size_t)np * (np + 1) * e, mats = (size_t)2 * np * np * e;
    const size_t zbuf = (size_t)ZROWS * (np + 1) * e;
    const bool wide_fits = plane <= lim && 2 * zbuf <= lim;
    if (code < 0) {
        pl.wide = wide_fits;
        if (pl.wide) {
            pl.stage_xy = plane + mats <= 140 * 1024;
            pl.stage_z = 2 * zbuf + mats <= 140 * 1024;
        } else {
            pl.stage_xy = plane + mats <= 96 * 1024;
            pl.stage_z = zbuf + mats <= 96 * 1024;
        }
    } else {
        pl.wide = (code & 1) != 0;
        pl.stage_xy = (code & 2) && plane + mats <= lim;
        pl.stage_z = (code & 2) && (pl.wide ? 2 : 1) * zbuf + mats <= lim;
        pl.block = (code & 4) && pl.wide;
    }
    pl.shm_xy = plane + (pl.stage_xy ? mats : 0);
    pl.shm_z = (pl.wide ? 2 : 1) * zbuf + (pl.stage_z ? mats : 0);
    return pl;
}

template <typename T>
bool fd_plan_fits(int np, int code) {
    if (code < 0) return true;
    if (code == FD_PLAN_SPLIT) return fd_plan<T>(np, code).shm_xy <= 160 * 1024;
    if (code > 7) return false;
    if ((code & 4) && !(code & 1)) return false;  // blocking exists in the wide kernel only
    const size_t lim = 160 * 1024, e = sizeof(T);
    const size_t plane = (size_t)np * (np + 1) * e, zbuf = (size_t)ZROWS * (np + 1) * e;
    // a staging plan must actually stage something to differ from its pair
    const FDPlan pl = fd_plan<T>(np, code);
    const bool fits = (code & 1) ? plane <= lim && 2 * zbuf <= lim : plane <= lim && zbuf <= lim;
    return fits && (!(code & 2) || pl.stage_xy || pl.stage_z);
}

template <typename T, bool SPLIT = false>
hipError_t run_P0(hp_ctx* c, const FDTables<T>& t, const Fields& in, const Fields& out, bool vel,
                  bool pres, bool accumulate, int nrhs, const FdDot* dot, const FdComb* comb) {
    // scratch for the two intermediate tensors (precision T), per rhs N values each
    const long long N = c->N;
    T* tmp1 = reinterpret_cast<T*>(c->ws + ops_ws_stride(c) * (long long)c->opts.max_rhs);
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
    if (comb) {
        for (int f = lo; f < hi; ++f) {
            xa.inb[f] = comb->b.f[f];
            xa.inc[f] = comb->c.f[f];
            xa.sinb[f] = comb->b.stride[f];
            xa.sinc[f] = comb->c.stride[f];
        }
        xa.ca = comb->ca;
        xa.cb = comb->cb;
        xa.cc = comb->cc;
    }
    const FDPlan pl = fd_plan<T>(NMp, fd_plan_in_use(c, std::is_same<T, double>::value ? 0 : (SPLIT ? 2 : 1)));
    const dim3 bxy(pl.wide ? FD_WIDE : FD_THREADS);
    auto launch_xy = [&](const XYArgs& xa_, bool to_double, int nfields) {
        dim3 g(nM, nfields * nrhs);
        if (pl.split) {
            XYArgs xs = xa_;
            xs.nrb = NMp / 16;
            const dim3 gs((unsigned)(8 * xs.nrb * ((nM + 7) / 8)), nfields * nrhs);
            if (to_double) hipLaunchKernelGGL((k_fd_xy_s<T, T, double, SPLIT>), gs, dim3(FD_SPLIT), pl.shm_xy, c->stream, xs, t);
            else hipLaunchKernelGGL((k_fd_xy_s<T, double, T, SPLIT>), gs, dim3(FD_SPLIT), pl.shm_xy, c->stream, xs, t);
        } else if (pl.wide && pl.block && !SPLIT) {
            if (to_double) {
                if (pl.stage_xy) hipLaunchKernelGGL((k_fd_xy_w<T, T, double, true, SPLIT, true>), g, bxy, pl.shm_xy, c->stream, xa_, t);
                else hipLaunchKernelGGL((k_fd_xy_w<T, T, double, false, SPLIT, true>), g, bxy, pl.shm_xy, c->stream, xa_, t);
            } else {
                if (pl.stage_xy) hipLaunchKernelGGL((k_fd_xy_w<T, double, T, true, SPLIT, true>), g, bxy, pl.shm_xy, c->stream, xa_, t);
                else hipLaunchKernelGGL((k_fd_xy_w<T, double, T, false, SPLIT, true>), g, bxy, pl.shm_xy, c->stream, xa_, t);
            }
        } else if (pl.wide) {
            if (to_double) {
                if (pl.stage_xy) hipLaunchKernelGGL((k_fd_xy_w<T, T, double, true, SPLIT>), g, bxy, pl.shm_xy, c->stream, xa_, t);
                else hipLaunchKernelGGL((k_fd_xy_w<T, T, double, false, SPLIT>), g, bxy, pl.shm_xy, c->stream, xa_, t);
            } else {
                if (pl.stage_xy) hipLaunchKernelGGL((k_fd_xy_w<T, double, T, true, SPLIT>), g, bxy, pl.shm_xy, c->stream, xa_, t);
                else hipLaunchKernelGGL((k_fd_xy_w<T, double, T, false, SPLIT>), g, bxy, pl.shm_xy, c->stream, xa_, t);
            }
        } else {
            if (to_double) {
                if (pl.stage_xy) hipLaunchKernelGGL((k_fd_xy<T, T, double, true>), g, bxy, pl.shm_xy, c->stream, xa_, t);
                else hipLaunchKernelGGL((k_fd_xy<T, T, double, false>), g, bxy, pl.shm_xy, c->stream, xa_, t);
            } else {
                if (pl.stage_xy) hipLaunchKernelGGL((k_fd_xy<T, double, T, true>), g, bxy, pl.shm_xy, c->stream, xa_, t);
                else hipLaunchKernelGGL((k_fd_xy<T, double, T, false>), g, bxy, pl.shm_xy, c->stream, xa_, t);
            }
        }
    };
    auto launch_z = [&](const ZArgs& za_, bool to_double, int nfields) {
        const long long maxplane = (long long)nM * nM;
        dim3 g((unsigned)((maxplane + ZROWS - 1) / ZROWS), nfields * nrhs);
        if (pl.split) {
            const dim3 gs((unsigned)((maxplane + 15) / 16), nfields * nrhs);
            if (to_double) hipLaunchKernelGGL((k_fd_z_w<T, T, double, false, SPLIT, 16, FD_SPLIT>), gs, dim3(FD_SPLIT), pl.shm_z, c->stream, za_, t);
            else hipLaunchKernelGGL((k_fd_z_w<T, T, T, false, SPLIT, 16, FD_SPLIT>), gs, dim3(FD_SPLIT), pl.shm_z, c->stream, za_, t);
        } else if (pl.wide) {
            dim3 b(FD_WIDE);
            if (to_double) {
                if (pl.stage_z) hipLaunchKernelGGL((k_fd_z_w<T, T, double, true, SPLIT>), g, b, pl.shm_z, c->stream, za_, t);
                else hipLaunchKernelGGL((k_fd_z_w<T, T, double, false, SPLIT>), g, b, pl.shm_z, c->stream, za_, t);
            } else {
                if (pl.stage_z) hipLaunchKernelGGL((k_fd_z_w<T, T, T, true, SPLIT>), g, b, pl.shm_z, c->stream, za_, t);
                else hipLaunchKernelGGL((k_fd_z_w<T, T, T, false, SPLIT>), g, b, pl.shm_z, c->stream, za_, t);
            }
        } else {
            dim3 b(FD_THREADS);
            if (to_double) {
                if (pl.stage_z) hipLaunchKernelGGL((k_fd_z<T, T, double, true>), g, b, pl.shm_z, c->stream, za_, t);
                else hipLaunchKernelGGL((k_fd_z<T, T, double, false>), g, b, pl.shm_z, c->stream, za_, t);
            } else {
                if (pl.stage_z) hipLaunchKernelGGL((k_fd_z<T, T, T, true>), g, b, pl.shm_z, c->stream, za_, t);
                else hipLaunchKernelGGL((k_fd_z<T, T, T, false>), g, b, pl.shm_z, c->stream, za_, t);
            }
        }
    };
    launch_xy(xa, false, nf);
    ZArgs za{};
    for (int f = 0; f < 4; ++f) {
        for (int d = 0; d < 3; ++d) za.dims[f][d] = (int)c->dims[f][d];
        za.in[f] = tmp1 + c->off[f];
        za.sin[f] = N;
        za.out[f] = tmp2 + c->off[f];
        za.sout[f] = N;
    }
    za.two_nu = 2.0 * c->nu;
    za.omega = c->opts.p0_scale;
    // the pressure's mode-3 step writes the final output; the velocity's
    // feeds the inverse xy step.  In FP64 both output types agree, so the
    // four fields share one launch.
    za.out[3] = out.f[3];
    za.sout[3] = out.stride[3];
    za.accumulate = accumulate ? (1 << 3) : 0;
    if (vel && pres && std::is_same<T, double>::value) {
        ZArgs zb = za;
        zb.fields_lo = 0;
        zb.fields_hi = 4;
        launch_z(zb, true, 4);
    } else {
        if (vel) {
            ZArgs zv = za;
            zv.fields_lo = 0;
            zv.fields_hi = 3;
            launch_z(zv, false, 3);
        }
        if (pres) {
            ZArgs zp = za;
            zp.fields_lo = 3;
            zp.fields_hi = 4;
            if (dot && !vel) {
                zp.dw = dot->with + c->off[3];
                zp.dpart = dot->part;
                zp.dp_stride = fd_dot_count(c, false);
            }
            launch_z(zp, true, 1);
        }
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
        if (dot) {
            // xy partials: per rhs 3 nM, times the row blocks of the split plan
            // (see fd_dot_count)
            for (int f = 0; f < 3; ++f) xi.dw[f] = dot->with + c->off[f];
            xi.dpart = dot->part;
            xi.dp_stride = fd_dot_count(c, true);
            xi.dp_planes = nM;
            xi.dp_rb = 3LL * nM;
        }
        launch_xy(xi, true, 3);
    }
    return hipGetLastError();
}

// ---- mode products as batched GEMMs (directions of any length) ----------------------
// The in-LDS kernels above hold a whole direction (<= 128) in MFMA tiles.  For
// longer directions -- and as the selectable plan FD_GEMM at any size -- each
// mode product of fast diagonalisation runs as a (batched) GEMM over HBM:
//     C(i, j) = sum_k A(i, k) B(k, j),  B(k, j) = B[k ldb + j] (a dense 1D table)
// with strided A and C; batch b adds (b % nb1) s1 + (b / nb1) s2 to A and C.
// Mode 1 is taken transposed (i over the (i2, i3) lines, j over i1') so that
// B is always a row-major 1D table and the tensor is the A operand:
//   mode 1: A(i, k) = X[k + i n1]            (k contiguous), C(i, j) = Y[j + i n1]
//   mode 2: A(i, k) = X[i + k n1], per i3    (i contiguous), C(i, j) = Y[i + j n1]
//   mode 3: A(i, k) = X[i + k n1 n2]         (i contiguous), C(i, j) = Y[i + j n1 n2]
// with B = U (forward) or U^T (inverse), M^^{-1} for the pressure.  The
// eigenvalue scaling (epilogue 2) is fused into the forward mode-3 product.
// Tile: 64 x 64 outputs per 256-thread workgroup, each wave 2 x 2 MFMA tiles
// of 16 x 16 (sub-tiles entirely outside the output are skipped, so a ragged
// direction costs at most 15 padded rows); the contraction runs in chunks of
// 16 staged k-major in LDS (pitch 80: the 16 lanes of one k row and the next
// k row fall in disjoint banks), double buffered, the next chunk loaded into
// registers while the current one is multiplied.  The output tile goes
// through LDS so that it is stored along C's contiguous direction.
constexpr int GT = 64;
constexpr int GK = 16;
constexpr int GP = 80;
constexpr int GTHREADS = 256;

struct GemmArgs {
    const void* A;
    long long a_i, a_k, a_s1, a_s2;
    const void* B;
    int ldb;
    void* C;
    long long c_i, c_j, c_s1, c_s2;
    int M, N, K, nb1, tiles_m;
    int epi;          // 0: C = acc, 1: C = alpha acc, 2: C = alpha acc / (l1[i1] + l2[i2] + l3[j])
    int accumulate;   // C += (epilogue value)
    double alpha;
    const double* l1;
    const double* l2;
    const double* l3;
    int n1;           // epilogue 2: i = i1 + n1 i2
};

template <typename T, typename TI, typename TO, bool A_KC, bool C_IC>
__global__ __launch_bounds__(GTHREADS) void k_mode_gemm(GemmArgs g) {
    using M = Mfma<T>;
    using V = typename M::V;
    constexpr int TILE_T = 2 * 2 * GK * GP;       // As, Bs, double buffered
    constexpr int CT_T = GT * (GT + 1);           // the output tile [i][j]
    __shared__ T sm[TILE_T > CT_T ? TILE_T : CT_T];
    T* As = sm;                                   // [buf][k][i]
    T* Bs = sm + 2 * GK * GP;                     // [buf][k][j]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int tm = blockIdx.x % g.tiles_m, tn = blockIdx.x / g.tiles_m;
    const int i0 = tm * GT, j0 = tn * GT;
    const long long bb = blockIdx.y;
    const long long boffA = (bb % g.nb1) * g.a_s1 + (bb / g.nb1) * g.a_s2;
    const long long boffC = (bb % g.nb1) * g.c_s1 + (bb / g.nb1) * g.c_s2;
    const TI* A = reinterpret_cast<const TI*>(g.A) + boffA;
    const T* B = reinterpret_cast<const T*>(g.B);
    // staging: four A and four B values per thread per chunk
    T ra[4], rb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int e = tid + GTHREADS * s;
            int i, k;
            if (A_KC) { k = e % GK; i = e / GK; }
            else { i = e % GT; k = e / GT; }
            const int gi = i0 + i, gk = k0 + k;
            ra[s] = (gi < g.M && gk < g.K) ? (T)A[gi * g.a_i + gk * g.a_k] : (T)0;
            const int j = e % GT, kb = e / GT;
            const int gj = j0 + j, gkb = k0 + kb;
            rb[s] = (gj < g.N && gkb < g.K) ? B[(long long)gkb * g.ldb + gj] : (T)0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int e = tid + GTHREADS * s;
            int i, k;
            if (A_KC) { k = e % GK; i = e / GK; }
            else { i = e % GT; k = e / GT; }
            As[buf * GK * GP + k * GP + i] = ra[s];
            Bs[buf * GK * GP + (e / GT) * GP + (e % GT)] = rb[s];
        }
    };
    const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
    bool on[2][2];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
            on[ii][jj] = (i0 + wr + 16 * ii < g.M) && (j0 + wc + 16 * jj < g.N);
    V acc[2][2];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) acc[ii][jj] = V{0, 0, 0, 0};
    load(0);
    for (int k0 = 0, it = 0; k0 < g.K; k0 += GK, ++it) {
        const int buf = it & 1;
        store(buf);
        __syncthreads();
        if (k0 + GK < g.K) load(k0 + GK);
        const T* as = As + buf * GK * GP;
        const T* bs = Bs + buf * GK * GP;
#pragma unroll
        for (int st = 0; st < GK / 4; ++st) {
            const int kk = 4 * st + lk;
            T av[2], bv[2];
#pragma unroll
            for (int ii = 0; ii < 2; ++ii) av[ii] = as[kk * GP + wr + 16 * ii + lr];
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) bv[jj] = bs[kk * GP + wc + 16 * jj + lr];
#pragma unroll
            for (int ii = 0; ii < 2; ++ii)
#pragma unroll
                for (int jj = 0; jj < 2; ++jj)
                    if (on[ii][jj]) acc[ii][jj] = M::mma(av[ii], bv[jj], acc[ii][jj]);
        }
    }
    __syncthreads();  // every wave is done with As/Bs: the output tile reuses them
    T* Ct = sm;
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
            if (on[ii][jj])
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    Ct[(wr + 16 * ii + M::row(lk, e)) * (GT + 1) + wc + 16 * jj + lr] = acc[ii][jj][e];
    __syncthreads();
    TO* C = reinterpret_cast<TO*>(g.C) + boffC;
    for (int s = 0; s < GT * GT / GTHREADS; ++s) {
        const int e = tid + GTHREADS * s;
        int i, j;
        if (C_IC) { i = e % GT; j = e / GT; }
        else { j = e % GT; i = e / GT; }
        const int gi = i0 + i, gj = j0 + j;
        if (gi >= g.M || gj >= g.N) continue;
        double v = (double)Ct[i * (GT + 1) + j];
        if (g.epi == 1) {
            v *= g.alpha;
        } else if (g.epi == 2) {
            const int i1 = gi % g.n1, i2 = gi / g.n1;
            v *= g.alpha / (g.l1[i1] + g.l2[i2] + g.l3[gj]);
        }
        TO* dst = C + (long long)gi * g.c_i + (long long)gj * g.c_j;
        if (g.accumulate) *dst += (TO)v;
        else *dst = (TO)v;
    }
}

// Partial sums of y . w for the Krylov dot of launch_P0, in the layout of the
// in-LDS kernels: velocity, one per (field, i3-plane) at f nM + k; pressure,
// one per ZROWS-row block of the (i1, i2) plane.  Fixed-order block sums.
__global__ __launch_bounds__(256) void k_fd_dot_vel(const double* y, const double* w,
                                                    long long stride, long long plane,
                                                    double* part, long long dp_stride,
                                                    int slot0) {
    __shared__ double red[4];
    const int k = blockIdx.x, r = blockIdx.y;
    const double* yr = y + (long long)r * stride + (long long)k * plane;
    const double* wr = w + (long long)r * stride + (long long)k * plane;
    double s = 0.0;
    for (long long i = threadIdx.x; i < plane; i += 256) s += yr[i] * wr[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        part[(long long)r * dp_stride + slot0 + k] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_fd_dot_pres(const double* y, const double* w,
                                                     long long stride, long long plane, int n3,
                                                     double* part, long long dp_stride) {
    __shared__ double red[4];
    const int r = blockIdx.y;
    const long long r0 = (long long)blockIdx.x * ZROWS;
    const double* yr = y + (long long)r * stride;
    const double* wr = w + (long long)r * stride;
    double s = 0.0;
    for (long long idx = threadIdx.x; idx < (long long)ZROWS * n3; idx += 256) {
        const long long kk = idx / ZROWS, row = idx - kk * ZROWS;
        if (r0 + row >= plane) continue;
        const long long o = r0 + row + kk * plane;
        s += yr[o] * wr[o];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        part[(long long)r * dp_stride + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

template <typename T, typename TI, typename TO, bool A_KC, bool C_IC>
hipError_t gemm_launch(hipStream_t st, GemmArgs g, int nbatch) {
    g.tiles_m = (g.M + GT - 1) / GT;
    const int tiles_n = (g.N + GT - 1) / GT;
    if (g.M <= 0 || g.N <= 0 || nbatch <= 0) return hipSuccess;
    if (nbatch > 65535) return hipErrorInvalidConfiguration;  // grid y limit
    hipLaunchKernelGGL((k_mode_gemm<T, TI, TO, A_KC, C_IC>), dim3(g.tiles_m * tiles_n, nbatch),
                       dim3(GTHREADS), 0, st, g);
    return hipGetLastError();
}

// P_0^{-1} by mode-product GEMMs (velocity: six products per component, the
// eigenvalue scaling fused into the forward mode-3 product; pressure: three
// products with M^^{-1}, the factor 2 nu w in the last).  Intermediates of
// precision T ping-pong between the two fast-diagonalisation scratch
// buffers; the combination input (comb) is formed first in the operator
// workspace, the dot partials are summed from the final output.
template <typename T>
hipError_t run_P0_gemm(hp_ctx* c, const FDTables<T>& t, const Fields& in, const Fields& out,
                       bool vel, bool pres, bool accumulate, int nrhs, const FdDot* dot,
                       const FdComb* comb) {
    const long long N = c->N, R = c->opts.max_rhs;
    T* tmp1 = reinterpret_cast<T*>(c->ws + ops_ws_stride(c) * R);
    T* tmp2 = tmp1 + N * R;
    const double omega = c->opts.p0_scale, two_nu = 2.0 * c->nu;
    hipError_t e = hipSuccess;
    for (int f = vel ? 0 : 3; f < (pres ? 4 : 3) && e == hipSuccess; ++f) {
        const int n1 = (int)c->dims[f][0], n2 = (int)c->dims[f][1], n3 = (int)c->dims[f][2];
        const long long n12 = (long long)n1 * n2;
        const double* x = in.f[f];
        long long sx = in.stride[f];
        if (comb && comb->b.f[f]) {
            // x = ca in + cb b + cc c into the operator workspace (n_Q per rhs >= any field)
            double* xc = c->ws;
            e = vec_axpbypcz(c->stream, n12 * n3, nrhs, comb->ca, x, sx, comb->cb, comb->b.f[f],
                             comb->b.stride[f], comb->cc, comb->c.f[f], comb->c.stride[f], xc,
                             ops_ws_stride(c));
            if (e != hipSuccess) break;
            x = xc;
            sx = ops_ws_stride(c);
        }
        T* Y1 = tmp1 + c->off[f];
        T* Y2 = tmp2 + c->off[f];
        const bool isp = (f == 3);
        // 1D tables per direction: forward B = U, inverse B = U^T (M^^{-1} for p)
        const T* Uf[3];
        const T* Ui[3];
        int ld[3];
        for (int d = 0; d < 3; ++d) {
            const bool kdir = (d == f);
            Uf[d] = isp ? t.Mi : (kdir ? t.UK : t.UT);
            Ui[d] = isp ? t.Mi : (kdir ? t.UKt : t.UTt);
            ld[d] = (!isp && kdir) ? t.NNp : t.NMp;
        }
        auto mode1 = [&](const void* src, long long ss, const T* U, int ldu, void* dst,
                         long long sd, bool to_out, int epi, double alpha, bool acc) {
            GemmArgs g{};
            g.A = src; g.a_i = n1; g.a_k = 1; g.a_s1 = ss; g.a_s2 = 0;
            g.B = U; g.ldb = ldu;
            g.C = dst; g.c_i = n1; g.c_j = 1; g.c_s1 = sd; g.c_s2 = 0;
            g.M = (int)(n2 * (long long)n3); g.N = n1; g.K = n1; g.nb1 = nrhs;
            g.epi = epi; g.alpha = alpha; g.accumulate = acc;
            if (to_out) return gemm_launch<T, T, double, true, false>(c->stream, g, nrhs);
            return gemm_launch<T, double, T, true, false>(c->stream, g, nrhs);
        };
        auto mode2 = [&](const T* src, const T* U, int ldu, T* dst) {
            GemmArgs g{};
            g.A = src; g.a_i = 1; g.a_k = n1; g.a_s1 = n12; g.a_s2 = N;
            g.B = U; g.ldb = ldu;
            g.C = dst; g.c_i = 1; g.c_j = n1; g.c_s1 = n12; g.c_s2 = N;
            g.M = n1; g.N = n2; g.K = n2; g.nb1 = n3;
            return gemm_launch<T, T, T, false, true>(c->stream, g, n3 * nrhs);
        };
        auto mode3 = [&](const T* src, const T* U, int ldu, void* dst, long long sd, bool to_out,
                         int epi, double alpha, bool acc) {
            GemmArgs g{};
            g.A = src; g.a_i = 1; g.a_k = n12; g.a_s1 = N; g.a_s2 = 0;
            g.B = U; g.ldb = ldu;
            g.C = dst; g.c_i = 1; g.c_j = n12; g.c_s1 = sd; g.c_s2 = 0;
            g.M = (int)n12; g.N = n3; g.K = n3; g.nb1 = nrhs;
            g.epi = epi; g.alpha = alpha; g.accumulate = acc;
            g.n1 = n1;
            g.l1 = (f == 0) ? t.lamK : t.lamT;
            g.l2 = (f == 1) ? t.lamK : t.lamT;
            g.l3 = (f == 2) ? t.lamK : t.lamT;
            if (to_out) return gemm_launch<T, T, double, false, true>(c->stream, g, nrhs);
            return gemm_launch<T, T, T, false, true>(c->stream, g, nrhs);
        };
        if (isp) {
            if ((e = mode1(x, sx, Uf[0], ld[0], Y1, N, false, 0, 1.0, false)) != hipSuccess) break;
            if ((e = mode2(Y1, Uf[1], ld[1], Y2)) != hipSuccess) break;
            e = mode3(Y2, Uf[2], ld[2], out.f[3], out.stride[3], true, 1, omega * two_nu,
                      accumulate);
        } else {
            if ((e = mode1(x, sx, Uf[0], ld[0], Y1, N, false, 0, 1.0, false)) != hipSuccess) break;
            if ((e = mode2(Y1, Uf[1], ld[1], Y2)) != hipSuccess) break;
            if ((e = mode3(Y2, Uf[2], ld[2], Y1, N, false, 2, omega / two_nu, false)) != hipSuccess)
                break;
            if ((e = mode3(Y1, Ui[2], ld[2], Y2, N, false, 0, 1.0, false)) != hipSuccess) break;
            if ((e = mode2(Y2, Ui[1], ld[1], Y1)) != hipSuccess) break;
            e = mode1(Y1, N, Ui[0], ld[0], out.f[f], out.stride[f], true, 0, 1.0, accumulate);
        }
    }
    if (e != hipSuccess || !dot) return e;
    const int nM = c->nM;
    if (vel && !pres) {
        for (int f = 0; f < 3; ++f) {
            const long long plane = c->dims[f][0] * c->dims[f][1];
            hipLaunchKernelGGL(k_fd_dot_vel, dim3((unsigned)c->dims[f][2], nrhs), dim3(256), 0,
                               c->stream, out.f[f], dot->with + c->off[f], out.stride[f], plane,
                               dot->part, 3LL * nM, f * nM);
        }
    } else if (pres && !vel) {
        const long long plane = (long long)nM * nM;
        hipLaunchKernelGGL(k_fd_dot_pres, dim3((unsigned)((plane + ZROWS - 1) / ZROWS), nrhs),
                           dim3(256), 0, c->stream, out.f[3], dot->with + c->off[3], out.stride[3],
                           plane, nM, dot->part, fd_dot_count(c, false));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t set_fd_attrs() {
    const int bytes = 160 * 1024;
    const void* ks[] = {
        reinterpret_cast<const void*>(&k_fd_xy<T, double, T, true>),
        reinterpret_cast<const void*>(&k_fd_xy<T, double, T, false>),
        reinterpret_cast<const void*>(&k_fd_xy<T, T, double, true>),
        reinterpret_cast<const void*>(&k_fd_xy<T, T, double, false>),
        reinterpret_cast<const void*>(&k_fd_z<T, T, T, true>),
        reinterpret_cast<const void*>(&k_fd_z<T, T, T, false>),
        reinterpret_cast<const void*>(&k_fd_z<T, T, double, true>),
        reinterpret_cast<const void*>(&k_fd_z<T, T, double, false>),
        reinterpret_cast<const void*>(&k_fd_xy_w<T, double, T, true>),
        reinterpret_cast<const void*>(&k_fd_xy_w<T, double, T, false>),
        reinterpret_cast<const void*>(&k_fd_xy_w<T, T, double, true>),
        reinterpret_cast<const void*>(&k_fd_xy_w<T, T, double, false>),
        reinterpret_cast<const void*>(&k_fd_xy_w<T, double, T, true, false, true>),
        reinterpret_cast<const void*>(&k_fd_xy_w<T, double, T, false, false, true>),
        reinterpret_cast<const void*>(&k_fd_xy_w<T, T, double, true, false, true>),
        reinterpret_cast<const void*>(&k_fd_xy_w<T, T, double, false, false, true>),
        reinterpret_cast<const void*>(&k_fd_z_w<T, T, T, true>),
        reinterpret_cast<const void*>(&k_fd_z_w<T, T, T, false>),
        reinterpret_cast<const void*>(&k_fd_z_w<T, T, double, true>),
        reinterpret_cast<const void*>(&k_fd_z_w<T, T, double, false>),
        reinterpret_cast<const void*>(&k_fd_xy_s<T, double, T>),
        reinterpret_cast<const void*>(&k_fd_xy_s<T, T, double>),
        reinterpret_cast<const void*>(&k_fd_z_w<T, T, T, false, false, 16, FD_SPLIT>),
        reinterpret_cast<const void*>(&k_fd_z_w<T, T, double, false, false, 16, FD_SPLIT>)};
    for (const void* k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t fd_init_attributes() {
    hipError_t e = set_fd_attrs<double>();
    if (e != hipSuccess) return e;
    e = set_fd_attrs<float>();
    if (e != hipSuccess) return e;
    const void* ks[] = {
        reinterpret_cast<const void*>(&k_fd_xy_w<float, double, float, true, true>),
        reinterpret_cast<const void*>(&k_fd_xy_w<float, double, float, false, true>),
        reinterpret_cast<const void*>(&k_fd_xy_w<float, float, double, true, true>),
        reinterpret_cast<const void*>(&k_fd_xy_w<float, float, double, false, true>),
        reinterpret_cast<const void*>(&k_fd_z_w<float, float, float, true, true>),
        reinterpret_cast<const void*>(&k_fd_z_w<float, float, float, false, true>),
        reinterpret_cast<const void*>(&k_fd_z_w<float, float, double, true, true>),
        reinterpret_cast<const void*>(&k_fd_z_w<float, float, double, false, true>),
        reinterpret_cast<const void*>(&k_fd_xy_s<float, double, float, true>),
        reinterpret_cast<const void*>(&k_fd_xy_s<float, float, double, true>),
        reinterpret_cast<const void*>(&k_fd_z_w<float, float, float, false, true, 16, FD_SPLIT>),
        reinterpret_cast<const void*>(&k_fd_z_w<float, float, double, false, true, 16, FD_SPLIT>)};
    for (const void* k : ks) {
        e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// directions longer than the in-LDS kernels hold (8 MFMA tiles of 16)
static bool fd_needs_gemm(const hp_ctx* c) { return ((c->nM + 15) & ~15) > 128; }

bool fd_plan_valid(const hp_ctx* c, int precision, int plan) {
    const int NMp = (c->nM + 15) & ~15;
    // the mode-product GEMMs run in FP64 or FP32 (split BF16 keeps to the in-LDS kernels)
    if (plan == FD_PLAN_GEMM) return precision != HP_PREC_BF16X3;
    if (fd_needs_gemm(c)) return false;
    if (precision == HP_PREC_BF16X3 && plan >= 0 && (plan & 4)) return false;  // not blocked
    return precision == HP_PREC_FP64 ? fd_plan_fits<double>(NMp, plan) : fd_plan_fits<float>(NMp, plan);
}

int fd_plan_in_use(const hp_ctx* c, int precision) {
    if (c->fd_force >= 0) return c->fd_force;
    if (c->opts.fd_plan >= 0 && fd_plan_valid(c, precision, c->opts.fd_plan)) return c->opts.fd_plan;
    if (fd_needs_gemm(c)) return FD_PLAN_GEMM;
    return c->fd_tuned[precision];
}

long long fd_dot_count(const hp_ctx* c, bool vel) {
    const long long nM = c->nM;
    if (fd_plan_in_use(c, HP_PREC_FP64) == FD_PLAN_SPLIT)
        return vel ? 3 * nM * (((nM + 15) & ~15) / 16) : (nM * nM + 15) / 16;
    return vel ? 3 * nM : (nM * nM + ZROWS - 1) / ZROWS;
}

long long fd_dot_capacity(const hp_ctx* c, bool vel) {
    const long long nM = c->nM;
    return vel ? 3 * nM * (((nM + 15) & ~15) / 16) : (nM * nM + 15) / 16;
}

hipError_t launch_P0(hp_ctx* c, const Fields& in, const Fields& out, bool vel, bool pres,
                     bool accumulate, int precision, int nrhs, const FdDot* dot,
                     const FdComb* comb) {
    if (dot && (precision != HP_PREC_FP64 || (vel && pres))) return hipErrorInvalidValue;
    if (fd_plan_in_use(c, precision) == FD_PLAN_GEMM || fd_needs_gemm(c)) {
        // long directions with split BF16 fall back to FP32 products
        if (precision == HP_PREC_FP64)
            return run_P0_gemm<double>(c, c->fd64, in, out, vel, pres, accumulate, nrhs, dot, comb);
        return run_P0_gemm<float>(c, c->fd32, in, out, vel, pres, accumulate, nrhs, dot, comb);
    }
    if (precision == HP_PREC_FP64)
        return run_P0<double>(c, c->fd64, in, out, vel, pres, accumulate, nrhs, dot, comb);
    if (precision == HP_PREC_BF16X3)
        return run_P0<float, true>(c, c->fd32, in, out, vel, pres, accumulate, nrhs, nullptr, comb);
    return run_P0<float>(c, c->fd32, in, out, vel, pres, accumulate, nrhs, nullptr, comb);
}

}  // namespace hp
