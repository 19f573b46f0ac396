// Sum-factorised application of the Stokes saddle-point operator
// (Sec. 3.3, eq. systemmatrix) on gfx950.
//
// With the difference identity C^ = D^T M^ (App. B.1, eq. reduction) the
// blocks of Sec. 3.3 factor as
//     B = D^T M_q,   B^T = M_q D,   A = nu L + nu D^T M_q D,
//     L_1 = M^ (x) M^ (x) K + 2 M^ (x) T^ (x) M + 2 T^ (x) M^ (x) M   (dir 3 (x) dir 2 (x) dir 1)
// (L_2, L_3 by permuting directions), M_q = M^ (x) M^ (x) M^ and D the
// +-1 coefficient difference (the discrete divergence, App. B.2).  Hence
//     K [u; p] = [ nu L u + D^T w ;  M_q D u ],   w = M_q (nu D u + p).
// Every factor is banded (half-width p for the degree-p factors, p-1 for
// the degree p-1 ones), so one application costs O(N p) flops and is bound
// by HBM traffic at large sizes.
//
// Two streaming kernels (the default; a single-pass alternative, k_fused,
// follows them); each reads its inputs and writes its outputs once:
//   k_pres : the pressure chain.  g = D u and z = nu g + p are formed while
//            staging; y_p = M_q g and w = M_q z.
//   k_vel  : per velocity component, y_c = nu L_c u_c + D_c^T w (with an
//            axpby epilogue), or y_c = M_V u_c for the velocity mass matrix.
// A workgroup owns a T1 x T2 tile of the (i1, i2) plane, one point per
// thread, and streams a chunk of i3-planes.  Per plane the tile and its halo
// are staged in LDS; the direction-1 band is applied to the tile's rows and
// halo rows (the thread's column of coefficients in registers), then the
// direction-2 band to the thread's own point (its row of coefficients in
// registers).  The results enter a register window over the last 2w+1 planes,
// from which the direction-3 band (coefficients uniform over the workgroup)
// gives the output plane w planes behind the stream.  The staging loads of
// the next plane are issued before the current plane is processed, so their
// latency overlaps the LDS work.  Tiles are numbered so that neighbouring
// tiles run on the same XCD and share their halo through its L2.
#include <algorithm>

#include "hp_internal.h"

namespace hp {

namespace {

// Tile shape: two-wave workgroups.  Small tiles keep the per-plane chain of
// a workgroup (stage, barrier, band, barrier, band) short and give more
// workgroups per CU to overlap it; the larger halo they re-read comes from L2.
// Measured on apply_K, degree 3 (16x8 against 32x16): 16.0 vs 23.4 us at
// 16^3, 17.7 vs 26.3 us at 32^3, 32.3 vs 40.7 us at 64^3, 329 vs 360 us at
// 192^3; 8x8, 16x4, 8x16 and 32x4 were no faster.
constexpr int T1 = 16;         // direction-1 points per tile
constexpr int T2 = 8;          // direction-2 points per tile
constexpr int NT = T1 * T2;    // threads per workgroup, one tile point each
constexpr int PF = 1;          // planes in flight ahead of the one processed

struct OpArgs {
    BandTables bt;
    const double* u[3];  // velocity inputs (may be null)
    const double* p;     // pressure input (may be null)
    long long su, sp;    // per-rhs strides of the inputs (all u blocks / p)
    double* ws;          // workspace base (holds w)
    long long ws_stride;  // per-rhs workspace stride
    int dims[4][3];
    int nN, nM;
    double nu;
    int mode;
    int kchunk;          // i3-planes per workgroup
    int ntile1, ntile2, nchunk;
    int nblocks;         // workgroups in the launch
    int comp_fast;       // velocity block order (see k_vel)
    int kbase, klim;     // i3-planes [kbase, klim) of this launch (a slab)
};

// Workgroups are dealt round-robin to the 8 XCDs in launch order.  Renumber
// them so that XCD x receives one contiguous range of logical block ids.
__device__ __forceinline__ int xcd_block(int L, int total) {
    const int per = total / 8, rem = total % 8;
    const int x = L % 8, q = L / 8;
    return x * per + min(x, rem) + q;
}

// Register window of the last 2W+1 values along the streamed direction.
template <int W>
struct Window {
    double v[2 * W + 1];
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int t = 0; t <= 2 * W; ++t) v[t] = 0.0;
    }
    __device__ __forceinline__ void push(double x) {
#pragma unroll
        for (int t = 0; t < 2 * W; ++t) v[t] = v[t + 1];
        v[2 * W] = x;
    }
    // sum_t row[t] v[t] for a row of a band table (A[k][k-W .. k+W]); the
    // row index is uniform, so the row is read through the scalar cache
    __device__ __forceinline__ double dot(const double* row_generic) const {
        const auto* row = reinterpret_cast<const __attribute__((address_space(4))) double*>(
            reinterpret_cast<uintptr_t>(row_generic));
        double s = 0.0;
#pragma unroll
        for (int t = 0; t <= 2 * W; ++t) s += row[t] * v[t];
        return s;
    }
};

template <int W>
__device__ __forceinline__ void load_band_row(const double* tab, int row, bool ok,
                                              double (&c)[2 * W + 1]) {
#pragma unroll
    for (int t = 0; t <= 2 * W; ++t) c[t] = ok ? tab[row * (2 * W + 1) + t] : 0.0;
}

// ---- memory access ---------------------------------------------------------------------
// The streaming loops read and write through buffer resources: a per-plane
// base address and byte size in scalar registers plus a per-lane 32-bit byte
// offset that is loop-invariant.  Reads outside the size return zero and
// writes outside it are dropped, so the zero padding of the staged halos,
// planes outside the mesh, fields a mode does not use and lanes without an
// output are all expressed through sizes and offsets: the loop body has no
// branches around memory operations.  The loads for plane kk+PF are issued
// into the registers plane kk has just left (PF register sets, the loop
// unrolled PF times), so no load result is copied while in flight and each
// wait covers only loads issued PF steps earlier;
// an output is stored in the step after it is computed, before that step's
// loads, so that waiting for loaded data never waits for a store issued just
// before it.
constexpr uint32_t OOB = 0x80000000u;  // an offset beyond any buffer size

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    // raw buffer (stride 0), 32-bit data format
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}

// ---- pressure chain --------------------------------------------------------------------
// Staged per plane kk: g = D u and z = nu g + p (z = p for B) on the tile and
// a halo of W = p-1.  u3 at plane kk-1 is the previous plane's u3 value of the
// same staging slot, so each plane reads u3 once.
// waves per SIMD the register budget allows: the band rows and the windows
// grow with the degree
template <int P>
constexpr int waves_for() {
    return P < 4 ? 4 : (P == 4 ? 3 : 2);
}

template <int P, int PT1, int PT2>
__global__ __launch_bounds__(PT1 * PT2) __attribute__((amdgpu_waves_per_eu(waves_for<P>()))) void k_pres(OpArgs a, double* yp, long long syp) {
    constexpr int PNT = PT1 * PT2;
    constexpr int W = P - 1;
    constexpr int SW = PT1 + 2 * W, SR = PT2 + 2 * W;
    constexpr int NS = (SR * SW + PNT - 1) / PNT;  // staging slots per thread
    __shared__ double gs[SR * SW], zs[SR * SW], pg[SR * PT1], pz[SR * PT1];
    const int nM = a.nM, nN = a.nN;
    int id = xcd_block(blockIdx.x, a.nblocks);
    const int t1 = id % a.ntile1;
    id /= a.ntile1;
    const int t2 = id % a.ntile2;
    id /= a.ntile2;
    const int ch = id % a.nchunk;
    const int r = id / a.nchunk;
    const int i0 = t1 * PT1, j0 = t2 * PT2, k0 = a.kbase + ch * a.kchunk;
    const int kend = min(min(k0 + a.kchunk, a.klim), nM);
    const int c = threadIdx.x % PT1, g = threadIdx.x / PT1;
    const int i = i0 + c, j = j0 + g;
    const bool act = i < nM && j < nM;
    const int mode = a.mode;
    const bool need_g = (mode == OP_K || mode == OP_BT);
    const bool need_z = (mode != OP_BT);
    const bool use_u = (mode != OP_B);
    const bool use_p = (mode == OP_K || mode == OP_B);
    const double zg = (mode == OP_B) ? 0.0 : a.nu;   // z = zg g + p
    double* wv = a.ws + (long long)r * a.ws_stride;
    const double* pp = use_p ? a.p + (long long)r * a.sp : wv;
    const double* u1 = use_u ? a.u[0] + (long long)r * a.su : pp;
    const double* u2 = use_u ? a.u[1] + (long long)r * a.su : pp;
    const double* u3 = use_u ? a.u[2] + (long long)r * a.su : pp;
    double* ypr = need_g ? yp + (long long)r * syp : wv;
    const double* tm = a.bt.ptr[BM_C];
    const long long P1 = (long long)nN * nM;   // plane of u1 (nN, nM, nM)
    const long long P2 = (long long)nM * nN;   // plane of u2 (nM, nN, nM)
    const long long P3 = (long long)nM * nM;   // plane of u3 (nM, nM, nN) and of p
    const uint32_t B1 = use_u ? 8u * (uint32_t)P1 : 0u, B2 = use_u ? 8u * (uint32_t)P2 : 0u;
    const uint32_t B3 = use_u ? 8u * (uint32_t)P3 : 0u, BP = use_p ? 8u * (uint32_t)P3 : 0u;
    // staging slots: byte offsets of u1[ii], u1[ii-1], u2[jj], u2[jj-1], and
    // of u3/p, each OOB where the value lies outside its field
    uint32_t oa[NS], ob[NS], oc[NS], od[NS], oe[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int idx = threadIdx.x + s * PNT;
        const int rr = idx / SW, cc = idx - rr * SW;
        const int jj = j0 - W + rr, ii = i0 - W + cc;
        const bool ok = idx < SR * SW && jj >= 0 && jj < nM && ii >= 0 && ii < nM;
        oa[s] = (ok && ii < nN) ? 8u * (nN * jj + ii) : OOB;
        ob[s] = (ok && ii >= 1) ? 8u * (nN * jj + ii - 1) : OOB;
        oc[s] = (ok && jj < nN) ? 8u * (ii + nM * jj) : OOB;
        od[s] = (ok && jj >= 1) ? 8u * (ii + nM * (jj - 1)) : OOB;
        oe[s] = ok ? 8u * (ii + nM * jj) : OOB;
    }
    // Plane addresses advanced by one plane per step (one 64-bit add each
    // instead of a product per plane); a plane outside the mesh gets a
    // zero-size resource, so its address is never dereferenced.
    auto addr = [](const double* base, long long elems) {
        return reinterpret_cast<uint64_t>(base) + (uint64_t)(elems * 8);
    };
    auto ptr = [](uint64_t a) { return reinterpret_cast<const double*>(a); };
    const uint64_t Q1 = 8ull * (uint64_t)P1, Q2 = 8ull * (uint64_t)P2, Q3 = 8ull * (uint64_t)P3;
    // raw values of plane kk (zero outside the mesh) from the plane addresses
    // a[0..3] of u1, u2, u3 and p at kk
    auto fetch = [&](int kk, const uint64_t (&ad)[4], double (&v)[NS][6]) {
        const bool kin = kk >= 0 && kk < nM;
        const bool k3in = kk >= 0 && kk < nN;
        const auto r1 = make_rsrc(ptr(ad[0]), kin ? B1 : 0u);
        const auto r2 = make_rsrc(ptr(ad[1]), kin ? B2 : 0u);
        const auto r3 = make_rsrc(ptr(ad[2]), k3in ? B3 : 0u);
        const auto rp = make_rsrc(ptr(ad[3]), kin ? BP : 0u);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            v[s][0] = bload(r1, oa[s]);
            v[s][1] = bload(r1, ob[s]);
            v[s][2] = bload(r2, oc[s]);
            v[s][3] = bload(r2, od[s]);
            v[s][4] = bload(r3, oe[s]);
            v[s][5] = bload(rp, oe[s]);
        }
    };
    double c1[2 * W + 1], c2[2 * W + 1];
    load_band_row<W>(tm, i, i < nM, c1);
    load_band_row<W>(tm, j, j < nM, c2);
    const uint32_t oo = act ? 8u * (i + nM * j) : OOB;  // this thread's output
    Window<W> wg, wz;
    wg.clear();
    wz.clear();
    auto planes = [&](int kk, uint64_t (&ad)[4]) {
        ad[0] = addr(u1, P1 * kk);
        ad[1] = addr(u2, P2 * kk);
        ad[2] = addr(u3, P3 * kk);
        ad[3] = addr(pp, P3 * kk);
    };
    double buf[PF][NS][6], a3prev[NS];
    {
        double t[NS][6];
        uint64_t ad[4];
        planes(k0 - W - 1, ad);
        fetch(k0 - W - 1, ad, t);
#pragma unroll
        for (int s = 0; s < NS; ++s) a3prev[s] = t[s][4];
    }
#pragma unroll
    for (int d = 0; d < PF; ++d) {
        uint64_t ad[4];
        planes(k0 - W + d, ad);
        fetch(k0 - W + d, ad, buf[d]);
    }
    int pk = -1;  // plane of the pending output (none yet)
    double py = 0.0, pw = 0.0;
    // at the first step kk = k0 - W: input plane kk + PF, pending output kk - W - 1
    uint64_t an[4];
    planes(k0 - W + PF, an);
    uint64_t ayo = addr(ypr, P3 * (k0 - 2 * W - 1)), awo = addr(wv, P3 * (k0 - 2 * W - 1));
    // one step: consume plane kk, store the pending output, refill the
    // registers with plane kk + PF, then process plane kk
    auto step = [&](int kk, double (&b)[NS][6]) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int idx = threadIdx.x + s * PNT;
            if (idx < SR * SW) {
                const double gv = (b[s][0] - b[s][1]) + (b[s][2] - b[s][3]) + (b[s][4] - a3prev[s]);
                gs[idx] = gv;
                zs[idx] = zg * gv + b[s][5];
            }
            a3prev[s] = b[s][4];
        }
        {
            const bool on = pk >= 0;
            bstore(make_rsrc(ptr(ayo), (on && need_g) ? 8u * (uint32_t)P3 : 0u), oo, py);
            bstore(make_rsrc(ptr(awo), (on && need_z) ? 8u * (uint32_t)P3 : 0u), oo, pw);
            ayo += Q3;
            awo += Q3;
        }
        fetch(kk + PF, an, b);
        an[0] += Q1;
        an[1] += Q2;
        an[2] += Q3;
        an[3] += Q3;
        __syncthreads();
        for (int rr = g; rr < SR; rr += PT2) {
            double sg = 0.0, sz = 0.0;
#pragma unroll
            for (int t = 0; t <= 2 * W; ++t) {
                sg += c1[t] * gs[rr * SW + c + t];
                sz += c1[t] * zs[rr * SW + c + t];
            }
            pg[rr * PT1 + c] = sg;
            pz[rr * PT1 + c] = sz;
        }
        __syncthreads();
        double sg = 0.0, sz = 0.0;
#pragma unroll
        for (int t = 0; t <= 2 * W; ++t) {
            sg += c2[t] * pg[(g + t) * PT1 + c];
            sz += c2[t] * pz[(g + t) * PT1 + c];
        }
        wg.push(sg);
        wz.push(sz);
        const int k = kk - W;
        pk = (k >= k0 && k < kend) ? k : -1;
        if (pk >= 0) {
            const double* rm = tm + k * (2 * W + 1);
            py = wg.dot(rm);
            pw = wz.dot(rm);
        }
    };
    // steps past kend + W - 1 (when the count is not a multiple of PF) output nothing
    for (int kk = k0 - W; kk < kend + W; kk += PF) {
#pragma unroll
        for (int d = 0; d < PF; ++d) step(kk + d, buf[d]);
    }
    if (pk >= 0) {
        bstore(make_rsrc(ypr + P3 * pk, need_g ? 8u * (uint32_t)P3 : 0u), oo, py);
        bstore(make_rsrc(wv + P3 * pk, need_z ? 8u * (uint32_t)P3 : 0u), oo, pw);
    }
}

// ---- pressure chain, all planes of a chunk at once --------------------------------------
// The counterpart of k_vel_all for k_pres: the loads of all kc + 2w planes
// (and the u3 plane before them) are issued at once, g and z are formed into
// LDS, directions 1 and 2 are one pass each over all planes and direction 3
// reads the thread's column from registers.  Same operation sequence per
// output as k_pres (bitwise-identical results), every mode k_pres serves.
// KC = kchunk (2 or 4), degrees 2 and 3.
template <int P, int KC>
__global__ __launch_bounds__(NT) void k_pres_all(OpArgs a, double* yp, long long syp) {
    constexpr int W = P - 1;
    constexpr int SW = T1 + 2 * W, SR = T2 + 2 * W;
    constexpr int NS = (SR * SW + NT - 1) / NT;
    constexpr int NP = KC + 2 * W;  // planes k0 - W .. k0 + KC + W - 1
    extern __shared__ double lds_p[];
    double* gs = lds_p;                  // NP x SR x SW
    double* zs = gs + NP * SR * SW;
    double* pg = zs + NP * SR * SW;      // NP x SR x T1
    double* pz = pg + NP * SR * T1;
    const int nM = a.nM, nN = a.nN;
    int id = xcd_block(blockIdx.x, a.nblocks);
    const int t1 = id % a.ntile1;
    id /= a.ntile1;
    const int t2 = id % a.ntile2;
    id /= a.ntile2;
    const int ch = id % a.nchunk;
    const int r = id / a.nchunk;
    const int i0 = t1 * T1, j0 = t2 * T2, k0 = a.kbase + ch * a.kchunk;
    const int kend = min(min(k0 + a.kchunk, a.klim), nM);
    const int c = threadIdx.x % T1, g = threadIdx.x / T1;
    const int i = i0 + c, j = j0 + g;
    const bool act = i < nM && j < nM;
    const int mode = a.mode;
    const bool need_g = (mode == OP_K || mode == OP_BT);
    const bool need_z = (mode != OP_BT);
    const bool use_u = (mode != OP_B);
    const bool use_p = (mode == OP_K || mode == OP_B);
    const double zg = (mode == OP_B) ? 0.0 : a.nu;   // z = zg g + p
    double* wv = a.ws + (long long)r * a.ws_stride;
    const double* pp = use_p ? a.p + (long long)r * a.sp : wv;
    const double* u1 = use_u ? a.u[0] + (long long)r * a.su : pp;
    const double* u2 = use_u ? a.u[1] + (long long)r * a.su : pp;
    const double* u3 = use_u ? a.u[2] + (long long)r * a.su : pp;
    double* ypr = need_g ? yp + (long long)r * syp : wv;
    const double* tm = a.bt.ptr[BM_C];
    const long long P1 = (long long)nN * nM;
    const long long P2 = (long long)nM * nN;
    const long long P3 = (long long)nM * nM;
    const uint32_t B1 = use_u ? 8u * (uint32_t)P1 : 0u, B2 = use_u ? 8u * (uint32_t)P2 : 0u;
    const uint32_t B3 = use_u ? 8u * (uint32_t)P3 : 0u, BP = use_p ? 8u * (uint32_t)P3 : 0u;
    uint32_t oa[NS], ob[NS], oc[NS], od[NS], oe[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int idx = threadIdx.x + s * NT;
        const int rr = idx / SW, cc = idx - rr * SW;
        const int jj = j0 - W + rr, ii = i0 - W + cc;
        const bool ok = idx < SR * SW && jj >= 0 && jj < nM && ii >= 0 && ii < nM;
        oa[s] = (ok && ii < nN) ? 8u * (nN * jj + ii) : OOB;
        ob[s] = (ok && ii >= 1) ? 8u * (nN * jj + ii - 1) : OOB;
        oc[s] = (ok && jj < nN) ? 8u * (ii + nM * jj) : OOB;
        od[s] = (ok && jj >= 1) ? 8u * (ii + nM * (jj - 1)) : OOB;
        oe[s] = ok ? 8u * (ii + nM * jj) : OOB;
    }
    // every load of the workgroup first: u3 from plane k0 - W - 1 on, the
    // other values from plane k0 - W on
    double v1a[NP][NS], v1b[NP][NS], v2c[NP][NS], v2d[NP][NS], vp[NP][NS], v3[NP + 1][NS];
#pragma unroll
    for (int q = 0; q <= NP; ++q) {
        const int kk = k0 - W - 1 + q;
        const bool k3in = kk >= 0 && kk < nN;
        const auto r3 = make_rsrc(u3 + P3 * (k3in ? kk : 0), k3in ? B3 : 0u);
#pragma unroll
        for (int s = 0; s < NS; ++s) v3[q][s] = bload(r3, oe[s]);
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int kk = k0 - W + q;
        const bool kin = kk >= 0 && kk < nM;
        const int kc = kin ? kk : 0;
        const auto r1 = make_rsrc(u1 + P1 * kc, kin ? B1 : 0u);
        const auto r2 = make_rsrc(u2 + P2 * kc, kin ? B2 : 0u);
        const auto rp = make_rsrc(pp + P3 * kc, kin ? BP : 0u);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            v1a[q][s] = bload(r1, oa[s]);
            v1b[q][s] = bload(r1, ob[s]);
            v2c[q][s] = bload(r2, oc[s]);
            v2d[q][s] = bload(r2, od[s]);
            vp[q][s] = bload(rp, oe[s]);
        }
    }
    double c1[2 * W + 1], c2[2 * W + 1];
    load_band_row<W>(tm, i, i < nM, c1);
    load_band_row<W>(tm, j, j < nM, c2);
    const uint32_t oo = act ? 8u * (i + nM * j) : OOB;
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int idx = threadIdx.x + s * NT;
            if (idx < SR * SW) {
                const double gv = (v1a[q][s] - v1b[q][s]) + (v2c[q][s] - v2d[q][s]) +
                                  (v3[q + 1][s] - v3[q][s]);
                gs[q * SR * SW + idx] = gv;
                zs[q * SR * SW + idx] = zg * gv + vp[q][s];
            }
        }
    __syncthreads();
    for (int q = 0; q < NP; ++q) {
        const double* gq = gs + q * SR * SW;
        const double* zq = zs + q * SR * SW;
        for (int rr = g; rr < SR; rr += T2) {
            double sg = 0.0, sz = 0.0;
#pragma unroll
            for (int t = 0; t <= 2 * W; ++t) {
                sg += c1[t] * gq[rr * SW + c + t];
                sz += c1[t] * zq[rr * SW + c + t];
            }
            pg[q * SR * T1 + rr * T1 + c] = sg;
            pz[q * SR * T1 + rr * T1 + c] = sz;
        }
    }
    __syncthreads();
    double sgv[NP], szv[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        double sg = 0.0, sz = 0.0;
#pragma unroll
        for (int t = 0; t <= 2 * W; ++t) {
            sg += c2[t] * pg[q * SR * T1 + (g + t) * T1 + c];
            sz += c2[t] * pz[q * SR * T1 + (g + t) * T1 + c];
        }
        sgv[q] = sg;
        szv[q] = sz;
    }
#pragma unroll
    for (int o = 0; o < KC; ++o) {
        const int k = k0 + o;
        const bool on = k < kend;
        const int kc = on ? k : k0;
        Window<W> wg, wz;
#pragma unroll
        for (int t = 0; t <= 2 * W; ++t) {
            wg.v[t] = sgv[o + t];
            wz.v[t] = szv[o + t];
        }
        const double* rm = tm + kc * (2 * W + 1);
        const double py = wg.dot(rm);
        const double pw = wz.dot(rm);
        bstore(make_rsrc(ypr + P3 * kc, (on && need_g) ? 8u * (uint32_t)P3 : 0u), oo, py);
        bstore(make_rsrc(wv + P3 * kc, (on && need_z) ? 8u * (uint32_t)P3 : 0u), oo, pw);
    }
}

template <int P, int KC>
constexpr int pres_all_lds_doubles() {
    constexpr int W = P - 1, SW = T1 + 2 * W, SR = T2 + 2 * W, NP = KC + 2 * W;
    return NP * (2 * SR * SW + 2 * SR * T1);
}

// ---- velocity component C --------------------------------------------------------------
template <int P, int C>
__device__ void vel_component(const OpArgs& a, const Fields& out, const Fields& src, double alpha,
                              double beta, int r, int i0, int j0, int k0, double* lds) {
    constexpr int W1 = (C == 0) ? P : P - 1;
    constexpr int W2 = (C == 1) ? P : P - 1;
    constexpr int W3 = (C == 2) ? P : P - 1;
    constexpr int SW = T1 + 2 * W1, SR = T2 + 2 * W2;
    constexpr int NS = (SR * SW + NT - 1) / NT;
    const int n1 = a.dims[C][0], n2 = a.dims[C][1], n3 = a.dims[C][2];
    if (i0 >= n1 || j0 >= n2 || k0 >= n3) return;
    const int kend = min(min(k0 + a.kchunk, a.klim), n3);
    const int c = threadIdx.x % T1, g = threadIdx.x / T1;
    const int i = i0 + c, j = j0 + g;
    const bool act = i < n1 && j < n2;
    const int mode = a.mode;
    const bool mv = (mode == OP_MV);
    const bool lop = (mode == OP_K || mode == OP_A);
    const int nM = a.nM;
    const double* wv = a.ws + (long long)r * a.ws_stride;
    const long long plane = (long long)n1 * n2;
    const long long wplane = (long long)nM * nM;
    const uint32_t YB = 8u * (uint32_t)plane, WB = 8u * (uint32_t)wplane;
    double* y = out.f[C] + (long long)r * out.stride[C];
    const bool has_src = beta != 0.0;
    const double* sv = has_src ? src.f[C] + (long long)r * src.stride[C] : y;
    const uint32_t SB = has_src ? YB : 0u;
    const uint32_t WBm = mv ? 0u : WB;  // the mass mode has no coupling term
    // this thread's point: byte offsets in the pressure plane (w at i, j and at
    // the +1 neighbour in direction C) and in the component plane
    const uint32_t wo = act ? 8u * (i + nM * j) : OOB;
    const uint32_t wo1 = act ? wo + (C == 0 ? 8u : C == 1 ? 8u * nM : 0u) : OOB;
    const uint32_t yo = act ? 8u * (i + n1 * j) : OOB;
    if (!lop && !mv) {
        // coupling only (B): y = alpha D_c^T w + beta src, four planes per
        // step with all their loads issued before the first is used
        if (!act) return;
        constexpr int U = 4;
        for (int k = k0; k < kend; k += U) {
            double a0[U], a1[U], sd[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = k + u < kend;
                const int kc = ok ? k + u : k0;
                a0[u] = bload(make_rsrc(wv + wplane * kc, ok ? WB : 0u), wo);
                a1[u] = bload(make_rsrc(wv + wplane * (C == 2 ? kc + 1 : kc), ok ? WB : 0u), wo1);
                sd[u] = bload(make_rsrc(sv + plane * kc, ok ? SB : 0u), yo);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = k + u < kend;
                const int kc = ok ? k + u : k0;
                bstore(make_rsrc(y + plane * kc, ok ? YB : 0u), yo,
                       alpha * (a0[u] - a1[u]) + beta * sd[u]);
            }
        }
        return;
    }
    double* xs = lds;             // SR x SW
    double* pa = xs + SR * SW;    // SR x T1
    double* pb = pa + SR * T1;
    const double* t1a = a.bt.ptr[C == 0 ? (mv ? BM_N : BK_N) : BM_C];
    const double* t1b = a.bt.ptr[C == 0 ? BM_N : BT_C];
    const double* m2t = a.bt.ptr[C == 1 ? BM_N : BM_C];   // mass of direction 2
    const double* k2t = a.bt.ptr[C == 1 ? BK_N : BT_C];   // K (C==1) or T^ (C==0, 2)
    const double* ta = a.bt.ptr[C == 2 ? (mv ? BM_N : BK_N) : BM_C];
    const double* tb = a.bt.ptr[C == 2 ? BM_N : BT_C];
    const double* x = a.u[C] + (long long)r * a.su;
    uint32_t so[NS];  // staging byte offsets, OOB outside the component
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int idx = threadIdx.x + s * NT;
        const int rr = idx / SW, cc = idx - rr * SW;
        const int jj = j0 - W2 + rr, ii = i0 - W1 + cc;
        const bool ok = idx < SR * SW && jj >= 0 && jj < n2 && ii >= 0 && ii < n1;
        so[s] = ok ? 8u * (jj * n1 + ii) : OOB;
    }
    auto fetch_x = [&](int kk, double (&v)[NS]) {
        const bool kin = kk >= 0 && kk < n3;
        const auto rx = make_rsrc(x + plane * (kin ? kk : 0), kin ? YB : 0u);
#pragma unroll
        for (int s = 0; s < NS; ++s) v[s] = bload(rx, so[s]);
    };
    // coupling (w at the point and at its +1 neighbour) and source of plane k
    auto fetch_out = [&](int k, double& w0, double& w1, double& sd) {
        const bool kin = k >= 0 && k < n3;
        const int kc = kin ? k : 0;
        w0 = bload(make_rsrc(wv + wplane * kc, kin ? WBm : 0u), wo);
        w1 = bload(make_rsrc(wv + wplane * (C == 2 ? kc + 1 : kc), kin ? WBm : 0u), wo1);
        sd = bload(make_rsrc(sv + plane * kc, kin ? SB : 0u), yo);
    };
    double ca[2 * W1 + 1], cb[2 * W1 + 1], cm[2 * W2 + 1], ck[2 * W2 + 1];
    load_band_row<W1>(t1a, i, i < n1, ca);
    load_band_row<W1>(t1b, i, i < n1 && !mv, cb);
    load_band_row<W2>(m2t, j, j < n2, cm);
    load_band_row<W2>(k2t, j, j < n2 && !mv, ck);
    Window<W3> wa, wb;
    wa.clear();
    wb.clear();
    struct OutTerms {
        double w0, w1, sd;
    };
    double xb[PF][NS];
    OutTerms ft[PF];
#pragma unroll
    for (int d = 0; d < PF; ++d) {
        fetch_x(k0 - W3 + d, xb[d]);
        fetch_out(k0 - 2 * W3 + d, ft[d].w0, ft[d].w1, ft[d].sd);
    }
    int pk = -1;  // plane of the pending output (none yet)
    double pv = 0.0;
    // one step: consume plane kk, store the pending output, refill the
    // registers with plane kk + PF, process plane kk, form the output of
    // plane kk - W3 and refill its coupling/source registers for kk - W3 + PF
    auto step = [&](int kk, double (&xr)[NS], OutTerms& f) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int idx = threadIdx.x + s * NT;
            if (idx < SR * SW) xs[idx] = xr[s];
        }
        bstore(make_rsrc(y + plane * (pk >= 0 ? pk : 0), pk >= 0 ? YB : 0u), yo, pv);
        fetch_x(kk + PF, xr);
        __syncthreads();
        for (int rr = g; rr < SR; rr += T2) {
            double sa = 0.0, sb = 0.0;
#pragma unroll
            for (int t = 0; t <= 2 * W1; ++t) {
                const double xv = xs[rr * SW + c + t];
                sa += ca[t] * xv;
                sb += cb[t] * xv;
            }
            pa[rr * T1 + c] = sa;
            pb[rr * T1 + c] = sb;
        }
        __syncthreads();
        double am = 0.0, ak = 0.0, bm = 0.0, bk = 0.0;
#pragma unroll
        for (int t = 0; t <= 2 * W2; ++t) {
            const double va = pa[(g + t) * T1 + c], vb = pb[(g + t) * T1 + c];
            am += cm[t] * va;
            ak += ck[t] * va;
            bm += cm[t] * vb;
            bk += ck[t] * vb;
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
        wa.push(ga);
        wb.push(gb);
        const int k = kk - W3;
        pk = (k >= k0 && k < kend) ? k : -1;
        if (pk >= 0) {
            double v;
            if (mv) v = wa.dot(ta + k * (2 * W3 + 1));
            else v = a.nu * (wa.dot(ta + k * (2 * W3 + 1)) + wb.dot(tb + k * (2 * W3 + 1))) + (f.w0 - f.w1);
            pv = alpha * v + beta * f.sd;
        }
        fetch_out(k + PF, f.w0, f.w1, f.sd);
    };
    // steps past kend + W3 - 1 (when the count is not a multiple of PF) output nothing
    for (int kk = k0 - W3; kk < kend + W3; kk += PF) {
#pragma unroll
        for (int d = 0; d < PF; ++d) step(kk + d, xb[d], ft[d]);
    }
    if (pk >= 0) bstore(make_rsrc(y + plane * pk, YB), yo, pv);
}

template <int P>
constexpr int vel_lds_doubles() {
    // the widest component: halo P in one of the two tile directions
    return (T2 + 2 * P) * (T1 + 2 * P) + 2 * (T2 + 2 * P) * T1;
}

template <int P>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(waves_for<P>()))) void k_vel(OpArgs a, Fields out, Fields src, double alpha,
                                            double beta) {
    __shared__ double lds[vel_lds_doubles<P>()];
    int id = xcd_block(blockIdx.x, a.nblocks);
    // order 1: the component is the fastest index, so that the three
    // components of one tile and chunk run together on one XCD and read w
    // through its L2 once; order 0: tiles fastest, components slowest
    int comp;
    if (a.comp_fast) {
        comp = id % 3;
        id /= 3;
    }
    const int t1 = id % a.ntile1;
    id /= a.ntile1;
    const int t2 = id % a.ntile2;
    id /= a.ntile2;
    const int ch = id % a.nchunk;
    id /= a.nchunk;
    if (!a.comp_fast) {
        comp = id % 3;
        id /= 3;
    }
    const int r = id;
    const int i0 = t1 * T1, j0 = t2 * T2, k0 = a.kbase + ch * a.kchunk;
    if (comp == 0) vel_component<P, 0>(a, out, src, alpha, beta, r, i0, j0, k0, lds);
    else if (comp == 1) vel_component<P, 1>(a, out, src, alpha, beta, r, i0, j0, k0, lds);
    else vel_component<P, 2>(a, out, src, alpha, beta, r, i0, j0, k0, lds);
}

// ---- velocity component C, planes staged by direct-to-LDS loads -------------------------
// The streaming velocity kernel above keeps one plane in flight, in
// registers: its waves wait on memory most of the time, and deeper register
// prefetch costs more occupancy than it adds.  This variant stages the tile
// and halo of each plane with buffer loads that write LDS directly
// (buffer_load_dword ... lds, no registers), into a ring of three LDS
// slots, so two planes are in flight.  The staged array is the same SR x SW
// doubles as xs, filled as 2 SR SW dwords by consecutive lanes (lane l of
// load s of wave w writes dword s NT + 64 w + l; lanes past the array write
// into the slot's padding, so every load of a plane is issued by every
// lane and the count per plane is fixed).  Each slot is its own __shared__
// array so that the compiler's wait for the loads into one slot leaves the
// later slots' loads in flight; a read of the thread's own element of the
// slot before the barrier makes the compiler wait for this wave's loads of
// that plane there, and the barrier (with only an LDS wait, no fence: a
// fence would wait for every load in flight) then orders every wave's.  The
// arithmetic per output is vel_component's, so the results agree bit for bit.
template <int P, int C>
constexpr int dma_dwords() {
    constexpr int W1 = (C == 0) ? P : P - 1, W2 = (C == 1) ? P : P - 1;
    return ((2 * (T2 + 2 * W2) * (T1 + 2 * W1) + NT - 1) / NT) * NT;
}
template <int P>
constexpr int dma_slot_doubles() {
    constexpr int a = dma_dwords<P, 0>(), b = dma_dwords<P, 1>(), c = dma_dwords<P, 2>();
    return (a > b ? (a > c ? a : c) : (b > c ? b : c)) / 2;
}
typedef __attribute__((address_space(3))) void* lds_vptr;
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int P, int C>
__device__ void vel_component_dma(const OpArgs& a, const Fields& out, const Fields& src,
                                  double alpha, double beta, int r, int i0, int j0, int k0,
                                  double* s0, double* s1, double* s2, double* pab) {
    constexpr int W1 = (C == 0) ? P : P - 1;
    constexpr int W2 = (C == 1) ? P : P - 1;
    constexpr int W3 = (C == 2) ? P : P - 1;
    constexpr int SW = T1 + 2 * W1, SR = T2 + 2 * W2;
    constexpr int ND = dma_dwords<P, C>() / NT;  // dword loads per thread and plane
    const int n1 = a.dims[C][0], n2 = a.dims[C][1], n3 = a.dims[C][2];
    if (i0 >= n1 || j0 >= n2 || k0 >= n3) return;
    const int kend = min(min(k0 + a.kchunk, a.klim), n3);
    const int c = threadIdx.x % T1, g = threadIdx.x / T1;
    const int i = i0 + c, j = j0 + g;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // uniform
    const bool act = i < n1 && j < n2;
    const int mode = a.mode;
    const bool mv = (mode == OP_MV);
    const int nM = a.nM;
    const double* wv = a.ws + (long long)r * a.ws_stride;
    const long long plane = (long long)n1 * n2;
    const long long wplane = (long long)nM * nM;
    const uint32_t YB = 8u * (uint32_t)plane, WB = 8u * (uint32_t)wplane;
    double* y = out.f[C] + (long long)r * out.stride[C];
    const bool has_src = beta != 0.0;
    const double* sv = has_src ? src.f[C] + (long long)r * src.stride[C] : y;
    const uint32_t SB = has_src ? YB : 0u;
    const uint32_t WBm = mv ? 0u : WB;
    const uint32_t wo = act ? 8u * (i + nM * j) : OOB;
    const uint32_t wo1 = act ? wo + (C == 0 ? 8u : C == 1 ? 8u * nM : 0u) : OOB;
    const uint32_t yo = act ? 8u * (i + n1 * j) : OOB;
    double* pa = pab;
    double* pb = pab + SR * T1;
    const double* t1a = a.bt.ptr[C == 0 ? (mv ? BM_N : BK_N) : BM_C];
    const double* t1b = a.bt.ptr[C == 0 ? BM_N : BT_C];
    const double* m2t = a.bt.ptr[C == 1 ? BM_N : BM_C];
    const double* k2t = a.bt.ptr[C == 1 ? BK_N : BT_C];
    const double* ta = a.bt.ptr[C == 2 ? (mv ? BM_N : BK_N) : BM_C];
    const double* tb = a.bt.ptr[C == 2 ? BM_N : BT_C];
    const double* x = a.u[C] + (long long)r * a.su;
    // byte offsets of this thread's dwords of the staged plane (OOB outside
    // the component and in the padding)
    uint32_t so[ND];
#pragma unroll
    for (int s = 0; s < ND; ++s) {
        const int d = threadIdx.x + s * NT;
        const int idx = d >> 1;
        const int rr = idx / SW, cc = idx - rr * SW;
        const int jj = j0 - W2 + rr, ii = i0 - W1 + cc;
        const bool ok = idx < SR * SW && jj >= 0 && jj < n2 && ii >= 0 && ii < n1;
        so[s] = ok ? 8u * (jj * n1 + ii) + 4u * (d & 1) : OOB;
    }
    // The planes a step touches, as byte addresses advanced by one plane per
    // step (one 64-bit add each instead of a product per plane); a plane
    // outside the field gets a zero-size resource, so its address, which may
    // lie outside the field, is never dereferenced.
    const uint64_t PY = 8ull * (uint64_t)plane, PW = 8ull * (uint64_t)wplane;
    auto addr = [](const double* base, long long elems) {
        return reinterpret_cast<uint64_t>(base) + (uint64_t)(elems * 8);
    };
    auto ptr = [](uint64_t a) { return reinterpret_cast<const double*>(a); };
    auto fetch_x = [&](int kk, uint64_t ax, double* slot) {
        const bool kin = kk >= 0 && kk < n3;
        const auto rx = make_rsrc(ptr(ax), kin ? YB : 0u);
        uint32_t* base = reinterpret_cast<uint32_t*>(slot) + 64 * wave;
#pragma unroll
        for (int s = 0; s < ND; ++s)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (lds_vptr)(base + s * NT), 4, so[s], 0, 0,
                                                     0);
    };
    auto fetch_out = [&](int k, uint64_t aw, uint64_t as, double& w0, double& w1, double& sd) {
        const bool kin = k >= 0 && k < n3;
        w0 = bload(make_rsrc(ptr(aw), kin ? WBm : 0u), wo);
        w1 = bload(make_rsrc(ptr(C == 2 ? aw + PW : aw), kin ? WBm : 0u), wo1);
        sd = bload(make_rsrc(ptr(as), kin ? SB : 0u), yo);
    };
    double ca[2 * W1 + 1], cb[2 * W1 + 1], cm[2 * W2 + 1], ck[2 * W2 + 1];
    load_band_row<W1>(t1a, i, i < n1, ca);
    load_band_row<W1>(t1b, i, i < n1 && !mv, cb);
    load_band_row<W2>(m2t, j, j < n2, cm);
    load_band_row<W2>(k2t, j, j < n2 && !mv, ck);
    Window<W3> wa, wb;
    wa.clear();
    wb.clear();
    double fw0, fw1, fsd;
    fetch_x(k0 - W3, addr(x, plane * (k0 - W3)), s0);
    fetch_x(k0 - W3 + 1, addr(x, plane * (k0 - W3 + 1)), s1);
    fetch_out(k0 - 2 * W3, addr(wv, wplane * (k0 - 2 * W3)), addr(sv, plane * (k0 - 2 * W3)), fw0,
              fw1, fsd);
    int pk = -1;
    double pv = 0.0;
    // at the first step kk = k0 - W3: x plane kk + 2, output plane kk - W3 - 1,
    // coupling and source planes kk - W3 + 1
    uint64_t ax = addr(x, plane * (k0 - W3 + 2));
    uint64_t ay = addr(y, plane * (k0 - 2 * W3 - 1));
    uint64_t aw = addr(wv, wplane * (k0 - 2 * W3 + 1));
    uint64_t as = addr(sv, plane * (k0 - 2 * W3 + 1));
    // one step: wait for plane kk (slot cur), start plane kk + 2 into the
    // slot plane kk - 1 used, store the pending output, process plane kk
    auto step = [&](int kk, double* cur, double* nxt) {
        {
            const double probe = cur[threadIdx.x];
            asm volatile("" ::"v"(probe));
        }
        lds_barrier();
        fetch_x(kk + 2, ax, nxt);
        ax += PY;
        // the pending output (plane kk - W3 - 1, if it is one)
        bstore(make_rsrc(ptr(ay), pk >= 0 ? YB : 0u), yo, pv);
        ay += PY;
        // direction 1 over rows g, g + T2, ... (unrolled: a loop would make the
        // compiler wait for every load into LDS at its header)
#pragma unroll
        for (int m = 0; m < (SR + T2 - 1) / T2; ++m) {
            const int rr = g + m * T2;
            if (rr < SR) {
                double sa = 0.0, sb = 0.0;
#pragma unroll
                for (int t = 0; t <= 2 * W1; ++t) {
                    const double xv = cur[rr * SW + c + t];
                    sa += ca[t] * xv;
                    sb += cb[t] * xv;
                }
                pa[rr * T1 + c] = sa;
                pb[rr * T1 + c] = sb;
            }
        }
        lds_barrier();
        double am = 0.0, ak = 0.0, bm = 0.0, bk = 0.0;
#pragma unroll
        for (int t = 0; t <= 2 * W2; ++t) {
            const double va = pa[(g + t) * T1 + c], vb = pb[(g + t) * T1 + c];
            am += cm[t] * va;
            ak += ck[t] * va;
            bm += cm[t] * vb;
            bk += ck[t] * vb;
        }
        double ga, gb = 0.0;
        if (mv) {
            ga = am;
        } else if (C == 0) {
            ga = am + 2.0 * bk;
            gb = 2.0 * bm;
        } else if (C == 1) {
            ga = ak + 2.0 * bm;
            gb = 2.0 * am;
        } else {
            ga = am;
            gb = 2.0 * (ak + bm);
        }
        wa.push(ga);
        wb.push(gb);
        const int k = kk - W3;
        pk = (k >= k0 && k < kend) ? k : -1;
        if (pk >= 0) {
            double v;
            if (mv) v = wa.dot(ta + k * (2 * W3 + 1));
            else v = a.nu * (wa.dot(ta + k * (2 * W3 + 1)) + wb.dot(tb + k * (2 * W3 + 1))) + (fw0 - fw1);
            pv = alpha * v + beta * fsd;
        }
        fetch_out(k + 1, aw, as, fw0, fw1, fsd);
        aw += PW;
        as += PY;
    };
    for (int kk = k0 - W3; kk < kend + W3; kk += 3) {
        step(kk, s0, s2);
        step(kk + 1, s1, s0);
        step(kk + 2, s2, s1);
    }
    if (pk >= 0) bstore(make_rsrc(y + plane * pk, YB), yo, pv);
    // no load into LDS may outlive the workgroup
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

template <int P>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(waves_for<P>()))) void k_vel_dma(
    OpArgs a, Fields out, Fields src, double alpha, double beta) {
    constexpr int SL = dma_slot_doubles<P>();
    __shared__ double s0[SL], s1[SL], s2[SL], pab[2 * (T2 + 2 * P) * T1];
    int id = xcd_block(blockIdx.x, a.nblocks);
    int comp;
    if (a.comp_fast) {
        comp = id % 3;
        id /= 3;
    }
    const int t1 = id % a.ntile1;
    id /= a.ntile1;
    const int t2 = id % a.ntile2;
    id /= a.ntile2;
    const int ch = id % a.nchunk;
    id /= a.nchunk;
    if (!a.comp_fast) {
        comp = id % 3;
        id /= 3;
    }
    const int r = id;
    const int i0 = t1 * T1, j0 = t2 * T2, k0 = a.kbase + ch * a.kchunk;
    if (a.mode != OP_K && a.mode != OP_A && a.mode != OP_MV) {
        // the coupling-only modes stage nothing
        if (comp == 0) vel_component<P, 0>(a, out, src, alpha, beta, r, i0, j0, k0, pab);
        else if (comp == 1) vel_component<P, 1>(a, out, src, alpha, beta, r, i0, j0, k0, pab);
        else vel_component<P, 2>(a, out, src, alpha, beta, r, i0, j0, k0, pab);
        return;
    }
    if (comp == 0) vel_component_dma<P, 0>(a, out, src, alpha, beta, r, i0, j0, k0, s0, s1, s2, pab);
    else if (comp == 1) vel_component_dma<P, 1>(a, out, src, alpha, beta, r, i0, j0, k0, s0, s1, s2, pab);
    else vel_component_dma<P, 2>(a, out, src, alpha, beta, r, i0, j0, k0, s0, s1, s2, pab);
}

// ---- velocity, all planes of a chunk at once (K and A) ------------------------------------
// For small meshes, where k_vel's per-plane chain (stage, barrier, band,
// barrier, band) repeated kc + 2w times sets its duration, this variant
// issues the loads of all kc + 2w planes of its tile and halo (and of every
// output's coupling and source) at once, applies direction 1 and direction 2
// as one pass each over all planes, and forms direction 3 from the thread's
// own column of results in registers.  Each output is the same sequence of
// floating-point operations as in k_vel, so the results agree bit for bit.
// KC = kchunk (2, 4 or 8), degrees 2..4.
template <int P, int C, int KC>
__device__ void vel_component_all(const OpArgs& a, const Fields& out, const Fields& src,
                                  double alpha, double beta, int r, int i0, int j0, int k0,
                                  double* lds) {
    constexpr int W1 = (C == 0) ? P : P - 1;
    constexpr int W2 = (C == 1) ? P : P - 1;
    constexpr int W3 = (C == 2) ? P : P - 1;
    constexpr int SW = T1 + 2 * W1, SR = T2 + 2 * W2;
    constexpr int NS = (SR * SW + NT - 1) / NT;
    constexpr int NP = KC + 2 * W3;  // staged planes k0 - W3 .. k0 + KC + W3 - 1
    const int n1 = a.dims[C][0], n2 = a.dims[C][1], n3 = a.dims[C][2];
    if (i0 >= n1 || j0 >= n2 || k0 >= n3) return;
    const int kend = min(min(k0 + a.kchunk, a.klim), n3);
    const int c = threadIdx.x % T1, g = threadIdx.x / T1;
    const int i = i0 + c, j = j0 + g;
    const bool act = i < n1 && j < n2;
    const int nM = a.nM;
    const double* wv = a.ws + (long long)r * a.ws_stride;
    const long long plane = (long long)n1 * n2;
    const long long wplane = (long long)nM * nM;
    const uint32_t YB = 8u * (uint32_t)plane, WB = 8u * (uint32_t)wplane;
    double* y = out.f[C] + (long long)r * out.stride[C];
    const bool has_src = beta != 0.0;
    const double* sv = has_src ? src.f[C] + (long long)r * src.stride[C] : y;
    const uint32_t SB = has_src ? YB : 0u;
    const uint32_t wo = act ? 8u * (i + nM * j) : OOB;
    const uint32_t wo1 = act ? wo + (C == 0 ? 8u : C == 1 ? 8u * nM : 0u) : OOB;
    const uint32_t yo = act ? 8u * (i + n1 * j) : OOB;
    const double* x = a.u[C] + (long long)r * a.su;
    uint32_t so[NS];  // staging byte offsets, OOB outside the component
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int idx = threadIdx.x + s * NT;
        const int rr = idx / SW, cc = idx - rr * SW;
        const int jj = j0 - W2 + rr, ii = i0 - W1 + cc;
        const bool ok = idx < SR * SW && jj >= 0 && jj < n2 && ii >= 0 && ii < n1;
        so[s] = ok ? 8u * (jj * n1 + ii) : OOB;
    }
    // every load of the workgroup, issued before the first is used
    double xr[NP][NS];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int kk = k0 - W3 + q;
        const bool kin = kk >= 0 && kk < n3;
        const auto rx = make_rsrc(x + plane * (kin ? kk : 0), kin ? YB : 0u);
#pragma unroll
        for (int s = 0; s < NS; ++s) xr[q][s] = bload(rx, so[s]);
    }
    double w0[KC], w1[KC], sd[KC];
#pragma unroll
    for (int o = 0; o < KC; ++o) {
        const int k = k0 + o;
        const bool on = k < kend;
        const int kc = on ? k : k0;
        w0[o] = bload(make_rsrc(wv + wplane * kc, on ? WB : 0u), wo);
        w1[o] = bload(make_rsrc(wv + wplane * (C == 2 ? kc + 1 : kc), on ? WB : 0u), wo1);
        sd[o] = bload(make_rsrc(sv + plane * kc, on ? SB : 0u), yo);
    }
    const double* t1a = a.bt.ptr[C == 0 ? BK_N : BM_C];
    const double* t1b = a.bt.ptr[C == 0 ? BM_N : BT_C];
    const double* m2t = a.bt.ptr[C == 1 ? BM_N : BM_C];
    const double* k2t = a.bt.ptr[C == 1 ? BK_N : BT_C];
    const double* ta = a.bt.ptr[C == 2 ? BK_N : BM_C];
    const double* tb = a.bt.ptr[C == 2 ? BM_N : BT_C];
    double ca[2 * W1 + 1], cb[2 * W1 + 1], cm[2 * W2 + 1], ck[2 * W2 + 1];
    load_band_row<W1>(t1a, i, i < n1, ca);
    load_band_row<W1>(t1b, i, i < n1, cb);
    load_band_row<W2>(m2t, j, j < n2, cm);
    load_band_row<W2>(k2t, j, j < n2, ck);
    double* xs = lds;                    // NP x SR x SW
    double* pa = xs + NP * SR * SW;      // NP x SR x T1
    double* pb = pa + NP * SR * T1;
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int idx = threadIdx.x + s * NT;
            if (idx < SR * SW) xs[q * SR * SW + idx] = xr[q][s];
        }
    __syncthreads();
    // direction 1 over the tile rows and halo rows of every plane
    for (int q = 0; q < NP; ++q) {
        const double* xq = xs + q * SR * SW;
        for (int rr = g; rr < SR; rr += T2) {
            double sa = 0.0, sb = 0.0;
#pragma unroll
            for (int t = 0; t <= 2 * W1; ++t) {
                const double xv = xq[rr * SW + c + t];
                sa += ca[t] * xv;
                sb += cb[t] * xv;
            }
            pa[q * SR * T1 + rr * T1 + c] = sa;
            pb[q * SR * T1 + rr * T1 + c] = sb;
        }
    }
    __syncthreads();
    // direction 2 at the thread's point of every plane
    double gav[NP], gbv[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const double* paq = pa + q * SR * T1;
        const double* pbq = pb + q * SR * T1;
        double am = 0.0, ak = 0.0, bm = 0.0, bk = 0.0;
#pragma unroll
        for (int t = 0; t <= 2 * W2; ++t) {
            const double va = paq[(g + t) * T1 + c], vb = pbq[(g + t) * T1 + c];
            am += cm[t] * va;
            ak += ck[t] * va;
            bm += cm[t] * vb;
            bk += ck[t] * vb;
        }
        double ga, gb = 0.0;
        if (C == 0) {
            ga = am + 2.0 * bk;
            gb = 2.0 * bm;
        } else if (C == 1) {
            ga = ak + 2.0 * bm;
            gb = 2.0 * am;
        } else {
            ga = am;
            gb = 2.0 * (ak + bm);
        }
        gav[q] = ga;
        gbv[q] = gb;
    }
    // direction 3 (band rows uniform over the workgroup, read through the
    // scalar cache) and the epilogue
#pragma unroll
    for (int o = 0; o < KC; ++o) {
        const int k = k0 + o;
        const bool on = k < kend;
        const int kc = on ? k : k0;
        Window<W3> wa, wb;
#pragma unroll
        for (int t = 0; t <= 2 * W3; ++t) {
            wa.v[t] = gav[o + t];
            wb.v[t] = gbv[o + t];
        }
        const double v = a.nu * (wa.dot(ta + kc * (2 * W3 + 1)) + wb.dot(tb + kc * (2 * W3 + 1))) +
                         (w0[o] - w1[o]);
        bstore(make_rsrc(y + plane * kc, on ? YB : 0u), yo, alpha * v + beta * sd[o]);
    }
}

template <int P, int KC>
constexpr int vel_all_lds_doubles() {
    // the largest component: NP planes of staged values and two band passes
    int m = 0;
    for (int C = 0; C < 3; ++C) {
        const int W1 = (C == 0) ? P : P - 1, W2 = (C == 1) ? P : P - 1, W3 = (C == 2) ? P : P - 1;
        const int SW = T1 + 2 * W1, SR = T2 + 2 * W2, NP = KC + 2 * W3;
        const int d = NP * (SR * SW + 2 * SR * T1);
        m = d > m ? d : m;
    }
    return m;
}

template <int P, int KC>
__global__ __launch_bounds__(NT) void k_vel_all(OpArgs a, Fields out, Fields src, double alpha,
                                                double beta) {
    extern __shared__ double lds_all[];
    int id = xcd_block(blockIdx.x, a.nblocks);
    int comp;
    if (a.comp_fast) {
        comp = id % 3;
        id /= 3;
    }
    const int t1 = id % a.ntile1;
    id /= a.ntile1;
    const int t2 = id % a.ntile2;
    id /= a.ntile2;
    const int ch = id % a.nchunk;
    id /= a.nchunk;
    if (!a.comp_fast) {
        comp = id % 3;
        id /= 3;
    }
    const int r = id;
    const int i0 = t1 * T1, j0 = t2 * T2, k0 = a.kbase + ch * a.kchunk;
    if (comp == 0) vel_component_all<P, 0, KC>(a, out, src, alpha, beta, r, i0, j0, k0, lds_all);
    else if (comp == 1) vel_component_all<P, 1, KC>(a, out, src, alpha, beta, r, i0, j0, k0, lds_all);
    else vel_component_all<P, 2, KC>(a, out, src, alpha, beta, r, i0, j0, k0, lds_all);
}

// ---- single pass (K and A) ---------------------------------------------------------------
// With B = D^T M_q the coupling of component c is D_c^T M_q z, z = nu D u + p
// (z = nu D u for A), which is the Kronecker product of M^ in the two other
// directions and of D^^T M^ (banded, half-width p) in direction c.  So no w is
// needed: per i3-plane the kernel stages u1, u2, u3 and p on the tile and a
// halo of p, forms g = D u and z in LDS, and runs all four outputs through the
// same scheme as k_vel -- a direction-1 band pass over the tile rows and halo
// rows, a direction-2 band pass at the thread's point, and direction-3 register
// windows:
//   y_1 = alpha ((nu [M^ M^ K + 2 M^ T^ M + 2 T^ M^ M] u_1) + (M^ M^ D^^T M^) z) + beta s_1
//   (y_2 likewise), y_3 with the own-direction factors in direction 3, and
//   y_p = M_q g (K only).
// u is read once and nothing intermediate is written.  The band rows of the
// tile's columns and rows sit in LDS (registers hold the direction-3 windows).
template <int P>
constexpr int fused_lds_doubles() {
    return 5 * (T2 + 2 * P) * (T1 + 2 * P) + 9 * (T2 + 2 * P) * T1 + 5 * (T1 + T2) * (2 * P + 1);
}

template <int P>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_fused(
    OpArgs a, Fields out, Fields src, double alpha, double beta) {
    constexpr int W = P;                   // staging halo and the widest band
    constexpr int B = 2 * P + 1;           // band row length (all rows padded to it)
    constexpr int SW = T1 + 2 * W, SR = T2 + 2 * W;
    constexpr int NS = (SR * SW + NT - 1) / NT;
    constexpr int RA = SR * SW;            // a staged array
    constexpr int RB = SR * T1;            // a direction-1 result
    __shared__ double lds[fused_lds_doubles<P>()];
    double* X1 = lds;
    double* X2 = X1 + RA;
    double* X3 = X2 + RA;
    double* ZS = X3 + RA;
    double* GS = ZS + RA;
    double* A1 = GS + RA;   // K u1, M u1 (direction 1)
    double* B1 = A1 + RB;
    double* Z1 = B1 + RB;   // D^^T M^ z
    double* A2 = Z1 + RB;   // M^ u2, T^ u2
    double* B2 = A2 + RB;
    double* A3 = B2 + RB;   // M^ u3, T^ u3
    double* B3 = A3 + RB;
    double* ZM = B3 + RB;   // M^ z (shared by components 2 and 3)
    double* GM = ZM + RB;   // M^ g
    double* R1 = GM + RB;   // band rows of the tile's columns: K, M, D^T M^, M^, T^ (x T1)
    double* R2 = R1 + 5 * T1 * B;  // band rows of the tile's rows (x T2)
    const int nM = a.nM, nN = a.nN;
    int id = xcd_block(blockIdx.x, a.nblocks);
    const int t1 = id % a.ntile1;
    id /= a.ntile1;
    const int t2 = id % a.ntile2;
    id /= a.ntile2;
    const int ch = id % a.nchunk;
    const int r = id / a.nchunk;
    const int i0 = t1 * T1, j0 = t2 * T2, k0 = a.kbase + ch * a.kchunk;
    const int kend = min(min(k0 + a.kchunk, a.klim), nM);
    const int c = threadIdx.x % T1, g = threadIdx.x / T1;
    const int i = i0 + c, j = j0 + g;
    const bool use_p = (a.mode == OP_K);
    const double nu = a.nu;
    const double* u1 = a.u[0] + (long long)r * a.su;
    const double* u2 = a.u[1] + (long long)r * a.su;
    const double* u3 = a.u[2] + (long long)r * a.su;
    const double* pp = use_p ? a.p + (long long)r * a.sp : u1;
    const long long P1 = (long long)nN * nM, P3 = (long long)nM * nM;
    const uint32_t B1b = 8u * (uint32_t)P1, B3b = 8u * (uint32_t)P3;
    const uint32_t BPb = use_p ? B3b : 0u;
    // band rows into LDS: R1[b][c][t] for the column index i0 + c, R2[b][g][t]
    // for the row index j0 + g; b = K, M (interior, n_N), D^T M^ (n_N), M^, T^ (n_M,
    // half-width p-1, stored shifted by one)
    for (int e = threadIdx.x; e < 5 * (T1 + T2) * B; e += NT) {
        const int t = e % B, q = e / B;
        const bool col = q < 5 * T1;
        const int qq = col ? q : q - 5 * T1;
        const int b = col ? qq / T1 : qq / T2;
        const int idx = (col ? i0 + qq % T1 : j0 + qq % T2);
        double v = 0.0;
        if (b <= 2) {
            const int tab = b == 0 ? BK_N : (b == 1 ? BM_N : BD_M);
            if (idx < nN) v = a.bt.ptr[tab][(long long)idx * B + t];
        } else {
            const int tab = b == 3 ? BM_C : BT_C;
            if (idx < nM && t >= 1 && t <= 2 * P - 1) v = a.bt.ptr[tab][(long long)idx * (B - 2) + t - 1];
        }
        if (col) R1[q * B + t] = v;
        else R2[qq * B + t] = v;
    }
    // staging offsets (as k_pres): u1[ii], u1[ii-1], u2[jj], u2[jj-1], u3 / p at (ii, jj)
    uint32_t oa[NS], ob[NS], oc[NS], od[NS], oe[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int idx = threadIdx.x + s * NT;
        const int rr = idx / SW, cc = idx - rr * SW;
        const int jj = j0 - W + rr, ii = i0 - W + cc;
        const bool ok = idx < RA && jj >= 0 && jj < nM && ii >= 0 && ii < nM;
        oa[s] = (ok && ii < nN) ? 8u * (nN * jj + ii) : OOB;
        ob[s] = (ok && ii >= 1) ? 8u * (nN * jj + ii - 1) : OOB;
        oc[s] = (ok && jj < nN) ? 8u * (ii + nM * jj) : OOB;
        od[s] = (ok && jj >= 1) ? 8u * (ii + nM * (jj - 1)) : OOB;
        oe[s] = ok ? 8u * (ii + nM * jj) : OOB;
    }
    auto fetch = [&](int kk, double (&v)[NS][6]) {
        const bool kin = kk >= 0 && kk < nM;
        const bool k3in = kk >= 0 && kk < nN;
        const int kc = kin ? kk : 0, k3 = k3in ? kk : 0;
        const auto r1 = make_rsrc(u1 + P1 * kc, kin ? B1b : 0u);
        const auto r2 = make_rsrc(u2 + P1 * kc, kin ? B1b : 0u);
        const auto r3 = make_rsrc(u3 + P3 * k3, k3in ? B3b : 0u);
        const auto rp = make_rsrc(pp + P3 * kc, kin ? BPb : 0u);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            v[s][0] = bload(r1, oa[s]);
            v[s][1] = bload(r1, ob[s]);
            v[s][2] = bload(r2, oc[s]);
            v[s][3] = bload(r2, od[s]);
            v[s][4] = bload(r3, oe[s]);
            v[s][5] = bload(rp, oe[s]);
        }
    };
    // outputs: component planes and this thread's offsets (OOB where no output)
    const uint32_t o1 = (i < nN && j < nM) ? 8u * (i + nN * j) : OOB;
    const uint32_t o2 = (i < nM && j < nN) ? 8u * (i + nM * j) : OOB;
    const uint32_t o3 = (i < nM && j < nM) ? 8u * (i + nM * j) : OOB;
    double* y1 = out.f[0] + (long long)r * out.stride[0];
    double* y2 = out.f[1] + (long long)r * out.stride[1];
    double* y3 = out.f[2] + (long long)r * out.stride[2];
    double* yp = use_p ? out.f[3] + (long long)r * out.stride[3] : y3;
    const bool has_src = beta != 0.0;
    const double* s1 = has_src ? src.f[0] + (long long)r * src.stride[0] : y1;
    const double* s2 = has_src ? src.f[1] + (long long)r * src.stride[1] : y2;
    const double* s3 = has_src ? src.f[2] + (long long)r * src.stride[2] : y3;
    const uint32_t SB1 = has_src ? B1b : 0u, SB3 = has_src ? B3b : 0u;
    const uint32_t YPB = use_p ? B3b : 0u;
    Window<P - 1> wa1, wb1, wa2, wb2, wp;
    Window<P> wa3, wb3, wz3;
    wa1.clear(); wb1.clear(); wa2.clear(); wb2.clear(); wp.clear();
    wa3.clear(); wb3.clear(); wz3.clear();
    double buf[NS][6], a3prev[NS];
    {
        double t[NS][6];
        fetch(k0 - W - 1, t);
#pragma unroll
        for (int s = 0; s < NS; ++s) a3prev[s] = t[s][4];
    }
    fetch(k0 - W, buf);
    for (int kk = k0 - W; kk < kend + W; ++kk) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int idx = threadIdx.x + s * NT;
            if (idx < RA) {
                const double gv = (buf[s][0] - buf[s][1]) + (buf[s][2] - buf[s][3]) + (buf[s][4] - a3prev[s]);
                X1[idx] = buf[s][0];
                X2[idx] = buf[s][2];
                X3[idx] = buf[s][4];
                GS[idx] = gv;
                ZS[idx] = nu * gv + buf[s][5];
            }
            a3prev[s] = buf[s][4];
        }
        fetch(kk + 1, buf);
        __syncthreads();
        // direction 1 over the tile rows and halo rows
        {
            const double* rk = R1 + (0 * T1 + c) * B;
            const double* rm = R1 + (1 * T1 + c) * B;
            const double* rd = R1 + (2 * T1 + c) * B;
            const double* rc = R1 + (3 * T1 + c) * B;
            const double* rt = R1 + (4 * T1 + c) * B;
            for (int rr = g; rr < SR; rr += T2) {
                double sk = 0.0, sm = 0.0, sd = 0.0, sz = 0.0, s2m = 0.0, s2t = 0.0, s3m = 0.0,
                       s3t = 0.0, sg = 0.0;
#pragma unroll
                for (int t = 0; t < B; ++t) {
                    const int o = rr * SW + c + t;
                    const double x1 = X1[o], x2 = X2[o], x3 = X3[o], zv = ZS[o], gv = GS[o];
                    const double ck = rk[t], cm = rm[t], cd = rd[t], cc = rc[t], ct = rt[t];
                    sk += ck * x1;
                    sm += cm * x1;
                    sd += cd * zv;
                    sz += cc * zv;
                    s2m += cc * x2;
                    s2t += ct * x2;
                    s3m += cc * x3;
                    s3t += ct * x3;
                    sg += cc * gv;
                }
                const int o = rr * T1 + c;
                A1[o] = sk;
                B1[o] = sm;
                Z1[o] = sd;
                ZM[o] = sz;
                A2[o] = s2m;
                B2[o] = s2t;
                A3[o] = s3m;
                B3[o] = s3t;
                GM[o] = sg;
            }
        }
        __syncthreads();
        // direction 2 at this thread's point; push into the direction-3 windows
        {
            const double* qk = R2 + (0 * T2 + g) * B;
            const double* qm = R2 + (1 * T2 + g) * B;
            const double* qd = R2 + (2 * T2 + g) * B;
            const double* qc = R2 + (3 * T2 + g) * B;
            const double* qt = R2 + (4 * T2 + g) * B;
            double am1 = 0, ak1 = 0, bm1 = 0, bk1 = 0, zz1 = 0;
            double am2 = 0, ak2 = 0, bm2 = 0, zz2 = 0;
            double am3 = 0, ak3 = 0, bm3 = 0, zz3 = 0, gp = 0;
#pragma unroll
            for (int t = 0; t < B; ++t) {
                const int o = (g + t) * T1 + c;
                const double cc = qc[t], ct = qt[t], ck = qk[t], cm = qm[t], cd = qd[t];
                const double va1 = A1[o], vb1 = B1[o], vz1 = Z1[o];
                const double va2 = A2[o], vb2 = B2[o], vzm = ZM[o];
                const double va3 = A3[o], vb3 = B3[o], vg = GM[o];
                am1 += cc * va1; ak1 += ct * va1; bm1 += cc * vb1; bk1 += ct * vb1; zz1 += cc * vz1;
                am2 += cm * va2; ak2 += ck * va2; bm2 += cm * vb2; zz2 += cd * vzm;
                am3 += cc * va3; ak3 += ct * va3; bm3 += cc * vb3; zz3 += cc * vzm;
                gp += cc * vg;
            }
            wa1.push(nu * (am1 + 2.0 * bk1) + zz1);
            wb1.push(2.0 * bm1);
            wa2.push(nu * (ak2 + 2.0 * bm2) + zz2);
            wb2.push(2.0 * am2);
            wa3.push(am3);
            wb3.push(2.0 * (ak3 + bm3));
            wz3.push(zz3);
            wp.push(gp);
        }
        // outputs: components 1, 2 and the pressure p-1 planes behind, component 3 p behind
        {
            const int k = kk - (P - 1);
            if (k >= k0 && k < kend) {
                const double* rmc = a.bt.ptr[BM_C] + k * (2 * P - 1);
                const double* rtc = a.bt.ptr[BT_C] + k * (2 * P - 1);
                const double v1 = wa1.dot(rmc) + nu * wb1.dot(rtc);
                const double v2 = wa2.dot(rmc) + nu * wb2.dot(rtc);
                const double e1 = bload(make_rsrc(s1 + P1 * k, SB1), o1);
                const double e2 = bload(make_rsrc(s2 + P1 * k, SB1), o2);
                bstore(make_rsrc(y1 + P1 * k, B1b), o1, alpha * v1 + beta * e1);
                bstore(make_rsrc(y2 + P1 * k, B1b), o2, alpha * v2 + beta * e2);
                bstore(make_rsrc(yp + P3 * k, YPB), o3, wp.dot(rmc));
            }
            const int k3 = kk - P;
            if (k3 >= k0 && k3 < kend && k3 < nN) {
                const double v3 = nu * (wa3.dot(a.bt.ptr[BK_N] + k3 * B) + wb3.dot(a.bt.ptr[BM_N] + k3 * B)) +
                                  wz3.dot(a.bt.ptr[BD_M] + k3 * B);
                const double e3 = bload(make_rsrc(s3 + P3 * k3, SB3), o3);
                bstore(make_rsrc(y3 + P3 * k3, B3b), o3, alpha * v3 + beta * e3);
            }
        }
    }
}

template <int P>
void launch_pres(dim3 grid, hipStream_t st, const OpArgs& a, double* yp, long long syp) {
    hipLaunchKernelGGL((k_pres<P, T1, T2>), grid, dim3(NT), 0, st, a, yp, syp);
}
// the pressure chain on 32 x 8 tiles: less halo per point (36 x 12 staged
// values per 256 outputs against 20 x 12 per 128), larger workgroups
constexpr int PW1 = 32, PW2 = 8;
template <int P>
void launch_pres_wide(dim3 grid, hipStream_t st, const OpArgs& a, double* yp, long long syp) {
    hipLaunchKernelGGL((k_pres<P, PW1, PW2>), grid, dim3(PW1 * PW2), 0, st, a, yp, syp);
}

template <int P>
void launch_vel(dim3 grid, hipStream_t st, const OpArgs& a, const Fields& out, const Fields& s,
                double alpha, double beta) {
    hipLaunchKernelGGL(k_vel<P>, grid, dim3(NT), 0, st, a, out, s, alpha, beta);
}

template <int P>
void launch_vel_dma(dim3 grid, hipStream_t st, const OpArgs& a, const Fields& out, const Fields& s,
                    double alpha, double beta) {
    hipLaunchKernelGGL(k_vel_dma<P>, grid, dim3(NT), 0, st, a, out, s, alpha, beta);
}

template <int P>
void launch_fused(dim3 grid, hipStream_t st, const OpArgs& a, const Fields& out, const Fields& s,
                  double alpha, double beta) {
    hipLaunchKernelGGL(k_fused<P>, grid, dim3(NT), 0, st, a, out, s, alpha, beta);
}
using FusedLaunch = void (*)(dim3, hipStream_t, const OpArgs&, const Fields&, const Fields&, double,
                             double);
// the single-pass kernel for degrees 2..4 (its windows and staging fill the
// register file beyond)
constexpr int FUSED_PMAX = 4;
const FusedLaunch fused_launch[FUSED_PMAX + 1] = {nullptr, nullptr, launch_fused<2>,
                                                  launch_fused<3>, launch_fused<4>};

// instantiations per degree 2..8 (index = degree)
using PresLaunch = void (*)(dim3, hipStream_t, const OpArgs&, double*, long long);
using VelLaunch = void (*)(dim3, hipStream_t, const OpArgs&, const Fields&, const Fields&, double,
                           double);
constexpr int PMAX = 8;
const PresLaunch pres_launch[PMAX + 1] = {nullptr,        nullptr,        launch_pres<2>,
                                          launch_pres<3>, launch_pres<4>, launch_pres<5>,
                                          launch_pres<6>, launch_pres<7>, launch_pres<8>};
const PresLaunch pres_wide_launch[PMAX + 1] = {
    nullptr,             nullptr,             launch_pres_wide<2>, launch_pres_wide<3>,
    launch_pres_wide<4>, launch_pres_wide<5>, launch_pres_wide<6>, launch_pres_wide<7>,
    launch_pres_wide<8>};
const VelLaunch vel_launch[PMAX + 1] = {nullptr,       nullptr,       launch_vel<2>,
                                        launch_vel<3>, launch_vel<4>, launch_vel<5>,
                                        launch_vel<6>, launch_vel<7>, launch_vel<8>};
const VelLaunch vel_dma_launch[PMAX + 1] = {nullptr,           nullptr,           launch_vel_dma<2>,
                                            launch_vel_dma<3>, launch_vel_dma<4>, launch_vel_dma<5>,
                                            launch_vel_dma<6>, launch_vel_dma<7>, launch_vel_dma<8>};

template <int P, int KC>
void launch_vel_all(dim3 grid, hipStream_t st, const OpArgs& a, const Fields& out, const Fields& s,
                    double alpha, double beta) {
    constexpr size_t shm = sizeof(double) * vel_all_lds_doubles<P, KC>();
    hipLaunchKernelGGL((k_vel_all<P, KC>), grid, dim3(NT), shm, st, a, out, s, alpha, beta);
}
template <int P, int KC>
hipError_t vel_all_attr() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vel_all<P, KC>),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(sizeof(double) * vel_all_lds_doubles<P, KC>()));
}
template <int P, int KC>
void launch_pres_all(dim3 grid, hipStream_t st, const OpArgs& a, double* yp, long long syp) {
    constexpr size_t shm = sizeof(double) * pres_all_lds_doubles<P, KC>();
    hipLaunchKernelGGL((k_pres_all<P, KC>), grid, dim3(NT), shm, st, a, yp, syp);
}
template <int P, int KC>
hipError_t pres_all_attr() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pres_all<P, KC>),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(sizeof(double) * pres_all_lds_doubles<P, KC>()));
}
// the all-planes pressure kernels: degrees 2, 3 x chunks 2, 4 (null: stream)
PresLaunch pres_all_launch(int P, int kc) {
    if (P == 2 && kc == 2) return launch_pres_all<2, 2>;
    if (P == 2 && kc == 4) return launch_pres_all<2, 4>;
    if (P == 3 && kc == 2) return launch_pres_all<3, 2>;
    if (P == 3 && kc == 4) return launch_pres_all<3, 4>;
    return nullptr;
}
// the all-planes velocity kernels: degrees 2..4 x chunks 2, 4, 8 (8: degree <= 3)
VelLaunch vel_all_launch(int P, int kc) {
    if (P == 2 && kc == 2) return launch_vel_all<2, 2>;
    if (P == 2 && kc == 4) return launch_vel_all<2, 4>;
    if (P == 2 && kc == 8) return launch_vel_all<2, 8>;
    if (P == 3 && kc == 2) return launch_vel_all<3, 2>;
    if (P == 3 && kc == 4) return launch_vel_all<3, 4>;
    if (P == 3 && kc == 8) return launch_vel_all<3, 8>;
    if (P == 4 && kc == 2) return launch_vel_all<4, 2>;
    if (P == 4 && kc == 4) return launch_vel_all<4, 4>;
    return nullptr;
}

}  // namespace

bool op_staged_ok(int degree, int kchunk) { return vel_all_launch(degree, kchunk) != nullptr; }

hipError_t ops_init_attributes() {
    const hipError_t es[] = {vel_all_attr<2, 2>(), vel_all_attr<2, 4>(), vel_all_attr<2, 8>(),
                             vel_all_attr<3, 2>(), vel_all_attr<3, 4>(), vel_all_attr<3, 8>(),
                             vel_all_attr<4, 2>(), vel_all_attr<4, 4>(),
                             pres_all_attr<2, 2>(), pres_all_attr<2, 4>(),
                             pres_all_attr<3, 2>(), pres_all_attr<3, 4>()};
    for (hipError_t e : es)
        if (e != hipSuccess) return e;
    return hipSuccess;
}

long long ops_ws_stride(const hp_ctx* c) { return c->nQ; }

OpShape op_model_shape(const hp_ctx* c, int nrhs) {
    // planes per workgroup: a workgroup takes kchunk + 2p steps, and the
    // velocity launch runs in ceil(blocks / resident) rounds (waves per SIMD
    // as the kernels' register budget allows, four SIMDs per CU); minimise
    // rounds x steps
    const int nM = c->nM, P = c->p;
    const long long per_chunk =
        (long long)((nM + T1 - 1) / T1) * ((nM + T2 - 1) / T2) * 3 * nrhs;
    const int waves = P < 4 ? 4 : (P == 4 ? 3 : 2);
    const long long resident = 256LL * (4 * waves / (NT / 64));
    long long best = -1, best_kc = 1;
    for (int kc = 2; kc <= 64; ++kc) {
        const long long nch = (nM + kc - 1) / kc;
        const long long cost = ((per_chunk * nch + resident - 1) / resident) * (kc + 2 * P);
        if (best < 0 || cost < best) {
            best = cost;
            best_kc = kc;
        }
        if (nch == 1) break;
    }
    return OpShape{(int)best_kc, 1, 1};
}

OpShape op_shape(const hp_ctx* c, int nrhs) {
    OpShape sh = op_model_shape(c, nrhs);
    for (int e = 0; e < 2; ++e)
        if (c->op_tuned[e].kchunk > 0 && c->op_tuned[e].nrhs == nrhs) sh = c->op_tuned[e].shape;
    if (c->opts.op_kchunk > 0) sh.kchunk = c->opts.op_kchunk;
    if (c->opts.op_slabs > 0) sh.slabs = c->opts.op_slabs;
    if (c->opts.op_order >= 0) sh.comp_fast = c->opts.op_order;
    if (c->opts.op_fused >= 0) sh.fused = c->opts.op_fused;
    if (c->opts.op_staged >= 0) sh.staged = c->opts.op_staged;
    if (c->opts.op_pres_wide >= 0) sh.pwide = c->opts.op_pres_wide;
    sh.dma = c->opts.op_dma != 0;
    if (c->op_force.kchunk > 0) sh = c->op_force;
    if (c->p > FUSED_PMAX) sh.fused = 0;
    return sh;
}

hipError_t launch_operator(hp_ctx* c, OpMode mode, const Fields& in, const Fields& out,
                           double alpha, double beta, const Fields* src, int nrhs) {
    if (c->p < 2 || c->p > PMAX || nrhs < 1) return hipErrorInvalidValue;
    OpArgs a{};
    a.bt = c->band;
    for (int i = 0; i < 3; ++i) a.u[i] = in.f[i];
    a.p = in.f[3];
    a.su = in.stride[0];
    a.sp = in.stride[3];
    a.ws = c->ws;
    a.ws_stride = ops_ws_stride(c);
    for (int b = 0; b < 4; ++b)
        for (int d = 0; d < 3; ++d) a.dims[b][d] = (int)c->dims[b][d];
    a.nN = c->nN;
    a.nM = c->nM;
    a.nu = c->nu;
    a.mode = mode;
    const int nM = c->nM;
    const int P = c->p;
    a.ntile1 = (nM + T1 - 1) / T1;
    a.ntile2 = (nM + T2 - 1) / T2;
    const OpShape sh = op_shape(c, nrhs);
    a.kchunk = std::max(1, std::min(sh.kchunk, nM));
    a.comp_fast = sh.comp_fast;
    Fields s = src ? *src : out;
    if (!src) beta = 0.0;
    double* yp = out.f[3];
    const long long syp = out.stride[3];
    const PresLaunch pall = sh.staged ? pres_all_launch(P, a.kchunk) : nullptr;
    const bool pwide = !pall && sh.pwide;
    auto pres = [&](int lo, int hi) {
        a.kbase = lo;
        a.klim = hi;
        a.nchunk = (hi - lo + a.kchunk - 1) / a.kchunk;
        if (pwide) {
            a.ntile1 = (nM + PW1 - 1) / PW1;
            a.ntile2 = (nM + PW2 - 1) / PW2;
        }
        a.nblocks = a.ntile1 * a.ntile2 * a.nchunk * nrhs;
        dim3 grid(a.nblocks);
        (pall ? pall : (pwide ? pres_wide_launch[P] : pres_launch[P]))(grid, c->stream, a, yp,
                                                                       syp);
        a.ntile1 = (nM + T1 - 1) / T1;  // the velocity kernels' tiles
        a.ntile2 = (nM + T2 - 1) / T2;
    };
    const VelLaunch vall = (sh.staged && (mode == OP_K || mode == OP_A))
                               ? vel_all_launch(P, a.kchunk) : nullptr;
    auto vel = [&](int lo, int hi) {
        a.kbase = lo;
        a.klim = hi;
        a.nchunk = (hi - lo + a.kchunk - 1) / a.kchunk;
        a.nblocks = a.ntile1 * a.ntile2 * a.nchunk * 3 * nrhs;
        dim3 grid(a.nblocks);
        (vall ? vall : (sh.dma ? vel_dma_launch[P] : vel_launch[P]))(grid, c->stream, a, out, s,
                                                                     alpha, beta);
    };
    if (sh.fused && (mode == OP_K || mode == OP_A)) {
        a.kbase = 0;
        a.klim = nM;
        a.nchunk = (nM + a.kchunk - 1) / a.kchunk;
        a.nblocks = a.ntile1 * a.ntile2 * a.nchunk * nrhs;
        fused_launch[P](dim3(a.nblocks), c->stream, a, out, s, alpha, beta);
        return hipGetLastError();
    }
    if (mode == OP_BT) {
        pres(0, nM);
    } else if (mode == OP_MV) {
        vel(0, nM);
    } else if (mode == OP_DT) {
        // the coupling-only velocity kernel reading the pressure input as w
        a.mode = OP_B;
        a.ws = in.f[3];
        a.ws_stride = in.stride[3];
        vel(0, nM);
    } else {
        // slabs of i3-planes, each pressure chain then velocity, so that the
        // second read of u and the round trip of w can stay in the Infinity
        // Cache; the pressure launch of a slab also produces w on the first
        // plane of the next slab, which D_3^T needs
        const int S = std::max(1, std::min(sh.slabs, nM));
        for (int sl = 0; sl < S; ++sl) {
            const int lo = (int)((long long)nM * sl / S), hi = (int)((long long)nM * (sl + 1) / S);
            if (hi <= lo) continue;
            pres(lo, std::min(hi + 1, nM));
            vel(lo, hi);
        }
    }
    return hipGetLastError();
}

}  // namespace hp
