// Quadrature-based (matrix-free) forward operator: the forward problem
// evaluated by global sum factorisation with p+1 Gauss-Legendre points per
// element in each direction (Sec. 5.3), on the weak form of Sec. 3.1 with
// the symmetric Nitsche terms of Sec. 3.3 on the faces.
//
// With G = grad u and P the pressure at a point of the tensor grid, the
// volume flux for the test function v_c is
//     coefficient of d_d v_c :  w nu (G_cd + G_dc) + w P delta_cd,
// and for the pressure test function q it is w (G_11 + G_22 + G_33):
// 2 nu eps(u):eps(v) = nu (grad u + grad u^T):grad v, b(v,p) = (p, div v).
// On a face with outward normal s e_d (s = -1 at x_d = 0, +1 at x_d = 1)
// the tangential components c != d carry
//     nu (2 alpha u_c v_c - v_c d_n u_c - u_c d_n v_c),  alpha = C_pen / h;
// the normal component vanishes there (strongly imposed v.n = 0), and so
// does d_c u_d on that face, which is why only d_n u_c enters.
//
// The points of one direction are [x = 0, the E (p+1) Gauss points, x = 1];
// the weight of an end point is 1, so that a point with one end-point
// coordinate carries the weight of the two-dimensional Gauss rule of its
// face.  Points with two or more end-point coordinates (edges) carry nothing.
//
// One application per right-hand side is six launches:
//   mode 1 then mode 2 evaluation (banded basis tables, k_qpass),
//   mode 3 evaluation fused with the pointwise flux (k_qflux),
//   and the transposed contractions mode 3 (k_qpass3t, four output rows
//   per thread), mode 2 and mode 1 (k_qpass).
// Every launch is HBM bound; the 10 flux fields at the (E(p+1)+2)^3 points
// dominate the traffic (written once, read once).
#include <algorithm>
#include <stdexcept>

#include "hp_internal.h"

namespace hp {

namespace {

constexpr int QT = 256;
constexpr int QMAXJOB = 10;

// One contraction: out = ma . a (+ mb . b) along the launch's mode; a and b
// have dims (d0, d1, d2), out has the mode's extent replaced by ma.rows.
struct QJob {
    const double* a;
    const double* b;
    double* out;
    QBand ma, mb;
    int d0, d1, d2;
    long long nout;
};
struct QJobs {
    QJob j[QMAXJOB];
};

__device__ inline double band_dot(const QBand& m, int r, const double* __restrict__ x,
                                  long long base, long long st) {
    const int s0 = m.start[r];
    const double* v = m.val + (long long)r * m.w;
    double s = 0.0;
    for (int t = 0; t < m.w; ++t) s += v[t] * x[base + (long long)(s0 + t) * st];
    return s;
}

// Modes 1 and 2 (MODE = 0, 1); mode 3 has its own kernels below.
template <int MODE>
__global__ __launch_bounds__(QT) void k_qpass(QJobs J) {
    static_assert(MODE == 0 || MODE == 1, "k_qpass contracts direction 1 or 2");
    const QJob& jb = J.j[blockIdx.y];
    // the grid is a multiple of 8 workgroups; XCD x (workgroups x, x+8, ...)
    // walks the x-th eighth of the output in order, so the input rows that
    // neighbouring outputs share are reused from that XCD's L2
    const long long L = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    const long long o = L * QT + threadIdx.x;
    if (o >= jb.nout) return;
    const long long d0 = jb.d0, d1 = jb.d1;
    const int R = jb.ma.rows;
    int r;
    long long base, st;
    if (MODE == 0) {
        r = (int)(o % R);
        base = (o / R) * d0;
        st = 1;
    } else {
        const long long i0 = o % d0, t = o / d0;
        r = (int)(t % R);
        base = i0 + (t / R) * d0 * d1;
        st = d0;
    }
    double s = band_dot(jb.ma, r, jb.a, base, st);
    if (jb.b) s += band_dot(jb.mb, r, jb.b, base, st);
    jb.out[o] = s;
}

// Transposed mode-3 contraction with QJB consecutive output rows per thread:
// rows r0 .. r0+QJB-1 of the band read overlapping windows of one line, so
// the union of the windows is loaded once.  Each row still sums its terms in
// window order (a and b separately, then added), as band_dot does.
constexpr int QJB = 4;

// Workgroup order of the mode-3 kernels: the tiles of one (i1, i2) plane are
// padded to a multiple of 8, so that a tile lands on the same XCD (workgroups
// are dealt round-robin to the 8 XCDs) at every i3 level and the planes that
// neighbouring levels share stay in that XCD's L2.
__host__ __device__ inline long long xcd_tiles(long long pl) { return (((pl + QT - 1) / QT) + 7) & ~7LL; }

__global__ __launch_bounds__(QT) void k_qpass3t(QJobs J) {
    const QJob& jb = J.j[blockIdx.y];
    const long long pl = (long long)jb.d0 * jb.d1;
    const int R = jb.ma.rows;
    const int nrb = (R + QJB - 1) / QJB;
    const long long ntp = xcd_tiles(pl);
    const long long base = (blockIdx.x % ntp) * QT + threadIdx.x;
    const int rb = (int)(blockIdx.x / ntp);
    if (base >= pl || rb >= nrb) return;
    const int r0 = rb * QJB;
    const int nr = min(QJB, R - r0);
    double acc[QJB], accb[QJB];
#pragma unroll
    for (int k = 0; k < QJB; ++k) acc[k] = accb[k] = 0.0;
    auto run = [&](const QBand& m, const double* __restrict__ x, double* out) {
        int st[QJB];
#pragma unroll
        for (int k = 0; k < QJB; ++k) st[k] = m.start[r0 + (k < nr ? k : nr - 1)];
        int lo = st[0], hi = st[0];
#pragma unroll
        for (int k = 0; k < QJB; ++k) {
            lo = min(lo, st[k]);
            hi = max(hi, st[k] + m.w);
        }
        for (int q = lo; q < hi; ++q) {
            const double xv = x[base + (long long)q * pl];
#pragma unroll
            for (int k = 0; k < QJB; ++k) {
                const int t = q - st[k];
                if (k < nr && t >= 0 && t < m.w)
                    out[k] += m.val[(long long)(r0 + k) * m.w + t] * xv;
            }
        }
    };
    run(jb.ma, jb.a, acc);
    if (jb.b) run(jb.mb, jb.b, accb);
#pragma unroll
    for (int k = 0; k < QJB; ++k)
        if (k < nr) jb.out[base + (long long)(r0 + k) * pl] = jb.b ? acc[k] + accb[k] : acc[k];
}

// Flux fields at the points (10): F_v of components 1..3 (0..2), the
// diagonal S_11, S_22, S_33 (3..5), S_12, S_13, S_23 (6..8) and F_q (9).
// S_cd serves as the coefficient of d_d v_c and of d_c v_d: equal at volume
// points; on a face normal to c only d_c v_d is nonzero (u_c is normal
// there), and S_cd is then read for component c only through its own
// direction-c value table, whose end-point rows vanish (interior functions),
// so one field carries both.
constexpr int QNF = 10;
__host__ __device__ constexpr int qsym(int c, int d) {
    return c == d ? 3 + c : (c + d == 1 ? 6 : (c + d == 2 ? 7 : 8));
}

struct QFluxArgs {
    const double* in[10];  // component c: (V1 V2), (V1 D2), (D1 V2) at 3c..3c+2; pressure 9
    double* out[QNF];
    QBand V[2], D[2];      // direction-3 tables: [0] degree p-1, [1] interior degree p
    const double* wq;
    int nq;
    double nu, alpha;
};

__global__ __launch_bounds__(QT) void k_qflux(QFluxArgs A) {
    const long long nq = A.nq, pl = nq * nq;
    const long long ntp = xcd_tiles(pl);
    const long long base = (blockIdx.x % ntp) * QT + threadIdx.x;
    const int i2 = (int)(blockIdx.x / ntp);
    if (base >= pl || i2 >= A.nq) return;
    const long long o = base + (long long)i2 * pl;
    const int i0 = (int)(base % nq), i1 = (int)(base / nq);
    double U[3], G[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int T = c == 2 ? 1 : 0;
        U[c] = band_dot(A.V[T], i2, A.in[3 * c], base, pl);
        G[c][2] = band_dot(A.D[T], i2, A.in[3 * c], base, pl);
        G[c][1] = band_dot(A.V[T], i2, A.in[3 * c + 1], base, pl);
        G[c][0] = band_dot(A.V[T], i2, A.in[3 * c + 2], base, pl);
    }
    const double P = band_dot(A.V[0], i2, A.in[9], base, pl);
    const int last = A.nq - 1;
    const bool e0 = i0 == 0 || i0 == last, e1 = i1 == 0 || i1 == last,
               e2 = i2 == 0 || i2 == last;
    const int ne = (int)e0 + (int)e1 + (int)e2;
    const double w = A.wq[i0] * A.wq[i1] * A.wq[i2];
    double F[QNF];
#pragma unroll
    for (int k = 0; k < QNF; ++k) F[k] = 0.0;
    if (ne == 0) {
        const double wn = w * A.nu;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            F[3 + c] = wn * (G[c][c] + G[c][c]) + w * P;
#pragma unroll
            for (int d = c + 1; d < 3; ++d) F[qsym(c, d)] = wn * (G[c][d] + G[d][c]);
        }
        F[9] = w * (G[0][0] + G[1][1] + G[2][2]);
    } else if (ne == 1) {
        // face normal to direction d (register arrays are only indexed by
        // unrolled constants)
        const double wn = w * A.nu;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const bool on = d == 0 ? e0 : (d == 1 ? e1 : e2);
            if (!on) continue;
            const int idx = d == 0 ? i0 : (d == 1 ? i1 : i2);
            const double s = idx == 0 ? -1.0 : 1.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (c == d) continue;
                F[c] = wn * (2.0 * A.alpha * U[c] - s * G[c][d]);
                F[qsym(c, d)] = -wn * s * U[c];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < QNF; ++k) A.out[k][o] = F[k];
}

// Band form of a dense row-major rows x cols matrix: one common width w,
// row r holds A[r][start[r] .. start[r] + w) (every non-zero of the row lies
// in that window; start is pulled left so that the window stays in range).
struct HostBand {
    int rows = 0, cols = 0, w = 1;
    std::vector<int> start;
    std::vector<double> val;
};
HostBand make_band(const std::vector<double>& A, int rows, int cols) {
    HostBand B;
    B.rows = rows;
    B.cols = cols;
    std::vector<int> first(rows, 0), lastnz(rows, -1);
    int w = 1;
    for (int r = 0; r < rows; ++r) {
        int f = -1, l = -1;
        for (int c = 0; c < cols; ++c)
            if (A[(size_t)r * cols + c] != 0.0) {
                if (f < 0) f = c;
                l = c;
            }
        if (f >= 0) {
            first[r] = f;
            lastnz[r] = l;
            w = std::max(w, l - f + 1);
        }
    }
    w = std::min(w, cols);
    B.w = w;
    B.start.resize(rows);
    B.val.assign((size_t)rows * w, 0.0);
    for (int r = 0; r < rows; ++r) {
        const int s = std::max(0, std::min(first[r], cols - w));
        B.start[r] = s;
        for (int t = 0; t < w; ++t) B.val[(size_t)r * w + t] = A[(size_t)r * cols + s + t];
        if (lastnz[r] >= s + w) throw std::runtime_error("band window too narrow");
    }
    return B;
}
std::vector<double> transpose(const std::vector<double>& A, int rows, int cols) {
    std::vector<double> T((size_t)rows * cols);
    for (int r = 0; r < rows; ++r)
        for (int c = 0; c < cols; ++c) T[(size_t)c * rows + r] = A[(size_t)r * cols + c];
    return T;
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + QT - 1) / QT); }

template <int MODE>
hipError_t run_pass(hipStream_t s, const QJobs& J, int njob) {
    long long m = 0;
    for (int i = 0; i < njob; ++i) m = std::max(m, J.j[i].nout);
    if (m == 0) return hipSuccess;
    const unsigned nb = (blocks_for(m) + 7) & ~7u;  // a multiple of 8 (see k_qpass)
    hipLaunchKernelGGL(k_qpass<MODE>, dim3(nb, njob), dim3(QT), 0, s, J);
    return hipGetLastError();
}

}  // namespace

hipError_t quad_setup(hp_ctx* c, QuadOp* q) {
    if (q->ready) return hipSuccess;
    const QuadTables1D Q = build_quad_tables(c->tab);
    const int nq = Q.nq, nN = c->nN, nM = c->nM;
    // [0] degree p-1 (M), [1] interior degree p (N); forward and transposed
    HostBand hb[8];
    try {
        hb[0] = make_band(Q.MV, nq, nM);
        hb[1] = make_band(Q.NV, nq, nN);
        hb[2] = make_band(Q.MD, nq, nM);
        hb[3] = make_band(Q.ND, nq, nN);
        hb[4] = make_band(transpose(Q.MV, nq, nM), nM, nq);
        hb[5] = make_band(transpose(Q.NV, nq, nN), nN, nq);
        hb[6] = make_band(transpose(Q.MD, nq, nM), nM, nq);
        hb[7] = make_band(transpose(Q.ND, nq, nN), nN, nq);
    } catch (const std::exception&) {
        return hipErrorInvalidValue;
    }
    size_t nd = (size_t)nq, ni = 0;
    for (const HostBand& b : hb) {
        nd += b.val.size();
        ni += b.start.size();
    }
    q->nq = nq;
    const long long s1 = (long long)nq * nM * nM, s2 = (long long)nq * nq * nM,
                    s3 = (long long)nq * nq * nq;
    q->scratch_doubles = (size_t)(7 * s1 + 10 * s2 + QNF * s3);
    // every early error return releases what was allocated so far, so that a
    // later call starts again from an empty QuadOp
    auto fail = [q](hipError_t err) {
        quad_free(q);
        return err;
    };
    hipError_t e;
    if ((e = hipMalloc(&q->tables, sizeof(double) * nd)) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&q->index, sizeof(int) * ni)) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&q->scratch, sizeof(double) * q->scratch_doubles)) != hipSuccess)
        return fail(e);
    std::vector<double> hv;
    std::vector<int> hi;
    hv.reserve(nd);
    hi.reserve(ni);
    QBand* dst[8] = {&q->V[0], &q->V[1], &q->D[0], &q->D[1], &q->VT[0], &q->VT[1], &q->DT[0],
                     &q->DT[1]};
    std::vector<size_t> vo(8), io(8);
    for (int k = 0; k < 8; ++k) {
        vo[k] = hv.size();
        io[k] = hi.size();
        hv.insert(hv.end(), hb[k].val.begin(), hb[k].val.end());
        hi.insert(hi.end(), hb[k].start.begin(), hb[k].start.end());
    }
    const size_t wo = hv.size();
    hv.insert(hv.end(), Q.w.begin(), Q.w.end());
    for (int k = 0; k < 8; ++k) {
        *dst[k] = QBand{q->index + io[k], q->tables + vo[k], hb[k].rows, hb[k].cols, hb[k].w};
    }
    q->wq = q->tables + wo;
    if ((e = hipMemcpy(q->tables, hv.data(), sizeof(double) * hv.size(), hipMemcpyHostToDevice)) !=
        hipSuccess)
        return fail(e);
    if ((e = hipMemcpy(q->index, hi.data(), sizeof(int) * hi.size(), hipMemcpyHostToDevice)) !=
        hipSuccess)
        return fail(e);
    q->ready = true;
    return hipSuccess;
}

void quad_free(QuadOp* q) {
    if (q->tables) (void)hipFree(q->tables);
    if (q->index) (void)hipFree(q->index);
    if (q->scratch) (void)hipFree(q->scratch);
    *q = QuadOp{};
}

hipError_t launch_quad_K(hp_ctx* c, const QuadOp* q, const Fields& in, const Fields& out,
                         int nrhs) {
    if (!q->ready) return hipErrorNotInitialized;
    const int nq = q->nq, nM = c->nM;
    const long long s1 = (long long)nq * nM * nM, s2 = (long long)nq * nq * nM,
                    s3 = (long long)nq * nq * nq;
    double* S1 = q->scratch;          // 7 fields after mode 1 (and after transposed mode 2)
    double* S2 = S1 + 7 * s1;         // 10 fields after mode 2 (and after transposed mode 3)
    double* FL = S2 + 10 * s2;        // QNF flux fields at the points
    hipStream_t st = c->stream;
    hipError_t e;
    // table type of component c along direction d: interior degree p in its own direction
    auto T = [](int comp, int dir) { return comp == dir ? 1 : 0; };
    for (int r = 0; r < nrhs; ++r) {
        // mode 1: a_c = V u_c, b_c = D u_c (slots 2c, 2c+1), pressure a_p = V p (slot 6)
        QJobs J{};
        int n = 0;
        for (int comp = 0; comp < 4; ++comp) {
            const long long* d = c->dims[comp];
            const double* x = in.f[comp] + (long long)r * in.stride[comp];
            const int t = comp < 3 ? T(comp, 0) : 0;
            const int nj = comp < 3 ? 2 : 1;
            for (int k = 0; k < nj; ++k) {
                QJob& j = J.j[n];
                j.a = x;
                j.b = nullptr;
                j.out = S1 + (long long)(comp < 3 ? 2 * comp + k : 6) * s1;
                j.ma = k == 0 ? q->V[t] : q->D[t];
                j.d0 = (int)d[0];
                j.d1 = (int)d[1];
                j.d2 = (int)d[2];
                j.nout = (long long)nq * d[1] * d[2];
                ++n;
            }
        }
        if ((e = run_pass<0>(st, J, n)) != hipSuccess) return e;
        // mode 2: (V1V2, V1D2) from a_c, (D1V2) from b_c into slots 3c..3c+2; pressure slot 9
        J = QJobs{};
        n = 0;
        for (int comp = 0; comp < 4; ++comp) {
            const long long* d = c->dims[comp];
            const int t = comp < 3 ? T(comp, 1) : 0;
            const int nj = comp < 3 ? 3 : 1;
            for (int k = 0; k < nj; ++k) {
                QJob& j = J.j[n];
                const int src = comp < 3 ? 2 * comp + (k == 2 ? 1 : 0) : 6;
                j.a = S1 + (long long)src * s1;
                j.b = nullptr;
                j.out = S2 + (long long)(comp < 3 ? 3 * comp + k : 9) * s2;
                j.ma = k == 1 ? q->D[t] : q->V[t];
                j.d0 = nq;
                j.d1 = (int)d[1];
                j.d2 = (int)d[2];
                j.nout = (long long)nq * nq * d[2];
                ++n;
            }
        }
        if ((e = run_pass<1>(st, J, n)) != hipSuccess) return e;
        // mode 3 evaluation and the flux at every point
        QFluxArgs A{};
        for (int k = 0; k < 10; ++k) A.in[k] = S2 + (long long)k * s2;
        for (int k = 0; k < QNF; ++k) A.out[k] = FL + (long long)k * s3;
        for (int t = 0; t < 2; ++t) {
            A.V[t] = q->V[t];
            A.D[t] = q->D[t];
        }
        A.wq = q->wq;
        A.nq = nq;
        A.nu = c->nu;
        A.alpha = c->tab.alpha;
        hipLaunchKernelGGL(k_qflux, dim3((unsigned)(xcd_tiles((long long)nq * nq) * nq)), dim3(QT), 0,
                           st, A);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // transposed mode 3: (V1V2) <- V^T F_v + D^T S_c3, (V1D2) <- V^T S_c2,
        // (D1V2) <- V^T S_c1; pressure <- V^T F_q.  Component 2's (D1V2) is
        // V^T S_12 with the degree p-1 table, as component 1's (V1D2): one job
        // (slot 1) serves both.
        J = QJobs{};
        n = 0;
        for (int comp = 0; comp < 4; ++comp) {
            const long long* d = c->dims[comp];
            const int t = comp < 3 ? T(comp, 2) : 0;
            const int nj = comp < 3 ? 3 : 1;
            for (int k = 0; k < nj; ++k) {
                if (comp == 1 && k == 2) continue;
                QJob& j = J.j[n];
                j.d0 = nq;
                j.d1 = nq;
                j.d2 = nq;
                j.nout = (long long)nq * nq * d[2];
                j.out = S2 + (long long)(comp < 3 ? 3 * comp + k : 9) * s2;
                j.b = nullptr;
                j.ma = q->VT[t];
                if (comp == 3) {
                    j.a = FL + 9 * s3;
                } else if (k == 0) {
                    j.a = FL + (long long)comp * s3;
                    j.b = FL + (long long)qsym(comp, 2) * s3;
                    j.mb = q->DT[t];
                } else {
                    j.a = FL + (long long)qsym(comp, k == 1 ? 1 : 0) * s3;
                }
                ++n;
            }
        }
        {
            int rmax = 0;
            for (int i = 0; i < n; ++i) rmax = std::max(rmax, J.j[i].ma.rows);
            const unsigned nb =
                (unsigned)(xcd_tiles((long long)nq * nq) * ((rmax + QJB - 1) / QJB));
            hipLaunchKernelGGL(k_qpass3t, dim3(nb, n), dim3(QT), 0, st, J);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        // transposed mode 2: a_c <- V^T (V1V2) + D^T (V1D2), b_c <- V^T (D1V2); pressure
        J = QJobs{};
        n = 0;
        for (int comp = 0; comp < 4; ++comp) {
            const long long* d = c->dims[comp];
            const int t = comp < 3 ? T(comp, 1) : 0;
            const int nj = comp < 3 ? 2 : 1;
            for (int k = 0; k < nj; ++k) {
                QJob& j = J.j[n];
                j.d0 = nq;
                j.d1 = nq;
                j.d2 = (int)d[2];
                j.nout = (long long)nq * d[1] * d[2];
                j.out = S1 + (long long)(comp < 3 ? 2 * comp + k : 6) * s1;
                j.ma = q->VT[t];
                j.b = nullptr;
                if (comp == 3) {
                    j.a = S2 + 9 * s2;
                } else if (k == 0) {
                    j.a = S2 + (long long)(3 * comp) * s2;
                    j.b = S2 + (long long)(3 * comp + 1) * s2;
                    j.mb = q->DT[t];
                } else {
                    j.a = S2 + (long long)(comp == 1 ? 1 : 3 * comp + 2) * s2;
                }
                ++n;
            }
        }
        if ((e = run_pass<1>(st, J, n)) != hipSuccess) return e;
        // transposed mode 1: y_c = V^T a_c + D^T b_c; y_p = V^T a_p
        J = QJobs{};
        n = 0;
        for (int comp = 0; comp < 4; ++comp) {
            const long long* d = c->dims[comp];
            const int t = comp < 3 ? T(comp, 0) : 0;
            QJob& j = J.j[n];
            j.d0 = nq;
            j.d1 = (int)d[1];
            j.d2 = (int)d[2];
            j.nout = d[0] * d[1] * d[2];
            j.out = out.f[comp] + (long long)r * out.stride[comp];
            j.ma = q->VT[t];
            j.b = nullptr;
            if (comp == 3) {
                j.a = S1 + 6 * s1;
            } else {
                j.a = S1 + (long long)(2 * comp) * s1;
                j.b = S1 + (long long)(2 * comp + 1) * s1;
                j.mb = q->DT[t];
            }
            ++n;
        }
        if ((e = run_pass<0>(st, J, n)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hp
