// Internal declarations shared by the HIP sources of the solver library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/hyperpower.h"
#include "setup1d.h"

namespace hp {

// Banded symmetric 1D matrices used by the sum-factorised operators.
// Row i of band matrix `id` holds A[i][i-w .. i+w] (zeros outside range).
// BD_M is D^^T M^ (interior degree-p rows, half-width p): the coupling of a
// velocity component with z in its own direction.
enum BandId { BK_N = 0, BM_N = 1, BM_C = 2, BT_C = 3, BD_M = 4, NBAND = 5 };

struct BandTables {
    const double* ptr[NBAND];  // device pointers, row-major n x (2w+1)
    int n[NBAND];
    int w[NBAND];
};

// Dense (padded) matrices for fast diagonalisation on MFMA tiles.
template <typename T>
struct FDTables {
    const T* UK;   // interior degree-p eigenvectors, NNp x NNp row-major (U)
    const T* UKt;  // U^T
    const T* UT;   // degree p-1 eigenvectors of (T^, M^)
    const T* UTt;
    const T* Mi;   // M^^{-1}, NMp x NMp
    const double* lamK;  // nN eigenvalues
    const double* lamT;  // nM eigenvalues
    int nN, nM, NNp, NMp;
};

// A set of pointers to the four blocks of one (batched) vector.
struct Fields {
    double* f[4];       // u1, u2, u3, p (any may be null when unused)
    long long stride[4];  // distance between right-hand sides, per block
};

struct Workspace {
    double* base = nullptr;
    size_t bytes = 0;
};

// Launch shape of the operator kernels: i3-planes per workgroup and the
// order of the velocity workgroups (1: component fastest).
struct OpShape {
    int kchunk = 0;
    int comp_fast = 1;
    int slabs = 1;  // i3-slabs, each running the pressure then the velocity kernel
    int fused = 0;  // K and A in one single-pass kernel (k_fused)
    int staged = 0;  // K and A velocity: all planes of a chunk at once (k_vel_all)
    int dma = 1;     // streaming velocity kernel: staging by direct-to-LDS loads (k_vel_dma)
    int pwide = 0;   // streaming pressure kernel on 32 x 8 tiles instead of 16 x 8
};
struct OpTuned {
    int nrhs = 0;
    int kchunk = 0;  // 0: not tuned
    OpShape shape;
};

// Banded table of the quadrature-based operator: row r holds
// A[r][start[r] .. start[r] + w) of a rows x cols matrix.
struct QBand {
    const int* start;
    const double* val;
    int rows, cols, w;
};

// Device state of the quadrature-based forward operator (quad.hip): basis
// tables at the points of one direction ([0] degree p-1, [1] interior degree
// p; V values, D derivatives, VT/DT their transposes), the point weights and
// the scratch of one right-hand side.
struct QuadOp {
    bool ready = false;
    int nq = 0;
    double* tables = nullptr;
    int* index = nullptr;
    double* scratch = nullptr;
    size_t scratch_doubles = 0;
    QBand V[2]{}, D[2]{}, VT[2]{}, DT[2]{};
    const double* wq = nullptr;
};

}  // namespace hp

struct hp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hp_opts opts{};
    int E = 0, p = 0, nN = 0, nM = 0;
    double nu = 1.0;
    long long dims[4][3]{};
    long long off[5]{};
    long long nV = 0, nQ = 0, N = 0;
    hp::Tables1D tab;
    // device tables
    double* d_tables = nullptr;  // one allocation for bands + FD tables
    float* d_tables32 = nullptr;
    hp::BandTables band{};
    hp::FDTables<double> fd64{};
    hp::FDTables<float> fd32{};
    bool fd_ok = false;  // fast-diagonalisation tables present
    // workspace (per right-hand side sizes scale with max_rhs)
    double* ws = nullptr;
    size_t ws_doubles = 0;
    // reduction scratch
    double* d_red = nullptr;
    double* h_red = nullptr;  // pinned host mirror
    int red_slots = 0;
    // launch shapes picked by the autotuner (for 1 and max_rhs right-hand
    // sides), a shape forced while tuning, and the fast-diagonalisation plan
    // per precision (-1: the default plan)
    hp::OpTuned op_tuned[2];
    hp::OpShape op_force{};
    int fd_tuned[3] = {-1, -1, -1};
    int fd_force = -1;
    double op_tuned_us[2] = {0.0, 0.0};
    double fd_tuned_us[3] = {0.0, 0.0, 0.0};
};

namespace hp {

// ---- operator kernels (ops.hip) -------------------------------------------
// Modes of the sum-factorised operator:
//  OP_K  : y_u = nu L u + D^T M_q (nu D u + p), y_p = M_q D u
//  OP_A  : y_u = nu L u + D^T M_q (nu D u)
//  OP_B  : y_u = D^T M_q p
//  OP_BT : y_p = M_q D u
//  OP_MV : y_u = M_V u (velocity mass matrix)
//  OP_DT : y_u = D^T p (the pressure input in the place of w; with
//          P_{Q,0}^{-1} = 2 nu M_q^{-1}, B P_{Q,0}^{-1} p = 2 nu D^T p)
enum OpMode { OP_K = 0, OP_A = 1, OP_B = 2, OP_BT = 3, OP_MV = 4, OP_DT = 5 };

// y_u := alpha * (op result) + beta * src_u  (src_u may alias y_u);
// y_p := op result.
hipError_t launch_operator(hp_ctx* c, OpMode mode, const Fields& in, const Fields& out,
                           double alpha, double beta, const Fields* src, int nrhs);

hipError_t ops_init_attributes();

// ---- quadrature-based forward operator (quad.hip) ---------------------------
// Builds the point tables and allocates the scratch (once per context).
hipError_t quad_setup(hp_ctx* c, QuadOp* q);
void quad_free(QuadOp* q);
// out = K in by global sum factorisation at the Gauss points (the same
// matrix as OP_K of launch_operator, up to rounding); out must not alias in.
hipError_t launch_quad_K(hp_ctx* c, const QuadOp* q, const Fields& in, const Fields& out,
                         int nrhs);
// the shape launch_operator uses for nrhs right-hand sides (forced, user
// option, tuned, else the cost model) and the cost model alone
OpShape op_shape(const hp_ctx* c, int nrhs);
OpShape op_model_shape(const hp_ctx* c, int nrhs);
// whether the all-planes velocity kernel exists for this degree and chunk
bool op_staged_ok(int degree, int kchunk);
// doubles of workspace per right-hand side used by launch_operator (holds w);
// the fast-diagonalisation scratch follows at ops_ws_stride(c) * max_rhs
long long ops_ws_stride(const hp_ctx* c);

// ---- fast diagonalisation (fd.hip) -----------------------------------------
hipError_t fd_init_attributes();
// y = P_0^{-1} x restricted to the selected blocks (velocity and/or pressure);
// accumulate: y += result instead of y = result.
// dot (FP64, the velocity blocks or the pressure block alone; may be null):
// the last launch also writes partial sums of (final output) . dot->with to
// dot->part[r * fd_dot_count(c, vel) + i] -- velocity: one per (field,
// i3-plane), i = f nM + k, and with FD_PLAN_SPLIT one per (field, plane, row
// block b), i = f nM + k + 3 nM b (slots no workgroup reaches -- planes or
// row blocks a field lacks -- are never written: kept zero by the caller);
// pressure: one per workgroup of its mode-3 launch.
// comb (FP64, may be null): the input is ca in + cb comb->b + cc comb->c,
// formed where the first launch reads it (as k_axpbypcz would).
struct FdDot {
    const double* with;  // full vector, same layout and rhs stride as the output's
    double* part;
};
struct FdComb {
    Fields b, c;
    double ca, cb, cc;
};
hipError_t launch_P0(hp_ctx* c, const Fields& in, const Fields& out, bool vel, bool pres,
                     bool accumulate, int precision, int nrhs, const FdDot* dot = nullptr,
                     const FdComb* comb = nullptr);
long long fd_dot_count(const hp_ctx* c, bool vel);
// the largest fd_dot_count over the plans (the partial buffers' size)
long long fd_dot_capacity(const hp_ctx* c, bool vel);
// fast-diagonalisation plans: bit 0 = one MFMA tile per wave (wide kernels),
// bit 1 = stage the 1D matrices in LDS, bit 2 = 2x2 tile blocks per wave;
// FD_PLAN_GEMM = the mode products as batched GEMMs over HBM (any direction
// length; the only plan for directions longer than 128); FD_PLAN_SPLIT = one
// 16-row block of a plane per 4-wave workgroup and 16 z rows per workgroup
// (several times the workgroups of plans 0-7, for small meshes).  Whether plan
// `plan` fits the LDS for `precision`, and the plan launch_P0 uses (forced,
// option, tuned, default).
constexpr int FD_PLAN_GEMM = 8;
constexpr int FD_PLAN_SPLIT = 9;
constexpr int FD_PLAN_LAST = 9;
bool fd_plan_valid(const hp_ctx* c, int precision, int plan);
int fd_plan_in_use(const hp_ctx* c, int precision);

// ---- vector kernels (krylov.hip) ----------------------------------------------
hipError_t vec_axpby(hipStream_t s, long long n, double a, const double* x, double b,
                     double* y);  // y = a x + b y
hipError_t vec_copy(hipStream_t s, long long n, const double* x, double* y);
hipError_t vec_zero(hipStream_t s, long long n, double* y);
// dot products of nrhs pairs of vectors (stride ld), results to host `out`
hipError_t vec_dots(hp_ctx* c, long long n, long long ld, const double* x, const double* y,
                    int nrhs, double* out);

}  // namespace hp
