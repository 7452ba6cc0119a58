// Internal declarations of the gpfvm library (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/gpfvm.h"

namespace gpfvm {

typedef long long i64;

// ---------------------------------------------------------------------------
// Grouped, batched, multi-segment GEMM descriptor.  One launch processes the
// output tiles (32x32 or 64x64, by the stage's kernel) of every descriptor in
// an array.  For descriptor D and
// batch b:
//   acc_s = sum over segments g with slot s of  alpha_g * A_g[b] (M x K_g) * B_g[b] (K_g x N)
//   C[b]  = acc_0 + escale[b] o acc_1 + gamma * X[b] + beta * C[b]
// Every operand is addressed through (row, col, batch) element strides, so
// transposes and Kronecker mode products of row-major tensors need no copies.
// ---------------------------------------------------------------------------
constexpr int MAXSEG = 12;
constexpr int TILE = 32;

struct Seg {
  const void* A;
  const void* B;
  i64 a_rs, a_cs, a_bs;
  i64 b_rs, b_cs, b_bs;
  int K;
  int slot;     // 0 or 1 (slot 1 is multiplied elementwise by escale)
  int tri;      // 0 dense; 1/2: A lower/upper-triangular; 3/4: B upper/lower-triangular
                // (the K loop skips the blocks that are zero for this output tile)
  int pad;
  double alpha;
};

struct GemmDesc {
  void* C;
  i64 c_rs, c_cs, c_bs;
  const double* escale;    // float64 scale (also for float32 plans)
  i64 e_rs, e_cs, e_bs;
  const void* X;           // elementwise addend (element type of C), or null
  i64 x_rs, x_cs, x_bs;
  double gamma;
  double beta;
  int M, N, batch, nseg;
  int tiles_m, tiles_n, lower_only, pad;
  i64 tile_begin;
  Seg seg[MAXSEG];
};

// Element type of a plan: float64; float32 on the float32 matrix cores; float32
// in HBM with the products on the bfloat16 matrix cores, each operand split
// into three bfloat16 slices (float32 accuracy, lowp.hip).
enum Elt { F64 = 0, F32 = 1, F32B = 2 };

// One kernel launch: a set of descriptors whose outputs do not overlap.
// Streaming products carried by a GEMM stage's launch as extra workgroups
// after its tiles (float64).  They must not touch the stage's own inputs or
// outputs.
//   RIDE_ROWS: out[j] = M[j,:] . v (divided by eta[j] when eta is set), j < nr
//   RIDE_COLS: out[c] = sum_j M[j][c] v[j], c < N (v: nr coefficients)
//   RIDE_QFV:  the nr work units of the factored point correction (QFactor)
enum RiderKind { RIDE_NONE = 0, RIDE_ROWS = 1, RIDE_COLS = 2, RIDE_QFV = 3 };

// Factored point correction for a 2-D volume tensor (n0 x n1 cells, dim 1
// fastest) whose point groups are each pinned in one dimension.  With
// G_bp = sum_r Gf_r (x)_{p_r} q_r (piece r = one group and one PDE term; q_r
// the group's factor over the cells of its pinned dimension p_r, Gf_r its
// n_b x n_{f_r} factor over the free one), Q = L^{-1} G_bp is
// sum_r M_r (x)_{p_r} q_r with M_r = L^{-1} Gf_r, and
//   Q^T Q x = sum_r q_r (x)_{p_r} (P w)_r,   w_r = x contracted with q_r over p_r,
// where P = M_cat^T M_cat (W x W) and M_cat = [M_0 | M_1 | ...] (n_b x W).
// Pieces pinned in dimension 0 come first.  v = P w is formed as nunit
// partial sums stored piece-major (vpart[nunit off_r + u nf_r + j]), so that
// sum_r q_r (x) v_r is two GEMM segments of the volume operator's last stage:
// [q_r columns, each repeated nunit times] x vpart (pinned dimension 0) and
// vpart^T x [q_r rows, repeated] (pinned dimension 1).
constexpr int QF_MAXR = 16, QF_MAXW = 2048;
constexpr int QF_UW = 16;          // free indices per work unit of v = P w
struct QFactor {
  int R = 0, W = 0, n0 = 0, n1 = 0;
  int nunit = 0;                   // work units of v = P w: QF_UW free indices of one piece each
  int w0 = 0;                      // free indices of the pieces pinned in dimension 0 (R0 n1)
  int p[QF_MAXR];                  // pinned dimension of piece r (0 or 1)
  int off[QF_MAXR];                // first index of piece r in the concatenated free index
  const double* q[QF_MAXR];        // n_{p_r} values
  const double* P = nullptr;       // W x W, row-major
};
struct Rider {
  int kind = RIDE_NONE;
  int nr = 0;
  i64 N = 0;
  const double* M = nullptr;   // nr x N, row-major
  const double* v = nullptr;
  const double* eta = nullptr;
  double* out = nullptr;
  const QFactor* qf = nullptr; // RIDE_QFV: the factored correction (device)
};

struct Stage {
  std::vector<GemmDesc> descs;
  GemmDesc* d_descs = nullptr;
  i64 tiles = 0;
  int kind = 0;    // GEMM_SPLITK / GEMM_LDS16 / GEMM_LDS32 / GEMM_LDS64 (set when the stage is uploaded)
  int slot1 = 0;   // some segment accumulates into slot 1
  Rider rider;     // launched with the stage (kind RIDE_NONE: none)
  // thin products (one output row or column, one segment, no epilogue): moved to the end
  // of descs at upload and run by a one-thread-per-output kernel; tile_begin holds their
  // output offsets
  int nthin = 0;
  i64 thin_outputs = 0;
};
enum GemmKind { GEMM_SPLITK = 0, GEMM_LDS32 = 1, GEMM_LDS64 = 2, GEMM_LDS16 = 3, GEMM_BF16S32 = 4, GEMM_BF16S64 = 5 };

// Point-block correction of the volume system as Q^T Q with Q = L^{-1} G_bp
// (n_b x N, row-major), used for one right-hand side when Q is small enough
// to stay resident (it replaces the cross-block Kronecker products and the
// point-block triangular solves of every operator application).
constexpr i64 QFORM_MAX_BYTES = 256LL << 20;
inline bool qform_ok(i64 N, i64 nb) { return nb > 0 && 8 * N * nb <= QFORM_MAX_BYTES; }

// Caching device allocator shared by the handles of one server: released
// blocks are kept and reused (best fit within 2x), so a serving loop in steady
// state calls neither hipMalloc nor hipFree (both can stall other streams).
struct DeviceCache {
  std::mutex mu;
  std::multimap<size_t, void*> free_blocks;    // size -> block
  std::map<void*, size_t> sizes;               // every block ever allocated
  i64 cached_bytes = 0, total_bytes = 0;
  void* get(size_t nbytes);
  void put(void* p);
  void release_all();
  i64 trim();                      // free the unused blocks only; returns their bytes
};

// Device memory arena owned by a handle (freed at destroy).  Allocations up
// to a quarter of a slab are carved from 8 MiB slabs (256-byte aligned), so a
// handle makes a few dozen runtime allocations instead of hundreds; larger
// ones get their own block.  Every allocation is registered as its own range.
constexpr size_t ARENA_SLAB = 8u << 20;
struct Arena {
  std::vector<void*> ptrs;         // slabs and large blocks (from hipMalloc or the cache)
  std::vector<void*> regs;         // registered allocations
  char* slab = nullptr;
  size_t slab_left = 0;
  i64 bytes = 0;                   // device bytes held (slabs counted whole)
  DeviceCache* cache = nullptr;    // when set, blocks come from / go back to it
  // fixed mode (fixed != null): allocations are carved from [fixed, fixed + fixed_cap)
  // and nothing is ever allocated from or returned to the runtime
  char* fixed = nullptr;
  size_t fixed_cap = 0, fixed_used = 0;
  void* alloc(size_t nbytes);      // returns nullptr on failure
  void release();
};

// ---- a Kronecker-sum operator ------------------------------------------------
// y = sum_s alpha_s * (Lscale_s o) (M_{s,0} x M_{s,1} x ... ) (Rscale_s o x_s)
// with x_s = x + in_off_s (per right-hand side), M_{s,i} row-major (rows_i x cols_i).
struct KronTerm {
  const void* M[3];      // device matrices (element type of the plan)
  i64 ld[3];             // leading dimension (row stride) of M
  int trans[3];          // 1: use M^T
  double alpha;
  int lscale, rscale;    // 1: scale by the per-volume coefficient
  i64 in_off;            // offset of this term's input inside x (per rhs)
};

struct KronOp {
  int d = 0;
  int in_shape[3] = {1, 1, 1};
  int out_shape[3] = {1, 1, 1};
  std::vector<KronTerm> terms;
  i64 in_len = 0;        // elements of x per rhs (>= max in_off + prod(in_shape))
  i64 out_off = 0;       // offset of the output inside y (per rhs)
};

// Elementwise pre-step of a plan: xs[r*len + i] = coef[i] * x[r*x_stride + i],
// i < len (the number of volumes), r < nrhs.
struct Prescale {
  const void* x = nullptr;
  const void* coef = nullptr;
  void* xs = nullptr;
  i64 len = 0;
  i64 x_stride = 0;
  int nrhs = 0;
};

// Compiled plan: stages of grouped GEMMs bound to fixed input/output buffers.
struct Plan {
  Elt elt = F64;
  int nrhs = 0;
  const void* x = nullptr;         // bound input (in_len * nrhs)
  void* y = nullptr;               // bound output (prod(out_shape) * nrhs)
  void* xs = nullptr;              // scaled input (cell_coef o x), if needed
  i64 in_len = 0, out_len = 0;
  const void* scale_src = nullptr; // per-volume coefficient (double or float)
  std::vector<Prescale> pre;       // elementwise pre-steps
  std::vector<Stage> stages;       // the final stages accumulate into y
  double flops = 0;                // executed flops per application (all rhs)
};

struct Factor {            // (n1 x n2) matrix on the device, row-major
  double* d = nullptr;
  float* f = nullptr;      // float32 copy for the mixed plan (or null)
  int n1 = 0, n2 = 0;
};

struct PointComp {         // coef * w(x) * d^deriv u_out(x), w separable over the grid
  int deriv[3] = {0, 0, 0};
  double coef = 1;
  int out = 0;
  std::vector<double> w[3];   // per-dim weights (empty: 1)
};

struct Group {
  int n[3] = {1, 1, 1};
  int deriv[3] = {0, 0, 0};   // the first component's derivative (single-term groups)
  double noise = 0;
  i64 size = 0, offset = 0;
  std::vector<double> axis[3];
  std::vector<PointComp> comps;   // the observation is the sum of its components
};

struct PdeTerm {           // coef * (cell_coef if cellwise) * d^alpha u_out, in equation eq
  int alpha[3] = {0, 0, 0};
  double coef = 0;
  int cellwise = 0;
  int out = 0, eq = 0;
};

struct GramTerm {          // merged volume-Gram term (block eq1 x eq2, outputscale included)
  int m[3] = {0, 0, 0};
  double coef = 0;
  int lflag = 0, rflag = 0;
  int e1 = 0, e2 = 0;
};

// Element offsets between the problems of a batch: problem z = blockIdx.y of a
// batched launch reads and writes each operand at base + z * stride (all zero:
// one problem).  M: stored matrices (directions, S D), v: length-N vectors,
// u: coefficient partials, eta: eta arrays, part: per-workgroup partial sums,
// scal / flag: the solver's device scalars and flags.
struct BatchStrides {
  i64 M = 0, v = 0, u = 0, eta = 0, part = 0, scal = 0, flag = 0;
};

// ---- kernels / launchers (kernels.hip) --------------------------------------
hipError_t launch_factor(int kind, int kq, int p, int q, int n1, const double* a1, int n2, const double* a2,
                         double ell, double scale, double* out, i64 ld, hipStream_t s);
hipError_t launch_gemm_stage(Elt elt, const Stage& st, hipStream_t s);   // kernel chosen by st.kind
hipError_t launch_gemm_bf16s(const Stage& st, hipStream_t s);           // GEMM_BF16S32 / 64 (lowp.hip)
hipError_t launch_scale(Elt elt, const void* src, i64 src_stride, const void* coef, void* dst, i64 dst_stride, i64 n,
                        int nrhs, hipStream_t s);
hipError_t launch_axpby(i64 n, double a, const double* x, double b, double* y, hipStream_t s);
hipError_t launch_copy_f64_to_f32(const double* x, float* y, i64 n, hipStream_t s);
hipError_t launch_copy_f32_to_f64(const float* x, double* y, i64 n, hipStream_t s);
hipError_t launch_lincomb(int nmat, const double* const* mats, const double* coefs, i64 len,
                          double* out, hipStream_t s);
hipError_t launch_fill(double* p, double v, i64 n, hipStream_t s);
hipError_t launch_add_diag(double* A, i64 ld, i64 n0, i64 n, const double* vals, hipStream_t s);

// deterministic reductions: out[0] = sum x*y (two passes, fixed order)
hipError_t launch_dot(i64 n, const double* x, const double* y, double* partial, double* out,
                      hipStream_t s, int batch = 1, const BatchStrides& bs = BatchStrides());
// same, then the IterGP stopping test on out[0] (see solver.hip for the layout)
hipError_t launch_dot_check(i64 n, const double* x, double* partial, double* scal, int* flag, int max_iter,
                            hipStream_t s, int batch = 1, const BatchStrides& bs = BatchStrides());
// partial sums of a (batched) dot product: DOT_PARTIALS per problem
constexpr int DOT_PARTIALS = 512;
// W = G_bb^{-1} U for n_b <= SMALL_GINV_MAX, one right-hand side, one workgroup
// (needs the transposes Lt = L^T and Linvt = L^{-T} as row-major copies)
constexpr int SMALL_GINV_MAX = 512;
hipError_t launch_ginv_small(int nb, const double* L, const double* Linv, const double* Lt, const double* Linvt,
                             const double* U, double* W, hipStream_t s);
hipError_t launch_transpose(const double* A, double* B, int n, hipStream_t s);
// Streaming products with a row-major nr x N matrix M:
//   rows_dot:    part[j * nch + ch] = sum_{k in chunk ch} M[j][k] x[k], nch = rows_dot_chunks(nr, N)
//                (part holds nr * nch <= nr + ROWS_DOT_TARGET - 1 values; with the column update's
//                finished coefficients after them, 2 nr + ROWS_DOT_TARGET - 1)
//   rows_dot_full: out[j] = sum_k M[j][k] x[k]
//   cols_update: u_j = (sum_ch u[j * u_nch + ch]) / (eta ? eta[j] : 1);
//                out[c] = base[c] - sum_j M[j][c] u_j (and out2[c] = out[c] if out2);
//                with M2: out3[c] = base2[c] - sum_j M2[j][c] u_j.   base may alias out.
//                For N >= 2^18 with u_nch > 1 or eta, the nr finished u_j are first written to
//                u + nr * u_nch: u then holds room for nr * (u_nch + 1) values.
//   (rows_dot with xm: the dots are taken with x - xm)
constexpr int ROWS_DOT_TARGET = 2048;   // workgroups a row-dot launch aims at
int rows_dot_chunks(int nr, i64 N);
hipError_t launch_rows_dot(int nr, i64 N, const double* M, const double* x, double* part, hipStream_t s,
                           const double* xm = nullptr, int batch = 1, const BatchStrides& bs = BatchStrides());
hipError_t launch_rows_dot_full(int nr, i64 N, const double* M, const double* x, double* out, hipStream_t s);
// the nunit partial sums of v = P w(x) of the factored point correction, on their own
hipError_t launch_qf_v(const QFactor* F, int nunit, const double* x, double* vpart, hipStream_t s);
//   With M2 and dot_part: also dot_part[g] = workgroup g's share of sum_c out[c] * out3[c]
//   (ceil(N/64) values; their fixed-order sum is the dot product).
//   With base2m: out3[c] = (base2[c] - base2m[c]) - sum_j M2[j][c] u_j.
hipError_t launch_cols_update(int nr, i64 N, const double* M, double* u, int u_nch, const double* eta,
                              const double* base, double* out, double* out2, const double* M2, const double* base2,
                              double* out3, hipStream_t s, double* dot_part = nullptr,
                              const double* base2m = nullptr, int batch = 1,
                              const BatchStrides& bs = BatchStrides());
// y[i] = add[i] + alpha * sum_k M[i][k] x[k] over k <= i (upper = 0) or k >= i (upper = 1)
hipError_t launch_trmv_rows(int n, const double* M, const double* x, double* y, double alpha, const double* add,
                            int upper, hipStream_t s);

}  // namespace gpfvm

namespace gpfvm { struct GramMeta; }

// Bound operator plans of one handle for one right-hand-side count.
struct gpfvm_opset {
  int nrhs = 0;
  // full-Gram matvec on [points; volumes] vectors (internal buffers XF, YF)
  double *XF = nullptr, *YF = nullptr, *TB = nullptr;
  gpfvm::Plan pp, bp, pb;
  gpfvm::Stage gbb_t, gbb_l;        // y_b += L (L^T x_b)
};

// Operators of the volume (Schur) system S = G_pp + s2 I - G_pb G_bb^{-1} G_bp.
// G_bb^{-1} is applied as two triangular solves with L, each computed with the
// explicit L^{-1} and corrected once by the residual with L (backward stable).
struct gpfvm_sop {
  int nrhs = 0;
  gpfvm::Elt elt = gpfvm::F64;      // element type of the volume block pp
  void *X = nullptr, *Y = nullptr;  // N * nrhs (float64)
  void *X32 = nullptr, *Y32 = nullptr;  // N * nrhs (float32, mixed operator)
  void *U = nullptr, *T = nullptr, *W = nullptr, *R = nullptr;   // n_b * nrhs
  gpfvm::Plan pp, bp, pb;           // pp: float64 or float32; bp, pb: float64
  std::vector<gpfvm::Stage> ginv;   // W = G_bb^{-1} U (six stages)
  bool ginv_small = false;          // one-workgroup kernel instead of the stages
  bool qform = false;               // correction as Q^T (Q x) with the handle's Q
  gpfvm::Plan front;                // pp and bp merged into shared launches
  double flops_pp = 0;
  // Q-form split application (two-pass solver loop): pp_split leaves Y = G_pp X + s2 X and
  // csub = Q^T (Q X), riding on the first and the last stage; consumers use Y - csub.
  gpfvm::Plan pp_split;
  double* csub = nullptr;
  bool split = false;
  // factored form of the correction (2-D, every point group pinned in one dimension): the
  // partial sums of v = P w ride on the first stage of pp_split, and sum_r q_r (x) v_r is
  // subtracted by two extra segments of its last stage, so pp_split gives Y = S X; no resident Q
  bool qf = false;
  double* qf_v = nullptr;          // nunit x W partial sums of v, piece-major
};

// State of a batched solve (problems sharing the handle's operator; see
// gpfvm::batch_solve): per-problem slices of the solver state, problem z at
// offset z * (its length).
struct GpfvmBatch {
  int R = 0;
  double* yobs = nullptr;          // R x n data [y_b; int_V f]
  double* bS = nullptr;            // R x N volume-system right-hand sides
  double* v = nullptr;             // R x N weights
  double* Dd = nullptr;            // R x max_iter x N directions
  double* Qd = nullptr;            // R x max_iter x N  S D
  double* eta = nullptr;           // R x max_iter
  std::vector<int> iters;          // directions stored per problem
};

struct gpfvm_handle {
  int d = 0;
  int nc[3] = {1, 1, 1};
  gpfvm::i64 N = 0, n = 0;         // N: volume observations (neq per cell), n = n_b + N
  gpfvm::i64 Nc = 0;               // cells
  int nb = 0;
  int nout = 1, neq = 1;           // outputs of the prior, equations per cell
  bool multi = false;              // several outputs or equations, or multi-term point groups
  double sfo[GPFVM_MAX_OUTPUTS] = {1, 1, 1, 1, 1, 1, 1, 1};   // outputscale per output
  double ell[3] = {1, 1, 1};
  int kq[3] = {-1, -1, -1};        // per dim: -1 squared exponential, q >= 0 Matern nu = q + 1/2
  double sf2 = 1;                  // outputscale of output 0
  double sig_pde = 0;
  int has_cc = 0;
  int tile = GPFVM_TILE_FP32;
  int max_iter = 0;
  hipStream_t stream = nullptr;
  std::string err;

  std::vector<gpfvm::PdeTerm> pterms;
  std::vector<gpfvm::GramTerm> gterms;
  std::vector<gpfvm::Group> groups;
  std::vector<double> edges_h[3];

  gpfvm::Arena arena;
  double* edges[3] = {nullptr, nullptr, nullptr};
  double* cellc = nullptr;         // per-volume coefficient, repeated for each equation (N values), or null
  float* cellc_f = nullptr;
  double* yobs = nullptr;          // n: [y_b ; int_V f]
  std::map<std::pair<int, int>, gpfvm::Factor> Dfac;   // (dim, order) -> D_i(order)
  std::vector<gpfvm::Factor> combos;                  // pre-summed factor matrices
  std::vector<std::vector<std::array<gpfvm::Factor, 3>>> Qfac;   // [group][comp * nterm + term][dim]
  double* L = nullptr;             // n_b x n_b Cholesky factor of G_bb (lower)
  double* Linv = nullptr;          // n_b x n_b L^{-1} (lower)
  double* Lt = nullptr;            // row-major copies of L^T and L^{-T}
  double* Linvt = nullptr;
  double* Qc = nullptr;            // n_b x N: L^{-1} G_bp (built on first use when qform_ok)
  gpfvm::QFactor* qf = nullptr;    // device: the factored correction (built on first use), or null
  int qf_nunit = 0;                // work units (workgroups) of v = P w
  int qf_w0 = 0, qf_k0 = 0, qf_k1 = 0;   // free indices of the dim-0 pieces; segment depths
  double* qf_aq = nullptr;         // n0 x k0: q_r (pinned dim 0) as columns, each nunit times
  double* qf_bq = nullptr;         // k1 x n1: q_r (pinned dim 1) as rows, each nunit times
  bool process_cache = false;      // arena blocks come from the per-process cache
  float* Linv_f = nullptr;         // float32 L^{-1} (mixed operator; corrections of the row-streaming solves)
  float* Linvt_f = nullptr;        // float32 L^{-T} (row-major), corrections of the row-streaming solves
  gpfvm::GramMeta* meta = nullptr;   // device
  std::vector<gpfvm::KronOp> op_pp, op_pp32;   // one operator per equation (output block)
  std::vector<gpfvm::KronOp> op_bp, op_pb, op_bp32, op_pb32;
  std::map<int, std::unique_ptr<gpfvm_opset>> full_ops;  // by nrhs
  std::map<int, std::unique_ptr<gpfvm_sop>> sops;        // by nrhs (F64)
  std::map<int, std::unique_ptr<gpfvm_sop>> sops32;      // by nrhs (F32)
  // volume-block plans bound to caller buffers: (x, y, nrhs) -> plan
  std::map<std::tuple<const void*, void*, int>, std::unique_ptr<gpfvm::Plan>> vplans;
  std::vector<const void*> user_ranges;                  // registered caller buffers

  // solver state
  bool solved = false;
  int iters = 0;
  double* bS = nullptr;            // volume-system right-hand side (N)
  double* ab0 = nullptr;           // G_bb^{-1} y_b
  double* v = nullptr;             // volume weights (N)
  double* Dd = nullptr;            // directions: column j at Dd + j * N
  double* Qd = nullptr;            // S applied to the directions (two-pass projection)
  bool sd_exact = false;           // Qd holds the float64 S D of every stored direction
  bool cg_only = false;            // the last solve was plain CG: weights only, no directions
  double* eta = nullptr;           // max_iter
  double* vec = nullptr;           // solver vectors (r, s, z, d, ...), 8 * N
  double* aux = nullptr;           // dot partials and coefficients
  double* scal = nullptr;          // device scalars
  int* flag = nullptr;             // device flags
  double* part = nullptr;          // per-workgroup partial sums: d.w (ceil(N/64)), then r.r twice (nblk(N))
  GpfvmBatch batch;                // the last batched solve
};
