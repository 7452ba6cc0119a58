// Cross-file internal interfaces of the gpfvm library.
#pragma once

#include <algorithm>

#include "common.h"

namespace gpfvm {

constexpr int MAXG = GPFVM_MAX_GROUPS;
constexpr int MAXT = GPFVM_MAX_TERMS;
constexpr int MAXGT = 64;                  // merged volume-Gram terms
constexpr int MAXM = 2 * GPFVM_MAX_DERIV + 1;
constexpr int MAXC = GPFVM_MAX_PTERMS;     // components of one point observation

// Everything the dense Gram-entry kernel needs, in one device struct.  Every
// coefficient carries its output's outputscale; a pair of terms on different
// outputs has coefficient 0 (and no factor).  Point-group factors carry the
// components' per-point weights on their group's side.
struct GramMeta {
  int d, nb, ngroup, nterm, ngterm, neq;
  i64 Nc;                                  // cells (volume observations: neq * Nc)
  int nc[3];
  int gn[MAXG][3];
  int gcomp[MAXG];
  i64 goff[MAXG + 1];
  double gnoise[MAXG];
  int tcw[MAXT], teq[MAXT];
  double qcoef[MAXG][MAXC][MAXT];          // point comp x PDE term
  int gm[MAXGT][3];
  double gcoef[MAXGT];
  int gl[MAXGT], gr[MAXGT], ge1[MAXGT], ge2[MAXGT];
  double pcoef[MAXG][MAXC][MAXG][MAXC];    // point comp x point comp
  const double* Dp[3][MAXM];               // cell-cell factors D_i(m), ld = nc[i]
  const double* Qp[MAXG][MAXC][MAXT][3];   // point-cell, ld = nc[i]
  const double* Pp[MAXG][MAXC][MAXG][MAXC][3];   // point-point, ld = gn[g2][i]
  const double* cellc;
  double sig_pde;
};

// The volume operators write disjoint blocks when there are several equations (each its
// own output block, so each its own first write); one operator accumulates its chunks.
inline int pp_accumulate(const gpfvm_handle* h) { return h->op_pp.size() == 1 ? 1 : 0; }

// rows (columns) of a row-major n1 x n2 matrix times wr (wc); a null vector means 1
hipError_t scale_rows_cols(double* A, int n1, int n2, const double* wr, const double* wc, hipStream_t s);

hipError_t launch_gram_block(const GramMeta* meta, i64 r0, i64 nr, i64 c0, i64 nc, double* out, i64 ld,
                             hipStream_t s);
// Checks every descriptor against the live-range registry, then uploads.
// Returns hipErrorInvalidValue (nothing uploaded) if an operand is out of bounds.
hipError_t upload_stages(std::vector<Stage>& stages, Arena& arena, hipStream_t s, Elt elt = F64);
void choose_kernel(Stage& st);
void register_range(const void* p, size_t nbytes);
void unregister_range(const void* p);
bool range_ok(const void* p, size_t nbytes);
int cholesky_and_inverse(double* A, double* Linv, int n, Arena& arena, hipStream_t s, std::string& err);

// Kronecker plans (plan.hip)
// scale_src: per-volume coefficients in the plan's element type (input scaling);
// escale64: the same in float64 (output scaling in the GEMM epilogue).
int compile_kron(const KronOp& op, Elt elt, int nrhs, const void* x, void* y, const void* scale_src,
                 const double* escale64, double beta, const void* addx, double gamma, Arena& arena,
                 hipStream_t s, Plan& out, std::string& err);
// A list of operators into one y: accumulate = 1 sums them (same output
// region), accumulate = 0 writes disjoint regions (KronOp::out_off).
int compile_kron_list(const std::vector<KronOp>& ops, Elt elt, int nrhs, const void* x, i64 x_rhs_stride,
                      void* y, i64 y_rhs_stride, const void* scale_src, const double* escale64, double beta,
                      const void* addx, double gamma, int accumulate, Arena& arena, hipStream_t s, Plan& out,
                      std::string& err);
hipError_t run_plan(const Plan& p, hipStream_t s);
// Merge plans whose outputs do not overlap: stage i of every part runs in one launch.
int merge_plans(const std::vector<const Plan*>& parts, Arena& arena, hipStream_t s, Plan& out, std::string& err);

// handle-level operators (api.hip / solver.hip)
int get_full_ops(gpfvm_handle* h, int nrhs, gpfvm_opset** out);
int get_sop(gpfvm_handle* h, int nrhs, Elt elt, gpfvm_sop** out);
int build_ops32(gpfvm_handle* h);
std::vector<Stage> ginv_stages(const gpfvm_handle* h, int nrhs, const double* U, double* T, double* W, double* R);
hipError_t run_stages(const std::vector<Stage>& st, hipStream_t s);
hipError_t ginv_rows(const gpfvm_handle* h, const double* U, double* T, double* W, double* R, hipStream_t s);
// Grid points per chunk of the posterior's point-block product L^{-1} K_b: n_b x chunk stays
// within 2 GiB per buffer (two buffers).  Chunks of 16384 points on the wave problem run the
// library TRMM 3.5% faster than chunks of 2048.
inline i64 posterior_chunk(i64 nb, i64 M) {
  return std::max<i64>(32, std::min<i64>(M, (256LL << 20) / std::max<i64>(1, nb)));
}

// Directions per batch of the posterior's combined-variance term: each per-batch buffer
// (widest of M, N, n_b by the batch) within 2 GiB, at least 64 directions.
inline i64 posterior_dir_batch(i64 K, i64 widest) {
  return std::min<i64>(K, std::max<i64>(64, (2048LL << 20) / (8 * std::max<i64>(1, widest))));
}

// rocBLAS triangular products (blas.hip) on row-major matrices, T lower-triangular,
// C distinct from B: C = alpha T B (T m x m; B, C m x k) and C = alpha B T (B, C m x k; T k x k)
// (batch > 1: that many products, operands st, sb, sc elements apart)
hipError_t trmm_rows_left_lower(int m, int k, double alpha, const double* T, int ldt, const double* B, int ldb,
                                double* C, int ldc, hipStream_t s, int batch = 1, i64 st = 0, i64 sb = 0, i64 sc = 0);
hipError_t trmm_rows_right_lower(int m, int k, double alpha, const double* T, int ldt, const double* B, int ldb,
                                 double* C, int ldc, hipStream_t s, int batch = 1, i64 st = 0, i64 sb = 0,
                                 i64 sc = 0);
// C = A B^T, all row-major: A m x k, B n x k, C m x n
hipError_t trmm_vecs_lower(int n, int nrhs, int trans, const double* A, const double* X, double* Y, hipStream_t s);
hipError_t gemm_rows_abt(int m, int n, int k, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                         hipStream_t s);
// C -= A A^T on the lower triangle (C row-major n x n, A row-major n x k)
hipError_t syrk_rows_lower_sub(int n, int k, const double* A, int lda, double* C, int ldc, hipStream_t s);

// batched solve of problems sharing the handle's operator (solver.hip)
struct BatchResult {
  int iters = 0, state = 0;        // directions stored; 0 budget, 1 converged, 2 breakdown
  double rel_res = 0;
};
int batch_solve(gpfvm_handle* h, int R, const double* yobs_host, double tol, int max_iter, int check_every,
                int replace_every, hipStream_t s, std::vector<BatchResult>& out);
int batch_posterior(gpfvm_handle* h, int z, int dim, const int* n, const double* const* axis, double* mean,
                    double* var, hipStream_t s);
GemmDesc desc1(void* C, i64 c_rs, const void* A, i64 a_rs, i64 a_cs, const void* B, i64 b_rs, i64 b_cs, int M,
               int N, int K, double alpha, double beta, int tri);

}  // namespace gpfvm
