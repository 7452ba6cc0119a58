// rocBLAS for a plain library product of the path: the posterior's triangular
// product with many right-hand sides (TRMM), where the library kernels run at
// 82% of the float64 MFMA peak on the wave problem's 16384 x 2048 x 16384
// shape (the grouped Kronecker GEMM reaches 60% there).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <map>

#include "common.h"
#include "internal.h"

namespace gpfvm {

namespace {
// One rocBLAS handle per thread and device (handles are not shared between
// threads: the server's workers call the posterior concurrently).
struct BlasHandles {
  std::map<int, rocblas_handle> h;
  ~BlasHandles() {
    for (auto& kv : h) (void)rocblas_destroy_handle(kv.second);
  }
};
thread_local BlasHandles t_handles;

rocblas_handle handle_for(hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  rocblas_handle& hd = t_handles.h[dev];
  if (!hd && rocblas_create_handle(&hd) != rocblas_status_success) {
    hd = nullptr;
    return nullptr;
  }
  if (rocblas_set_stream(hd, s) != rocblas_status_success) return nullptr;
  return hd;
}
}  // namespace

// Row-major matrices are handed to rocBLAS as their column-major transposes:
// a row-major lower-triangular T (leading dimension ldt) is the column-major
// upper-triangular T^T, and a product with T on one side is a product with T^T
// on the other.

// C = alpha T B: T row-major m x m lower-triangular, B and C row-major m x k
// (C and B distinct).  batch > 1: that many products, the operands st, sb, sc
// elements apart.
hipError_t trmm_rows_left_lower(int m, int k, double alpha, const double* T, int ldt, const double* B, int ldb,
                                double* C, int ldc, hipStream_t s, int batch, i64 st, i64 sb, i64 sc) {
  rocblas_handle hd = handle_for(s);
  if (!hd) return hipErrorNotInitialized;
  const rocblas_status r =
      batch > 1 ? rocblas_dtrmm_strided_batched(hd, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                                                rocblas_diagonal_non_unit, k, m, &alpha, T, ldt, st, B, ldb, sb, C, ldc,
                                                sc, batch)
                : rocblas_dtrmm(hd, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                                rocblas_diagonal_non_unit, k, m, &alpha, T, ldt, B, ldb, C, ldc);
  return r == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure;
}

// C = alpha B T: B and C row-major m x k (distinct), T row-major k x k lower-triangular.
hipError_t trmm_rows_right_lower(int m, int k, double alpha, const double* T, int ldt, const double* B, int ldb,
                                 double* C, int ldc, hipStream_t s, int batch, i64 st, i64 sb, i64 sc) {
  rocblas_handle hd = handle_for(s);
  if (!hd) return hipErrorNotInitialized;
  const rocblas_status r =
      batch > 1 ? rocblas_dtrmm_strided_batched(hd, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                                                rocblas_diagonal_non_unit, k, m, &alpha, T, ldt, st, B, ldb, sb, C, ldc,
                                                sc, batch)
                : rocblas_dtrmm(hd, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                                rocblas_diagonal_non_unit, k, m, &alpha, T, ldt, B, ldb, C, ldc);
  return r == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure;
}

// Y[r] = A X[r] (trans = 0) or A^T X[r] (trans = 1) for nrhs vectors of length n stored one after
// another (X[r] at X + r n), A row-major n x n lower-triangular.  Column-major, the vectors are the
// columns of an n x nrhs matrix and A's storage is the upper-triangular A^T.
hipError_t trmm_vecs_lower(int n, int nrhs, int trans, const double* A, const double* X, double* Y, hipStream_t s) {
  rocblas_handle hd = handle_for(s);
  if (!hd) return hipErrorNotInitialized;
  const double one = 1.0;
  const rocblas_status st = rocblas_dtrmm(hd, rocblas_side_left, rocblas_fill_upper,
                                          trans ? rocblas_operation_none : rocblas_operation_transpose,
                                          rocblas_diagonal_non_unit, n, nrhs, &one, A, n, X, n, Y, n);
  return st == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure;
}

// C = A B^T for row-major A (m x k, leading dimension lda), B (n x k, ldb) and
// C (m x n, ldc).  In the column-major views (A^T, B^T, C^T) this is
// C^T = (B^T)^T A^T: a GEMM with the first operand transposed.
hipError_t gemm_rows_abt(int m, int n, int k, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                         hipStream_t s) {
  rocblas_handle hd = handle_for(s);
  if (!hd) return hipErrorNotInitialized;
  const double one = 1.0, zero = 0.0;
  const rocblas_status st = rocblas_dgemm(hd, rocblas_operation_transpose, rocblas_operation_none, n, m, k, &one, B,
                                          ldb, A, lda, &zero, C, ldc);
  return st == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure;
}

// C -= A A^T on the lower triangle: C row-major n x n (leading dimension ldc),
// A row-major n x k (leading dimension lda).  Column-major, C^T is upper and
// the update is (A^T)^T (A^T): an upper SYRK with the transposed operand.
hipError_t syrk_rows_lower_sub(int n, int k, const double* A, int lda, double* C, int ldc, hipStream_t s) {
  rocblas_handle hd = handle_for(s);
  if (!hd) return hipErrorNotInitialized;
  const double minus_one = -1.0, one = 1.0;
  const rocblas_status st = rocblas_dsyrk(hd, rocblas_fill_upper, rocblas_operation_transpose, n, k, &minus_one, A, lda,
                                          &one, C, ldc);
  return st == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure;
}

}  // namespace gpfvm
