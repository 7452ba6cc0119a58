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

// C = A B for row-major A (n x n, lower-triangular, leading dimension n) and
// row-major B, C (n x nx, leading dimension nx).  In rocBLAS's column-major
// view these are C^T = B^T A^T with A^T upper-triangular, a right-side TRMM.
hipError_t trmm_lower_rows(int n, int nx, const double* A, const double* B, double* C, hipStream_t s) {
  rocblas_handle hd = handle_for(s);
  if (!hd) return hipErrorNotInitialized;
  const double one = 1.0;
  const rocblas_status st = rocblas_dtrmm(hd, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                                          rocblas_diagonal_non_unit, nx, n, &one, A, n, B, nx, C, nx);
  return st == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure;
}

}  // namespace gpfvm
