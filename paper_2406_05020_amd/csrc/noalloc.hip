// The volume-Gram matvec without device allocation: every intermediate of the
// Kronecker plan and its GEMM descriptors live in one static device array of
// GPFVM_NOALLOC_SCRATCH_BYTES per GPU, so the call makes no hipMalloc/hipFree.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "common.h"
#include "internal.h"

using namespace gpfvm;

namespace {

// Device scratch of the allocation-free entry point.  In host code this name
// stands for the symbol only: its device address is taken once per device
// with hipGetSymbolAddress (each GPU holds its own copy until the process
// ends) and only that address is passed on.
static __device__ __align__(256) unsigned char scratch[GPFVM_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;     // device -> address of its copy of `scratch`

// Address of this device's scratch (resolved on the first call on the device).
hipError_t scratch_address(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = g_scratch_ptr.emplace(dev, (char*)p).first;
  }
  *out = it->second;
  return hipSuccess;
}

}  // namespace

extern "C" int gpfvm_volume_matvec_noalloc(gpfvm_handle* h, int nrhs, const double* x, double* y, void* stream) {
  if (!h) return GPFVM_E_INVALID;
  if (nrhs < 1 || nrhs > 4096 || !x || !y) { h->err = "volume_matvec_noalloc: bad nrhs or NULL buffer"; return GPFVM_E_INVALID; }
  const size_t bytes = (size_t)h->N * nrhs * sizeof(double);
  if ((const char*)x < (const char*)y + bytes && (const char*)y < (const char*)x + bytes) {
    h->err = "volume_matvec_noalloc: x and y overlap";
    return GPFVM_E_INVALID;
  }
  char* base = nullptr;
  const hipError_t e = scratch_address(&base);
  if (e != hipSuccess) { h->err = std::string("volume_matvec_noalloc: scratch address: ") + hipGetErrorString(e); return GPFVM_E_HIP; }
  hipStream_t s = (hipStream_t)stream;
  h->stream = s;
  // the caller's buffers join the plan's bounds check for the duration of the call
  register_range(x, bytes);
  register_range(y, bytes);
  Arena a;
  a.fixed = base;
  a.fixed_cap = GPFVM_NOALLOC_SCRATCH_BYTES;
  Plan pl;
  std::string err;
  int rc = compile_kron_list(h->op_pp, F64, nrhs, x, h->N, y, h->N, h->cellc, h->cellc, 0.0, x, h->sig_pde,
                             pp_accumulate(h), a, s, pl, err);
  if (rc == GPFVM_E_NOMEM) {
    rc = GPFVM_E_INVALID;
    err = "volume_matvec_noalloc: the plan for this problem and nrhs needs more than the " +
          std::to_string((long long)GPFVM_NOALLOC_SCRATCH_BYTES >> 20) + " MiB device scratch";
  }
  if (!rc && run_plan(pl, s) != hipSuccess) {
    rc = GPFVM_E_HIP;
    err = "volume_matvec_noalloc: launch failed";
  }
  a.release();
  unregister_range(x);
  unregister_range(y);
  if (rc) h->err = err;
  return rc;
}
