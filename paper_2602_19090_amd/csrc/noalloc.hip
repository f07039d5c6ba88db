// refine_eigvecs without any device allocation: the workspace is a file-scope device
// array, one copy per GPU, for callers that cannot allocate (graph capture, serving loops,
// harnesses that forbid hipMalloc).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/refeig.h"

namespace {

// Largest order served, and the array that holds its workspace (the default options at
// n = 1024 need 326 MiB: digit planes, INT32 slots, residue planes of A at four digit
// levels and of X^(1), X^(1) itself and the per-column vectors).
constexpr int kNoAllocMaxN = REFEIG_NOALLOC_MAX_N;
constexpr size_t kNoAllocBytes = 336ull << 20;

static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];   // device address of `scratch` on each GPU (host-side copy)

}  // namespace

extern "C" int refine_eigvecs_noalloc(const double *A, int lda, double *X, int ldx, double *D,
                                      int n, double target_fwd_err, const refeig_opts *o,
                                      refeig_stream_t stream, refeig_report *report) {
  if (n < 1 || n > kNoAllocMaxN) {
    fprintf(stderr, "refeig: refine_eigvecs_noalloc serves n <= %d (got %d)\n", kNoAllocMaxN, n);
    return REFEIG_E_NOMEM;
  }
  refeig_opts opts;
  if (o) opts = *o;
  else refeig_default_opts(&opts);
  // the FP64 plain form needs a BLAS handle (an allocation)
  if (opts.mode != REFEIG_OZAKI_INT8) return REFEIG_E_ARG;
  size_t need = 0;
  int st = refeig_workspace_bytes(n, &opts, &need);
  if (st != REFEIG_OK) return st;
  if (need > kNoAllocBytes) {
    fprintf(stderr, "refeig: refine_eigvecs_noalloc: n = %d needs %zu workspace bytes, the "
                    "static array holds %zu\n", n, need, kNoAllocBytes);
    return REFEIG_E_NOMEM;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return REFEIG_E_HIP;
  void *ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
      // the array's name is a host-side stand-in; its device address comes from the runtime
      void *p = nullptr;
      hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        fprintf(stderr, "refeig: hipGetSymbolAddress(scratch): %s\n", hipGetErrorString(e));
        return REFEIG_E_HIP;
      }
      g_ptr[dev] = p;
    }
    ptr = g_ptr[dev];
  }
  return refine_eigvecs(A, lda, X, ldx, D, n, target_fwd_err, &opts, ptr, kNoAllocBytes, stream,
                        report);
}
