// Allocation-free variant of omp_solve (omp_solve_noalloc): the solve's
// workspace is a file-scope device array instead of caller memory, for
// callers that cannot allocate device memory.
//
// Each GPU the library runs on holds its own copy of `scratch` (of
// OMP_NOALLOC_SCRATCH_BYTES) until the process ends. Host code never passes
// the array's name to a kernel: in host code that name is only a stand-in for
// the symbol. Its device address is looked up once per device, with that device
// current, and that address is what the solve's kernels receive. The solve's
// initialisation kernel writes every part of the workspace the later kernels
// read, so nothing in the array has to be cleared between calls; calls that
// overlap on one GPU share the array and race.

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/batched_omp.h"
#include "omp_internal.h"

namespace bomp {
namespace {

static __device__ __align__(256) unsigned char scratch[OMP_NOALLOC_SCRATCH_BYTES];

// Device address of this device's `scratch` (looked up on the first call on
// each device and kept).
int scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_error(e);
  static std::mutex mu;
  static std::vector<void *> addr;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return device_error(e);
    if (!p) return device_error(hipErrorInvalidSymbol);
    addr[dev] = p;
  }
  *out = addr[dev];
  return OMP_OK;
}

}  // namespace
}  // namespace bomp

using namespace bomp;

extern "C" {

int omp_solve_noalloc(const float *A, int64_t M, int64_t N, int64_t lda, const float *Y, int64_t B, int64_t ldy,
                      int32_t S, float eps, float *X_out, int32_t *support_out, const omp_opts_t *opts,
                      void *stream) {
  if (!opts || opts->phase_ms || opts->phase_launches) return OMP_EINVAL;
  const size_t need = solve_bytes(M, N, B, S, opts);
  if (need == 0) return OMP_EINVAL;
  if (need > (size_t)OMP_NOALLOC_SCRATCH_BYTES) return OMP_ENOTSUPP;
  int rc = check_device();
  if (rc != OMP_OK) return rc;
  void *ws = nullptr;
  rc = scratch_address(&ws);
  if (rc != OMP_OK) return rc;
  return solve_impl(A, M, N, lda, Y, B, ldy, S, eps, X_out, support_out, opts, stream, ws,
                    (size_t)OMP_NOALLOC_SCRATCH_BYTES, true);
}

size_t omp_noalloc_max_bytes(void) { return (size_t)OMP_NOALLOC_SCRATCH_BYTES; }

}  // extern "C"
