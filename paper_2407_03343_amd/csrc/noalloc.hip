// The block product with G_hat on library-held scratch memory, for callers
// that cannot allocate device memory (code under stream capture, serving
// loops, harnesses that forbid allocation).
//
// The scratch is one file-scope device array per GPU, resident until the
// process ends.  In host code its name is a host-side stand-in, not a device
// address, so its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// used afterwards.  Every call on a GPU shares the array: calls that overlap
// on one GPU (two streams, two threads) race on it.  The kernels of the
// product write every element they later read (strengths, Sigma^-1 U^T mu
// per sphere, partial sums), so nothing has to be cleared between calls.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/smfs.h"
#include "internal.h"

namespace smfs {
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // SMFS_NOALLOC_SCRATCH_BYTES
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up on the first call on
// each device; the current device is the caller's).
int scratch_ptr(void **out) {
  int dev = -1;
  SMFS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("smfs_apply_block_noalloc: device index out of range");
    return SMFS_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    SMFS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("smfs_apply_block_noalloc: no device address for the scratch array");
      return SMFS_E_DEVICE;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return SMFS_OK;
}

}  // namespace
}  // namespace smfs

using namespace smfs;

extern "C" {

size_t smfs_noalloc_scratch_bytes(void) { return kScratchBytes; }

int smfs_apply_block_noalloc(smfs_problem *pb, int32_t nrhs, const double *mu, double *y, int64_t ld,
                             smfs_stream stream) {
  SMFS_READY(pb);
  if (nrhs <= 0 || nrhs > 65535) { set_error("smfs_apply_block_noalloc: nrhs must be in [1, 65535]"); return SMFS_E_INVALID_ARG; }
  if (!mu || !y || ld < 3 * pb->T) { set_error("smfs_apply_block_noalloc: bad vectors"); return SMFS_E_INVALID_ARG; }
  const char *a0 = (const char *)mu, *a1 = a0 + 8 * (nrhs * ld);
  const char *b0 = (const char *)y, *b1 = b0 + 8 * (nrhs * ld);
  if (a0 < b1 && b0 < a1) { set_error("smfs_apply_block_noalloc: mu and y overlap"); return SMFS_E_INVALID_ARG; }
  const size_t need = block_apply_bytes(*pb, nrhs);
  if (need > kScratchBytes) {
    set_error("smfs_apply_block_noalloc: this problem and nrhs need " + std::to_string(need) +
              " bytes of scratch, above the library's fixed " + std::to_string(kScratchBytes) +
              "; use smfs_apply_block with a caller workspace");
    return SMFS_E_NOMEM;
  }
  void *base = nullptr;
  int rc = scratch_ptr(&base);
  if (rc) return rc;
  // no event recording here: the profiling pool may create events
  const bool prof = pb->prof;
  pb->prof = false;
  rc = block_apply_on(*pb, nrhs, mu, y, ld, (char *)base, (hipStream_t)stream);
  pb->prof = prof;
  return rc;
}

}  // extern "C"
