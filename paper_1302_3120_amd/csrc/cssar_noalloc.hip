// Allocation-free iterative thresholding: cssar_ita_solve with its
// workspace in a fixed device array of the library, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops).
#include <mutex>

#include "cssar_internal.hpp"

using namespace cssar;
using namespace cssar::detail;

namespace {

// The solver's workspace for every call of cssar_ita_solve_static on a
// device.  Each device holds its own copy for the life of the process.  In
// host code this name stands for no device address: its address on a device
// comes from hipGetSymbolAddress with that device current (scratch_on).
constexpr size_t kScratchBytes = CSSAR_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of scratch on the current device (looked up once per
// device), or NULL with the error recorded.
void* scratch_on(int dev, int* rc) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (dev < 0 || dev >= kMaxDevices) {
    *rc = fail(CSSAR_EUNSUPPORTED, "device ordinal %d beyond %d", dev, kMaxDevices);
    return nullptr;
  }
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *rc = fail(CSSAR_EHIP, "hipGetSymbolAddress of the static workspace: %s", hipGetErrorString(e));
      return nullptr;
    }
    g_ptr[dev] = p;
  }
  *rc = CSSAR_OK;
  return g_ptr[dev];
}

}  // namespace

extern "C" {

int cssar_ita_solve_static(cssar_op* op, const void* y, const void* mask_bits, float lambda, int iters,
                           void* x_out, float* resid_hist, void* stream) {
  int rc = check_op(op);
  if (rc) return rc;
  const size_t need = cssar_workspace_size(op, 1);
  if (need > kScratchBytes)
    return fail(CSSAR_EINVAL,
                "a %d x %d solve needs %zu workspace bytes, beyond the %zu of the static workspace "
                "(use cssar_ita_solve with a workspace of cssar_workspace_size(op, 1) bytes)",
                op->na, op->nr, need, kScratchBytes);
  if (op->profiling) return fail(CSSAR_EINVAL, "per-launch timing creates events: disable it first");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(CSSAR_EHIP, "hipGetDevice failed");
  if (dev != op->device)
    return fail(CSSAR_EINVAL, "the current device (%d) is not the operator's (%d)", dev, op->device);
  void* ws = scratch_on(dev, &rc);
  if (!ws) return rc;
  // The solver writes every part of its workspace before reading it (the
  // first pass writes P and the marked copy of m o y; the first update pass
  // reads no iterate), so nothing is cleared between calls.
  return cssar_ita_solve(op, y, mask_bits, lambda, iters, x_out, resid_hist, ws, stream);
}

}  // extern "C"
