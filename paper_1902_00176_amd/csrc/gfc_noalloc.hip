// gfc_noalloc.hip - a forward solve that allocates nothing.
//
// gfc_solve_batch takes its workspace (the half spectra between the passes, the split side
// arrays, the column partial sums) from the caller. Callers that cannot allocate device
// memory at all (code under graph capture, tight serving loops, harnesses that forbid it)
// use gfc_solve_batch_noalloc instead: the same kernels, with that workspace in a fixed
// file-scope device array of this library. Each GPU the library runs on holds one copy of the
// array until the process ends. Every call on a GPU shares that GPU's copy, so calls that may
// overlap on one GPU (other streams, other threads) race on it; calls in order on one
// stream do not. No kernel of the solve expects the workspace to start at any value.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gfc.h"
#include "gfc_internal.h"
#include "gfc_plan.h"

using namespace gfc;

constexpr size_t kScratchBytes = size_t(GFC_NOALLOC_SCRATCH_BYTES);
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

// The fixed workspace. In host code this name is only a stand-in for the symbol: kernels and
// copies must be given the device address hipGetSymbolAddress returns for the current GPU.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mtx;
void* g_ptr[kMaxDevices] = {};  // device address of `scratch` on each GPU, once looked up

// The address of this GPU's copy of the array, looked up once per device with that device
// current (each GPU holds its own copy at its own address).
gfc_status scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return GFC_E_HIP;
  if (dev >= kMaxDevices) return GFC_E_ARG;
  std::lock_guard<std::mutex> lk(g_mtx);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GFC_E_HIP;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return GFC_OK;
}

}  // namespace

extern "C" gfc_status gfc_solve_batch_noalloc(gfc_plan_t p, const float* gx, const float* gy,
                                              float* u, int B, void* stream) {
  if (!p || B < 0) return GFC_E_ARG;
  if (!p->built) return GFC_E_NOT_BUILT;
  if (B == 0) return GFC_OK;
  if (!gx || !gy || !u) return GFC_E_ARG;
  // the whole workspace of this call must fit the fixed array
  if (ws_layout(p, B).total > kScratchBytes) return GFC_E_WORKSPACE;
  void* ws = nullptr;
  const gfc_status st = scratch_ptr(&ws);
  if (st != GFC_OK) return st;
  return gfc_solve_batch(p, gx, gy, u, B, ws, kScratchBytes, stream);
}
