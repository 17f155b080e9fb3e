// gfc_buf.h - raw buffer loads and stores for gfx950.
//
// A buffer descriptor (four SGPRs) holds the base address and the byte range; each access
// takes a 32-bit per-lane byte offset (VGPR) and a uniform byte offset (SGPR). Rows that are
// far apart then cost one scalar add instead of a 64-bit address pair per lane, and an
// access past the range reads 0 / is dropped by the hardware.
#pragma once
#include <hip/hip_runtime.h>

namespace gfc {

using rsrc_t = __amdgpu_buffer_rsrc_t;

// descriptor word 3 for raw (untyped, stride 0) buffers on gfx9-family parts
constexpr int kBufWord3 = 0x00020000;

__device__ __forceinline__ rsrc_t make_buf(const void* base, long long bytes) {
  const int n = bytes > 0x7fffffffLL ? 0x7fffffff : int(bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, n, kBufWord3);
}

struct f2b {
  float x, y;
};

// Cache-policy operand of an access: 0 is the default; kNT marks it nontemporal (streamed
// through the caches with low retention). A pass that reads a block once and writes it
// once moves its bytes faster when both its loads and its stores carry kNT.
constexpr int kNT = 2;

template <int CP = 0>
__device__ __forceinline__ f2b bld2(rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(f2b, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, CP));
}
template <int CP = 0>
__device__ __forceinline__ float bld1(rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, CP));
}
template <int CP = 0>
__device__ __forceinline__ void bst2(rsrc_t r, float x, float y, int voff, int soff) {
  using v2u = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, f2b{x, y}), r, voff, soff, CP);
}
template <int CP = 0>
__device__ __forceinline__ void bst1(rsrc_t r, float x, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, voff, soff, CP);
}

// Lane t's part of a sum of n float64 values (the partial sums one pass leaves for the
// next): elements t, t + W, t + 2W, ... added in that order. A loop of single loads pays a
// memory latency per element; here U loads are in flight at a time, and elements past n
// read 0 through the buffer range (adding +0 changes no sum). Callers combine the lanes'
// parts in a fixed order.
template <int W, int U>
__device__ __forceinline__ double strided_sum(const double* p, int n, int t) {
  const rsrc_t r = make_buf(p, (long long)n * 8);
  double s = 0.0;
  for (int j0 = 0; j0 < n; j0 += U * W) {
    double v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) v[k] = __builtin_bit_cast(double, bld2(r, (j0 + t + W * k) * 8, 0));
#pragma unroll
    for (int k = 0; k < U; ++k) s += v[k];
  }
  return s;
}

}  // namespace gfc
