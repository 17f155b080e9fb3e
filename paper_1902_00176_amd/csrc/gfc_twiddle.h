// gfc_twiddle.h - per-lane twiddle factors of the four-step FFTs from a few table rows.
//
// The step between the two DFT stages multiplies lane j's value k by w^(k j) for k < K. Read
// one table row per k, those loads were about as many bytes through the texture data path
// as the data loads of the forward row pass, and that path is what bounds the row kernels
// (it is busier than for a plain device copy moving more bytes). So only the rows k < R and
// k = R q are read (R = ceil(sqrt(K))) and w^(k j) = w^(R q j) w^(r j) for k = R q + r is
// formed in registers: about 2 sqrt(K) loads instead of K - 1, for one more float32 complex
// rounding of the twiddle (the tables stay float64-built).
#pragma once
#include "gfc_buf.h"
#include "gfc_dft.h"

namespace gfc {

constexpr int isqrt_ceil(int n) {
  int r = 1;
  while (r * r < n) ++r;
  return r;
}

// apply(k, w^(k j)) for k = 1 .. K - 1; table row k starts at k * STRIDE complex entries,
// lane j reads entry j of a row. EXACT reads every row: for transforms whose rounding is
// amplified afterwards with no split of the lowest frequencies (a given divergence, volumes)
template <int K, int STRIDE, bool EXACT = false, class F>
__device__ __forceinline__ void twiddles(rsrc_t tw, int lane, int tz, F&& apply) {
  if constexpr (EXACT) {
#pragma unroll
    for (int k = 1; k < K; ++k) {
      const f2b w = bld2(tw, lane * 8, tz + k * STRIDE * 8);
      apply(k, cx{w.x, w.y});
    }
    return;
  }
  constexpr int R = isqrt_ceil(K);
  cx tr[R];
#pragma unroll
  for (int r = 1; r < R; ++r) {
    const f2b w = bld2(tw, lane * 8, tz + r * STRIDE * 8);
    tr[r] = {w.x, w.y};
  }
  cx tq = {1.f, 0.f};
#pragma unroll
  for (int k = 1; k < K; ++k) {
    const int q = k / R, r = k % R;
    if (r == 0) {
      const f2b w = bld2(tw, lane * 8, tz + k * STRIDE * 8);
      tq = {w.x, w.y};
      apply(k, tq);
    } else if (q == 0) {
      apply(k, tr[r]);
    } else {
      apply(k, cmul(tq, tr[r]));
    }
  }
}

}  // namespace gfc
