// gfc_edit.h - on-device gradient edits of one pixel, shared by the row pass and the
// kernel that adds low row bins, so both see bit-identical edited gradients.
#pragma once
#include <hip/hip_runtime.h>

#include "gfc_internal.h"

namespace gfc {

// Gradient edits of one pixel (before the divergence). Threshold: the decision uses the
// same float32 rounding sequence as its specification (no contraction). GDM: eq. (26)'s
// weighted geometric mean as a scale of E, |E|^(1-alpha) C^alpha / |E| =
// 2^(alpha (log2 C - log2 m / 2)) with m = |E|^2, in float32. Each log2 is the exponent plus
// the hardware log2 of the mantissa in [0.5, 1) (frexp), which needs no range scaling for
// subnormal C or m; the hardware exp2 flushes a scale below the normal range to zero (a
// pixel shrunk below 2^-126 of its size). C = 0 gives 0, C < 0 or NaN gives NaN (C^alpha),
// alpha = 0 leaves E unchanged (C^0 = 1) and E = 0 stays 0.
template <int EDIT>
__device__ __forceinline__ void edit_pixel(float& gx, float& gy, float c, float tau2,
                                           float alpha) {
  if constexpr (EDIT == kEditThreshold) {
    const float m = __fadd_rn(__fmul_rn(gx, gx), __fmul_rn(gy, gy));
    if (!(m >= tau2)) gx = gy = 0.f;
  } else if constexpr (EDIT == kEditGdm) {
    const float m = gx * gx + gy * gy;
    const float lm = float(__builtin_amdgcn_frexp_expf(m)) +
                     __builtin_amdgcn_logf(__builtin_amdgcn_frexp_mantf(m));
    const float lc = float(__builtin_amdgcn_frexp_expf(c)) +
                     __builtin_amdgcn_logf(__builtin_amdgcn_frexp_mantf(c));
    const float e = __builtin_amdgcn_exp2f(alpha * (lc - 0.5f * lm));
    const float sc = m > 0.f ? (alpha > 0.f ? e : 1.f) : 0.f;
    gx *= sc;
    gy *= sc;
  }
}

}  // namespace gfc
