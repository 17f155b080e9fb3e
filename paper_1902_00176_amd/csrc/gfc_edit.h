// gfc_edit.h - on-device gradient edits of one pixel, shared by the row pass and the
// kernel that adds low row bins, so both see bit-identical edited gradients.
#pragma once
#include <hip/hip_runtime.h>

#include "gfc_internal.h"

namespace gfc {

// Gradient edits of one pixel (before the divergence). Threshold: the decision uses the
// same float32 rounding sequence as its specification (no contraction). GDM: the weighted
// geometric mean of eq. (26) through log2/exp2 in float32.
template <int EDIT>
__device__ __forceinline__ void edit_pixel(float& gx, float& gy, float c, float tau2,
                                           float alpha) {
  if constexpr (EDIT == kEditThreshold) {
    const float m = __fadd_rn(__fmul_rn(gx, gx), __fmul_rn(gy, gy));
    if (!(m >= tau2)) gx = gy = 0.f;
  } else if constexpr (EDIT == kEditGdm) {
    const float m = gx * gx + gy * gy;
    const float lc = alpha > 0.f ? alpha * log2f(c) : 0.f;  // C^alpha, with C^0 = 1
    const float sc = m > 0.f ? exp2f(lc - 0.5f * alpha * log2f(m)) : 0.f;
    gx *= sc;
    gy *= sc;
  }
}

}  // namespace gfc
