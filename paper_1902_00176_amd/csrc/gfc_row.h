// gfc_row.h - row passes of the GFC solve: length-N FFTs along the image rows.
//
// Each FFT of length N = N1 * N2 runs in a "slot" of G lanes (G = the power of two >= the
// larger factor; 64/G slots share a wavefront). Four-step split with one LDS transpose:
//   forward:  lane j holds z[N2*y1 + j] (y1 < N1) -> DFT_N1 -> twiddle w_N^(k1 j) -> LDS
//             lane k reads row k of the transpose -> DFT_N2 -> Z[k + N1*k2]
//   inverse:  lane k holds Z[k + N1*k2] -> IDFT_N2 -> twiddle w_N^-(k j2) -> LDS
//             lane j reads -> IDFT_N1 -> z[j + N2*j1]
// The small DFTs are register-resident (gfc_dft.h). Real-signal handling: two real
// sequences share one complex FFT (packing a + i b), separated by the mirror bins N - l
// through a second LDS pass in natural order.
#pragma once
#include "gfc_dft.h"
#include "gfc_internal.h"

namespace gfc {

constexpr int pow2ceil(int v) { return v <= 8 ? 8 : v <= 16 ? 16 : v <= 32 ? 32 : 64; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int N1, int N2>
struct RowCfg {
  static constexpr int N = N1 * N2;
  static constexpr int G = pow2ceil(cmax(N1, N2));
  static constexpr int SA = (N2 % 2 == 0) ? N2 + 1 : N2;  // odd LDS stride, forward transpose
  static constexpr int SB = (N1 % 2 == 0) ? N1 + 1 : N1;  // odd LDS stride, inverse transpose
  static constexpr int LDSC = cmax(cmax(N1 * SA, N2 * SB), N);  // floats per plane per slot
  static constexpr int NH = N / 2 + 1;
  static constexpr int NI = (NH + G - 1) / G;  // half-spectrum bins owned per lane
  static_assert(N1 <= 64 && N2 <= 64, "row factors must fit one wavefront");
};

__device__ __forceinline__ cx ld2(const f2* p) {
  const f2 v = *p;
  return {v.x, v.y};
}
__device__ __forceinline__ void st2(f2* p, cx v) { *p = f2{v.x, v.y}; }

// Forward four-step body. On entry lane j < N2 holds a[y1] = z[N2*y1 + j]; on exit the
// spectrum Z is in LDS (re/im planes) in natural order.
template <int N1, int N2>
__device__ __forceinline__ void fwd_fft_to_lds(cx (&a)[N1], float* re, float* im, int lane,
                                               const f2* __restrict__ twA) {
  using C = RowCfg<N1, N2>;
  if (lane < N2) {
    Dft<N1, -1>::run(a);
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) a[k1] = cmul(a[k1], ld2(twA + k1 * N2 + lane));
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      re[k1 * C::SA + lane] = a[k1].x;
      im[k1 * C::SA + lane] = a[k1].y;
    }
  }
  __syncthreads();
  cx b[N2];
  if (lane < N1) {
#pragma unroll
    for (int j = 0; j < N2; ++j) b[j] = {re[lane * C::SA + j], im[lane * C::SA + j]};
    Dft<N2, -1>::run(b);
  }
  __syncthreads();
  if (lane < N1) {
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      re[lane + N1 * k2] = b[k2].x;
      im[lane + N1 * k2] = b[k2].y;
    }
  }
  __syncthreads();
}

// Inverse four-step body. On entry lane k < N1 holds b[k2] = Z[k + N1*k2]; on exit lane
// j < N2 holds a[j1] = z[j + N2*j1] (unnormalised inverse DFT).
template <int N1, int N2>
__device__ __forceinline__ void inv_fft_from_regs(cx (&b)[N2], cx (&a)[N1], float* re,
                                                  float* im, int lane,
                                                  const f2* __restrict__ twB) {
  using C = RowCfg<N1, N2>;
  if (lane < N1) {
    Dft<N2, +1>::run(b);
#pragma unroll
    for (int j2 = 1; j2 < N2; ++j2) b[j2] = cmulconj(b[j2], ld2(twB + j2 * N1 + lane));
#pragma unroll
    for (int j2 = 0; j2 < N2; ++j2) {
      re[j2 * C::SB + lane] = b[j2].x;
      im[j2 * C::SB + lane] = b[j2].y;
    }
  }
  __syncthreads();
  if (lane < N2) {
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) a[k1] = {re[lane * C::SB + k1], im[lane * C::SB + k1]};
    Dft<N1, +1>::run(a);
  }
}

// ---------------------------------------------------------------------------------------
// Forward row pass (divergence + row R2C, eq. (3) and the row half of F(L) in eq. (23)).
// Rows of the block are processed in strips so the previous row's Ey^ stays in registers.
template <int N1, int N2, int SLOTS>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
k_row_fwd(RowFwdArgs p) {
  using C = RowCfg<N1, N2>;
  __shared__ float s_re[SLOTS][C::LDSC];
  __shared__ float s_im[SLOTS][C::LDSC];
  const int slot = threadIdx.x / C::G;
  const int lane = threadIdx.x % C::G;
  float* re = s_re[slot];
  float* im = s_im[slot];
  const int b = blockIdx.y;
  const int strip = blockIdx.x * SLOTS + slot;
  const bool strip_ok = strip < p.nstrips;
  const int y0 = strip * p.strip;
  const float* __restrict__ gx = p.gx + b * p.img_in;
  const float* __restrict__ gy = p.gy + b * p.img_in;
  f2* __restrict__ T1 = p.T1 + b * p.img_t1;
  f2* __restrict__ SBo = p.SB + b * p.img_sb;
  const int K1 = p.K + 1;

  cx prev[C::NI];
#pragma unroll
  for (int i = 0; i < C::NI; ++i) prev[i] = {0.f, 0.f};

  for (int it = 0; it <= p.strip; ++it) {
    const int y = y0 - 1 + it;
    const bool row_in = strip_ok && y >= 0 && y < p.H;
    cx a[N1];
    if (lane < N2) {
#pragma unroll
      for (int y1 = 0; y1 < N1; ++y1) {
        const int x = N2 * y1 + lane;
        if (row_in && x < p.W) {
          a[y1] = {gx[(long long)y * p.W + x], gy[(long long)y * p.W + x]};
        } else {
          a[y1] = {0.f, 0.f};
        }
      }
    }
    fwd_fft_to_lds<N1, N2>(a, re, im, lane, p.twA);
    const bool emit = strip_ok && it > 0 && y <= p.H;
#pragma unroll
    for (int i = 0; i < C::NI; ++i) {
      const int l = lane + C::G * i;
      if (l < C::NH) {
        const int m = (l == 0) ? 0 : C::N - l;
        const float ar = re[l], ai = im[l], br = re[m], bi = im[m];
        const cx ex = {0.5f * (ar + br), 0.5f * (ai - bi)};
        const cx ey = {0.5f * (ai + bi), 0.5f * (br - ar)};
        if (emit) {
          cx t = cmul(ld2(p.sx + l), ex);
          if (l > p.K) {
            t = cadd(t, csub(ey, prev[i]));
          } else if (y < p.H) {
            st2(SBo + (long long)y * K1 + l, ey);
          }
          st2(T1 + (long long)y * C::NH + l, t);
        }
        prev[i] = ey;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// Inverse row pass (row C2R of eq. (23), real part, crop and Algorithm B's constant).
template <int N1, int N2, int SLOTS>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
k_row_inv(RowInvArgs p) {
  using C = RowCfg<N1, N2>;
  __shared__ float s_re[SLOTS][C::LDSC];
  __shared__ float s_im[SLOTS][C::LDSC];
  const int slot = threadIdx.x / C::G;
  const int lane = threadIdx.x % C::G;
  float* re = s_re[slot];
  float* im = s_im[slot];
  const int b = blockIdx.y;
  const int q = blockIdx.x * SLOTS + slot;
  const bool ok = q < p.npairs;
  const int y1 = 2 * q, y2 = 2 * q + 1;
  const bool has2 = ok && y2 < p.H;
  const f2* __restrict__ T2 = p.T2 + b * p.img_t2;
  float* __restrict__ u = p.u + b * p.img_u;

  double vr = 0.0;
  for (int j = 0; j < p.nparts; ++j) vr += p.partial[(long long)b * p.nparts + j];
  const float vref = float(vr);

  cx bz[N2];
  if (lane < N1) {
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int kk = lane + N1 * k2;
      cx X1 = {0.f, 0.f}, X2 = {0.f, 0.f};
      const int m = kk < C::NH ? kk : C::N - kk;
      if (ok) X1 = ld2(T2 + (long long)y1 * C::NH + m);
      if (has2) X2 = ld2(T2 + (long long)y2 * C::NH + m);
      if (kk < C::NH) bz[k2] = {X1.x - X2.y, X1.y + X2.x};
      else bz[k2] = {X1.x + X2.y, X2.x - X1.y};
    }
  }
  cx a[N1];
  inv_fft_from_regs<N1, N2>(bz, a, re, im, lane, p.twB);
  if (lane < N2 && ok) {
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) {
      const int x = lane + N2 * j1;
      if (x < p.W) {
        u[(long long)y1 * p.W + x] = a[j1].x - vref;
        if (has2) u[(long long)y2 * p.W + x] = a[j1].y - vref;
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// Backward row pass 1: row R2C of du (two rows per complex FFT) and partial sums of du.
template <int N1, int N2, int SLOTS>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
k_row_bfwd(RowBwdFwdArgs p) {
  using C = RowCfg<N1, N2>;
  __shared__ float s_re[SLOTS][C::LDSC];
  __shared__ float s_im[SLOTS][C::LDSC];
  __shared__ double s_sum[SLOTS * C::G];
  const int slot = threadIdx.x / C::G;
  const int lane = threadIdx.x % C::G;
  float* re = s_re[slot];
  float* im = s_im[slot];
  const int b = blockIdx.y;
  const int q = blockIdx.x * SLOTS + slot;
  const bool ok = q < p.npairs;
  const int y1 = 2 * q, y2 = 2 * q + 1;
  const bool has2 = ok && y2 < p.H;
  const float* __restrict__ du = p.du + b * p.img_in;
  f2* __restrict__ U = p.U + b * p.img_u;

  cx a[N1];
  float lsum = 0.f;
  if (lane < N2) {
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) {
      const int x = N2 * j1 + lane;
      float r = 0.f, s = 0.f;
      if (ok && x < p.W) r = du[(long long)y1 * p.W + x];
      if (has2 && x < p.W) s = du[(long long)y2 * p.W + x];
      a[j1] = {r, s};
      lsum += r + s;
    }
  }
  s_sum[threadIdx.x] = double(lsum);
  fwd_fft_to_lds<N1, N2>(a, re, im, lane, p.twA);
  if (ok) {
#pragma unroll
    for (int i = 0; i < C::NI; ++i) {
      const int l = lane + C::G * i;
      if (l < C::NH) {
        const int m = (l == 0) ? 0 : C::N - l;
        const float ar = re[l], ai = im[l], br = re[m], bi = im[m];
        st2(U + (long long)y1 * C::NH + l, cx{0.5f * (ar + br), 0.5f * (ai - bi)});
        if (has2) st2(U + (long long)y2 * C::NH + l, cx{0.5f * (ai + bi), 0.5f * (br - ar)});
      }
    }
  }
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < SLOTS * C::G; ++i) t += s_sum[i];
    p.sums[(long long)b * gridDim.x + blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------------------
// Backward row pass 2: apply -D_x as its symbol, -D_y from the column pass (low columns) or
// as a row difference (other columns), and one complex C2R per row for (dgx, dgy).
template <int N1, int N2, int SLOTS>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
k_row_binv(RowBwdInvArgs p) {
  using C = RowCfg<N1, N2>;
  __shared__ float s_re[SLOTS][C::LDSC];
  __shared__ float s_im[SLOTS][C::LDSC];
  const int slot = threadIdx.x / C::G;
  const int lane = threadIdx.x % C::G;
  float* re = s_re[slot];
  float* im = s_im[slot];
  const int b = blockIdx.y;
  const int strip = blockIdx.x * SLOTS + slot;
  const bool strip_ok = strip < p.nstrips;
  const int y0 = strip * p.strip;
  const f2* __restrict__ Wv = p.Wv + b * p.img_w;
  const f2* __restrict__ SD = p.SD + b * p.img_sd;
  float* __restrict__ gxo = p.dgx + b * p.img_out;
  float* __restrict__ gyo = p.dgy + b * p.img_out;
  const int Kb1 = p.Kb + 1;

  cx cur[C::NI];
#pragma unroll
  for (int i = 0; i < C::NI; ++i) {
    const int l = lane + C::G * i;
    cur[i] = {0.f, 0.f};
    if (strip_ok && l < C::NH && y0 < p.H) cur[i] = ld2(Wv + (long long)y0 * C::NH + l);
  }
  for (int it = 0; it < p.strip; ++it) {
    const int y = y0 + it;
    const bool row_ok = strip_ok && y < p.H;
#pragma unroll
    for (int i = 0; i < C::NI; ++i) {
      const int l = lane + C::G * i;
      if (l < C::NH) {
        cx nxt = {0.f, 0.f};
        if (row_ok) nxt = ld2(Wv + (long long)(y + 1) * C::NH + l);
        const cx X1 = cmul(ld2(p.sxm + l), cur[i]);
        cx X2;
        if (l <= p.Kb) {
          X2 = row_ok ? ld2(SD + (long long)y * Kb1 + l) : cx{0.f, 0.f};
        } else {
          X2 = csub(cur[i], nxt);
        }
        // full spectrum of dgx + i dgy at bins l and N - l
        re[l] = X1.x - X2.y;
        im[l] = X1.y + X2.x;
        if (l != 0 && 2 * l != C::N) {
          re[C::N - l] = X1.x + X2.y;
          im[C::N - l] = X2.x - X1.y;
        }
        cur[i] = nxt;
      }
    }
    __syncthreads();
    cx bz[N2];
    if (lane < N1) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) bz[k2] = {re[lane + N1 * k2], im[lane + N1 * k2]};
    }
    __syncthreads();
    cx a[N1];
    inv_fft_from_regs<N1, N2>(bz, a, re, im, lane, p.twB);
    if (lane < N2 && row_ok) {
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) {
        const int x = lane + N2 * j1;
        if (x < p.W) {
          gxo[(long long)y * p.W + x] = a[j1].x;
          gyo[(long long)y * p.W + x] = a[j1].y;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// launchers and the table of compiled lengths

template <int N1, int N2>
struct RowLaunch {
  using C = RowCfg<N1, N2>;
  static constexpr int SLOTS = (C::G == 64) ? 4 : (256 / C::G);
  static hipError_t fwd(const RowFwdArgs& a, int B, hipStream_t s) {
    dim3 grid((a.nstrips + SLOTS - 1) / SLOTS, B);
    hipLaunchKernelGGL((k_row_fwd<N1, N2, SLOTS>), grid, dim3(SLOTS * C::G), 0, s, a);
    return hipGetLastError();
  }
  static hipError_t inv(const RowInvArgs& a, int B, hipStream_t s) {
    dim3 grid((a.npairs + SLOTS - 1) / SLOTS, B);
    hipLaunchKernelGGL((k_row_inv<N1, N2, SLOTS>), grid, dim3(SLOTS * C::G), 0, s, a);
    return hipGetLastError();
  }
  static hipError_t bfwd(const RowBwdFwdArgs& a, int B, hipStream_t s) {
    dim3 grid((a.npairs + SLOTS - 1) / SLOTS, B);
    hipLaunchKernelGGL((k_row_bfwd<N1, N2, SLOTS>), grid, dim3(SLOTS * C::G), 0, s, a);
    return hipGetLastError();
  }
  static hipError_t binv(const RowBwdInvArgs& a, int B, hipStream_t s) {
    dim3 grid((a.nstrips + SLOTS - 1) / SLOTS, B);
    hipLaunchKernelGGL((k_row_binv<N1, N2, SLOTS>), grid, dim3(SLOTS * C::G), 0, s, a);
    return hipGetLastError();
  }
};

#define GFC_ROW_ENTRY(n1, n2)                                                               \
  RowKernels{n1 * n2, n1, n2, RowCfg<n1, n2>::G, RowLaunch<n1, n2>::SLOTS,                   \
             &RowLaunch<n1, n2>::fwd, &RowLaunch<n1, n2>::inv, &RowLaunch<n1, n2>::bfwd,     \
             &RowLaunch<n1, n2>::binv}

}  // namespace gfc
