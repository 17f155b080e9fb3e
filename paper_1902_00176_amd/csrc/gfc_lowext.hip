// gfc_lowext.hip - more row bins in split form for thin, wide images.
//
// The column pass amplifies a rounding error in row bin l of the divergence spectrum by up
// to 1/lambda_l ~ (N / (2 pi l))^2 at column frequency 0 (Sec. 3, eq. (23)). The row pass
// therefore hands the lowest bins l <= kLowBins over in the split form (1 - w_N^l) Ex^ and
// Ey^, whose rounding is not amplified that way. When the torus has few rows (M small) the
// column frequency 0 carries a large share of the solution and the bins just above
// kLowBins still cost precision, so such plans split up to K bins: this kernel overwrites
// T1[y, l] and SB[y, l] for kLowBins < l <= K with the split values
//   T1[y, l] = (1 - w_N^l) sum_x Ex[y, x] w_N^(l x)   (y <= H; row H of Ex is 0)
//   SB[y, l] = sum_x Ey[y, x] w_N^(l x)               (y < H)
// as float32 direct sums. Workgroup: one row y, kExtWaves wavefronts of kExtBins bins each;
// lane j takes x = j, j + 64, ... and the 64 lane sums are added through LDS.
#include <hip/hip_runtime.h>

#include "gfc_buf.h"
#include "gfc_edit.h"
#include "gfc_internal.h"

namespace gfc {
namespace {

constexpr int kExtBins = 4;   // bins per wavefront
constexpr int kExtWaves = 4;  // wavefronts per workgroup
constexpr int kExtVals = 4 * kExtBins;  // floats per lane: (Ex, Ey) x (re, im) per bin

struct cxf {
  float x, y;
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One row y of one image; grp selects kExtWaves * kExtBins consecutive bins.
template <int EDIT>
__device__ __forceinline__ void low_ext_row(const RowFwdArgs& p, int y, int grp) {
  __shared__ float s_sum[kExtWaves][kExtVals][65];
  const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
  const int lb = kLowBins + 1 + (grp * kExtWaves + wave) * kExtBins;  // first bin of the wave
  if (lb > p.K) return;  // the waves of a workgroup never wait for each other
  cxf ax[kExtBins], ay[kExtBins];
  int m[kExtBins], d[kExtBins];
#pragma unroll
  for (int i = 0; i < kExtBins; ++i) {
    const int l = lb + i;
    ax[i] = ay[i] = {0.f, 0.f};
    m[i] = (l * lane) % p.N;  // exponent l x mod N for x = lane
    d[i] = (l * 64) % p.N;    // its step from x to x + 64
  }
  if (y < p.H) {
    const float* gx = p.gx + (long long)y * p.W;
    const float* gy = p.gy + (long long)y * p.W;
    const float* gc = EDIT == kEditGdm ? p.C + (long long)y * p.W : nullptr;
    for (int x = lane; x < p.W; x += 64) {
      float vx = gx[x], vy = gy[x];
      if constexpr (EDIT != kEditNone)
        edit_pixel<EDIT>(vx, vy, EDIT == kEditGdm ? gc[x] : 0.f, p.tau2, p.alpha);
#pragma unroll
      for (int i = 0; i < kExtBins; ++i) {
        const f2 w = p.twX[m[i]];
        ax[i].x = __builtin_fmaf(vx, w.x, ax[i].x);
        ax[i].y = __builtin_fmaf(vx, w.y, ax[i].y);
        ay[i].x = __builtin_fmaf(vy, w.x, ay[i].x);
        ay[i].y = __builtin_fmaf(vy, w.y, ay[i].y);
        m[i] += d[i];
        if (m[i] >= p.N) m[i] -= p.N;
      }
    }
  }
  // Ex bins times 1 - w_N^l (float64-built), then the sums over the lanes
  float* s = &s_sum[wave][0][0];
#pragma unroll
  for (int i = 0; i < kExtBins; ++i) {
    const int l = lb + i <= kMaxLowBins ? lb + i : 0;
    const f2 o = p.twX[p.N + l];
    s[(4 * i + 0) * 65 + lane] = ax[i].x * o.x - ax[i].y * o.y;
    s[(4 * i + 1) * 65 + lane] = ax[i].x * o.y + ax[i].y * o.x;
    s[(4 * i + 2) * 65 + lane] = ay[i].x;
    s[(4 * i + 3) * 65 + lane] = ay[i].y;
  }
  wave_sync();
  if (lane < kExtVals) {
    float sum = 0.f;
    for (int j = 0; j < 64; ++j) sum += s[lane * 65 + j];
    const int i = lane / 4, comp = lane & 1;
    const int l = lb + i;
    if (l <= p.K) {
      float* t1 = reinterpret_cast<float*>(p.T1);
      float* sb = reinterpret_cast<float*>(p.SB);
      if ((lane & 2) == 0)
        t1[2 * (long long)tile_index(y, l, p.H + 1) + comp] = sum;  // tile-major T1
      else if (y < p.H)
        sb[2 * ((long long)y * p.KP + l) + comp] = sum;
    }
  }
}

template <int EDIT>
__global__ void __launch_bounds__(64 * kExtWaves) k_low_ext(RowFwdArgs p) {
  const long long b = blockIdx.z;
  p.gx += b * p.img_in;
  p.gy += b * p.img_in;
  if (EDIT == kEditGdm) p.C += b * p.img_in;
  p.T1 += b * p.img_t1;
  p.SB += b * p.img_sb;
  low_ext_row<EDIT>(p, int(blockIdx.x), int(blockIdx.y));
}

__global__ void __launch_bounds__(64 * kExtWaves)
k_low_ext_rg(const RgBase* basep, const RgRowFwd* tab, const RgItem* items) {
  const RgBase base = *basep;  // written by launch_set_base on this stream
  const RgItem it = items[blockIdx.x];
  const RgRowFwd& e = tab[it.img];
  RowFwdArgs p = e.a;
  p.gx = base.gx + e.in;
  p.gy = base.gy + e.in;
  p.T1 = reinterpret_cast<f2*>(base.ws + e.t);
  p.SB = reinterpret_cast<f2*>(base.ws + e.side);
  low_ext_row<kEditNone>(p, it.blk, int(blockIdx.y));
}

constexpr int kBinsPerGroup = kExtWaves * kExtBins;
constexpr int kMaxGroups = (kMaxLowBins - kLowBins + kBinsPerGroup - 1) / kBinsPerGroup;

}  // namespace

hipError_t launch_low_ext(const RowFwdArgs& a, int B, hipStream_t s) {
  if (a.K <= kLowBins || B <= 0) return hipSuccess;
  if (a.K > kMaxLowBins || 2 * a.K >= a.N || !a.twX || !a.gx || !a.gy ||
      (a.edit == kEditGdm && !a.C) || B > 65535)
    return hipErrorInvalidValue;
  const dim3 grid(unsigned(a.H + 1), unsigned((a.K - kLowBins + kBinsPerGroup - 1) / kBinsPerGroup),
                  unsigned(B));
  const dim3 block(64 * kExtWaves);
  switch (a.edit) {
    case kEditNone: k_low_ext<kEditNone><<<grid, block, 0, s>>>(a); break;
    case kEditThreshold: k_low_ext<kEditThreshold><<<grid, block, 0, s>>>(a); break;
    case kEditGdm: k_low_ext<kEditGdm><<<grid, block, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_low_ext_rg(const RgBase* base, const RgRowFwd* tab, const RgItem* items,
                             int nitems, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  // every image of the list has K <= kMaxLowBins; groups past an image's K return at once
  k_low_ext_rg<<<dim3(unsigned(nitems), unsigned(kMaxGroups)), dim3(64 * kExtWaves), 0, s>>>(
      base, tab, items);
  return hipGetLastError();
}

}  // namespace gfc

// ---------------------------------------------------------------------------------------
// A given Laplacian (Algorithm B's input): its lowest row bins in the split form a + (1 - S) b
// of the column pass. b[y, l] = P[y, l] for y < H, a[y, l] = 0 for y < H, a[H, l] = P[H, l],
// where P[y, l] = sum_{y' <= y} L^[y', l]: then a + (1 - S) b is L^ on every row, and the
// sum over the rows (the column frequency 0, which the Green's function amplifies most) is
// the one value P[H, l] instead of a difference of rounded values. An FFT of L in float32
// leaves an error of the size of |L| in these bins, where the true values nearly cancel.
namespace gfc {
namespace {

constexpr int kLapWaves = 4;  // rows per workgroup of k_lap_rows, one per wavefront
constexpr int kLapBins = 5;   // bins summed per sweep over a row (K = 4: one sweep)
constexpr int kLapChunk = 8;   // elements per lane loaded together in a sweep

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// L^[y, l] for l <= K of one row per wavefront: lane j takes x_k = j + 64 k, and its part
// is w^(l j) sum_k v_k z^k with z = w^(64 l) (w = w_N, forward sign). The sum over k runs as
// Goertzel's second-order recurrence in float64, s_k = v_k + 2 Re(z) s_(k-1) - s_(k-2), whose
// end gives sum_k v_k conj(z)^(n-1-k) = s_(n-1) - z s_(n-2); times z^(n-1) w^(l j), one table
// entry, that is the lane's part (two operations per element and bin, where rotating the
// twiddle took ten). The lane's elements are loaded kLapChunk at a time, all in flight
// together; past x = W they read 0, which the count n of processed elements includes.
__global__ void __launch_bounds__(64 * kLapWaves) k_lap_rows(LapLowArgs a) {
  const int lane = int(threadIdx.x) & 63;
  const int y = int(blockIdx.x) * kLapWaves + (int(threadIdx.x) >> 6);
  const int b = blockIdx.y;
  if (y > a.H) return;  // no workgroup barrier below
  const float* row = a.L + b * a.img_L + (long long)y * (a.W + 1);
  const rsrc_t rrow = make_buf(row, (long long)(a.W + 1) * 4);
  double* out = a.Lh + b * a.img_lh + (long long)y * (a.K + 1) * 2;
  for (int l0 = 0; l0 <= a.K; l0 += kLapBins) {
    double c2[kLapBins], s1[kLapBins], s2[kLapBins];
#pragma unroll
    for (int i = 0; i < kLapBins; ++i) {
      const int l = l0 + i <= a.K ? l0 + i : 0;
      c2[i] = 2.0 * a.twD[2 * int((long long)l * 64 % a.N)];
      s1[i] = s2[i] = 0.0;
    }
    int n = 0;  // elements processed per lane (the same on every lane)
    for (int x0 = lane; x0 - lane <= a.W; x0 += 64 * kLapChunk) {
      float vc[kLapChunk];
#pragma unroll
      for (int k = 0; k < kLapChunk; ++k) vc[k] = bld1(rrow, (x0 + 64 * k) * 4, 0);
#pragma unroll
      for (int k = 0; k < kLapChunk; ++k) {
#pragma unroll
        for (int i = 0; i < kLapBins; ++i) {
          const double s0 = __builtin_fma(c2[i], s1[i], double(vc[k]) - s2[i]);
          s2[i] = s1[i];
          s1[i] = s0;
        }
      }
      n += kLapChunk;
    }
#pragma unroll
    for (int i = 0; i < kLapBins; ++i) {
      const int l = l0 + i <= a.K ? l0 + i : 0;
      const int d = int((long long)l * 64 % a.N);
      const double zr = a.twD[2 * d], zi = a.twD[2 * d + 1];
      const double qr = __builtin_fma(-zr, s2[i], s1[i]), qi = -zi * s2[i];
      const int m = int(((long long)l * lane + (long long)l * 64 * (n - 1)) % a.N);
      const double pr = a.twD[2 * m], pi = a.twD[2 * m + 1];
      const double ar = __builtin_fma(pr, qr, -pi * qi), ai = __builtin_fma(pr, qi, pi * qr);
      const double sr_ = wave_sum(ar), si_ = wave_sum(ai);
      if (lane == 0 && l0 + i <= a.K) {
        out[2 * (l0 + i)] = sr_;
        out[2 * (l0 + i) + 1] = si_;
      }
    }
  }
}

// P[y, l] = running sum of L^[y, l] over y (one wavefront per (l, image), chunks of 64 rows,
// float64 Hillis-Steele scans with a carry between chunks: a fixed order), then the split
// form: SB[y, l] = P[y, l] and T1[y, l] = 0 for y < H, T1[H, l] = P[H, l].
__global__ void __launch_bounds__(64) k_lap_prefix(LapLowArgs a) {
  const int lane = threadIdx.x;
  const int l = blockIdx.x, b = blockIdx.y;
  const double* in = a.Lh + b * a.img_lh;
  f2* t1 = a.T1 + b * a.img_t1;
  f2* sb = a.SB + b * a.img_sb;
  double cr = 0.0, ci = 0.0;
  for (int y0 = 0; y0 <= a.H; y0 += 64) {
    const int y = y0 + lane;
    double vr = 0.0, vi = 0.0;
    if (y <= a.H) {
      vr = in[((long long)y * (a.K + 1) + l) * 2];
      vi = in[((long long)y * (a.K + 1) + l) * 2 + 1];
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const double ur = __shfl_up(vr, d, 64), ui = __shfl_up(vi, d, 64);
      if (lane >= d) {
        vr += ur;
        vi += ui;
      }
    }
    const double pr = cr + vr, pi = ci + vi;
    if (y < a.H) {
      sb[(long long)y * a.KP + l] = f2{float(pr), float(pi)};
      t1[tile_index(y, l, a.H + 1)] = f2{0.f, 0.f};  // tile-major T1 of H + 1 rows
    } else if (y == a.H) {
      t1[tile_index(y, l, a.H + 1)] = f2{float(pr), float(pi)};
    }
    cr = __shfl(pr, 63, 64);
    ci = __shfl(pi, 63, 64);
  }
}

}  // namespace

hipError_t launch_lap_low(const LapLowArgs& a, int B, hipStream_t s) {
  if (a.K < 0 || a.K >= a.KP || a.H < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lap_rows, dim3(unsigned((a.H + 1 + kLapWaves - 1) / kLapWaves), unsigned(B)),
                     dim3(64 * kLapWaves), 0, s, a);
  hipLaunchKernelGGL(k_lap_prefix, dim3(unsigned(a.K + 1), unsigned(B)), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace gfc
