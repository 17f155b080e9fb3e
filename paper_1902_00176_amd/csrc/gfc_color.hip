// gfc_color.hip - colour-preserving correction of eq. (25):
//     I_corr = (I_c - mean(I_c)) * sigma(I) / sigma(I_c) + mean(I),
// applied in place to the solved images. The inverse row pass leaves float64 sums of u and
// u^2 per workgroup; here every workgroup of an image reduces that image's sums in one fixed
// order (so all of them derive bit-identical statistics), then rescales its share of the
// pixels. sigma is the population standard deviation; the caller's sigma(I) must use the
// same normalisation. A constant image (sigma(I_c) = 0) maps to mean(I).
#include "gfc_buf.h"
#include "gfc_internal.h"

namespace gfc {

constexpr int kColorThreads = 256;
constexpr int kColorPerThread = 16;  // pixels per thread: a workgroup covers 4096

__global__ void __launch_bounds__(kColorThreads)
k_color_apply(float* u, const double* mom, int nparts, const float* I_mean, const float* I_std,
              long long npix) {
  __shared__ double s1[kColorThreads], s2[kColorThreads];
  const int b = blockIdx.y;
  const int t = threadIdx.x;
  // thread-strided sums of the moment pairs, four pairs in flight at a time (pairs past
  // nparts read 0), then the LDS tree
  const rsrc_t rm = make_buf(mom + 2 * (long long)b * nparts, (long long)nparts * 16);
  double a1 = 0.0, a2 = 0.0;
  for (int j0 = 0; j0 < nparts; j0 += 4 * kColorThreads) {
    double v1[4], v2[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int o = (j0 + t + kColorThreads * k) * 16;
      v1[k] = __builtin_bit_cast(double, bld2(rm, o, 0));
      v2[k] = __builtin_bit_cast(double, bld2(rm, o + 8, 0));
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a1 += v1[k];
      a2 += v2[k];
    }
  }
  s1[t] = a1;
  s2[t] = a2;
  __syncthreads();
  for (int h = kColorThreads / 2; h > 0; h >>= 1) {
    if (t < h) {
      s1[t] += s1[t + h];
      s2[t] += s2[t + h];
    }
    __syncthreads();
  }
  const double n = double(npix);
  const double mean = s1[0] / n;
  const double var = s2[0] / n - mean * mean;
  const double sd = var > 0.0 ? __builtin_sqrt(var) : 0.0;
  const float ratio = sd > 0.0 ? float(double(I_std[b]) / sd) : 0.0f;
  const float mf = float(mean), im = I_mean[b];
  const rsrc_t r = make_buf(u + b * npix, npix * 4);
  const int base = blockIdx.x * kColorThreads * kColorPerThread + t;
  float v[kColorPerThread];
#pragma unroll
  for (int k = 0; k < kColorPerThread; ++k) v[k] = bld1(r, (base + k * kColorThreads) * 4, 0);
#pragma unroll
  for (int k = 0; k < kColorPerThread; ++k)
    bst1(r, __builtin_fmaf(v[k] - mf, ratio, im), (base + k * kColorThreads) * 4, 0);
}

hipError_t launch_color_apply(float* u, const double* mom, int nparts, const float* I_mean,
                              const float* I_std, long long npix, int B, hipStream_t s) {
  const long long per = (long long)kColorThreads * kColorPerThread;
  dim3 grid(unsigned((npix + per - 1) / per), B);
  hipLaunchKernelGGL(k_color_apply, grid, dim3(kColorThreads), 0, s, u, mom, nparts, I_mean,
                     I_std, npix);
  return hipGetLastError();
}

}  // namespace gfc


namespace gfc {

constexpr int kScanThreads = 256;  // threads of the small per-plane kernels below

// Volumes: the split bins l <= K of the column input are a = (1 - w_N^l) Ex^ + (1 - w_P^kz) Ez^
// and b = Ey^ (the y difference is applied inside the column recursion). T holds the z
// transform of (1 - w_N^l) Ex^ for those bins; here the z difference of Ez is added as its
// symbol, one thread per (y, l).
__global__ void __launch_bounds__(kScanThreads)
k_sz_combine(f2* T, const f2* SZ, const f2* omz, int H, int NHP, int K, int KP, int P,
             long long plane_t, long long plane_s) {
  const int pl = blockIdx.y;  // volume * P + kz
  const int kz = pl % P;
  const int i = blockIdx.x * kScanThreads + threadIdx.x;
  const int K1 = K + 1;
  if (i >= H * K1) return;
  const int y = i / K1, l = i % K1;
  const f2 o = omz[kz];
  const f2 z = SZ[pl * plane_s + (long long)y * KP + l];
  f2& t = T[pl * plane_t + tile_index(y, l, H + 1)];  // tile-major planes of H + 1 rows
  (void)NHP;
  t.x += o.x * z.x - o.y * z.y;
  t.y += o.x * z.y + o.y * z.x;
}

hipError_t launch_sz_combine(f2* T, const f2* SZ, const f2* omz, int H, int NHP, int K, int KP,
                             int P, long long plane_t, long long plane_s, int B, hipStream_t s) {
  if (K < 0 || K >= KP || H < 1) return hipErrorInvalidValue;
  const int n = H * (K + 1);
  hipLaunchKernelGGL(k_sz_combine, dim3((n + kScanThreads - 1) / kScanThreads, B * P),
                     dim3(kScanThreads), 0, s, T, SZ, omz, H, NHP, K, KP, P, plane_t, plane_s);
  return hipGetLastError();
}

// Volumes: the corner constant is the sum of one partial per (plane, column tile), P times
// more than for an image. Every inverse row workgroup of a volume would re-read them all, so
// they are summed once here (fixed order: thread-strided sums, then an LDS tree).
__global__ void __launch_bounds__(kScanThreads)
k_partial_sums(const double* partial, int nparts, double* total) {
  __shared__ double sh[kScanThreads];
  const int t = threadIdx.x;
  const double* in = partial + (long long)blockIdx.x * nparts;
  double a = strided_sum<kScanThreads, 4>(in, nparts, t);
  sh[t] = a;
  __syncthreads();
  for (int d = kScanThreads / 2; d > 0; d >>= 1) {
    if (t < d) sh[t] += sh[t + d];
    __syncthreads();
  }
  if (t == 0) total[blockIdx.x] = sh[0];
}

hipError_t launch_partial_sums(const double* partial, int nparts, double* total, int B,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_partial_sums, dim3(B), dim3(kScanThreads), 0, s, partial, nparts, total);
  return hipGetLastError();
}

}  // namespace gfc
