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
#include "gfc_buf.h"
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
  static constexpr int NHP = ((NH + 31) / 32) * 32;  // row stride of spectra (256-byte rows)
  static constexpr int NI = (NH + G - 1) / G;  // half-spectrum bins owned per lane
  static_assert(N1 <= 64 && N2 <= 64, "row factors must fit one wavefront");
};

__device__ __forceinline__ cx ld2(const f2* p) {
  const f2 v = *p;
  return {v.x, v.y};
}
__device__ __forceinline__ void st2(f2* p, cx v) { *p = f2{v.x, v.y}; }

// A slot never spans two wavefronts, so its LDS exchanges only need the wavefront to be in
// step: release/acquire fences at wavefront scope around a wave barrier.
__device__ __forceinline__ void slot_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2. This maps
// the linear workgroup index so that every XCD receives a contiguous range of blocks:
// neighbouring rows, which share their boundary row, then meet in the same L2.
constexpr int kXcds = 8;
__device__ __forceinline__ void xcd_contiguous(int& bx, int& by) {
  const int total = gridDim.x * gridDim.y;
  const int lin = blockIdx.x + gridDim.x * blockIdx.y;
  const int q = total / kXcds, r = total % kXcds;
  const int xcd = lin % kXcds, pos = lin / kXcds;
  const int nl = xcd < r ? xcd * (q + 1) + pos : r * (q + 1) + (xcd - r) * q + pos;
  bx = nl % gridDim.x;
  by = nl / gridDim.x;
}

// An integer the optimiser must treat as changed at each loop iteration: added to the uniform
// offsets of loop-invariant table loads so they are issued where used instead of being
// hoisted out of the row loop and held live. Empty asm: no instruction is emitted.
__device__ __forceinline__ int fresh_zero() {
  int z = 0;
  asm volatile("" : "+s"(z));
  return z;
}

// Forward four-step body. On entry lane j < N2 holds a[y1] = z[N2*y1 + j]; on exit the
// spectrum Z is in LDS (re/im planes) in natural order.
template <int N1, int N2>
__device__ __forceinline__ void fwd_fft_to_lds(cx (&a)[N1], float* re, float* im, int lane,
                                               rsrc_t twA, int tz) {
  using C = RowCfg<N1, N2>;
  if (lane < N2) {
    Dft<N1, -1>::run(a);
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
      const f2b w = bld2(twA, lane * 8, tz + k1 * N2 * 8);
      a[k1] = cmul(a[k1], cx{w.x, w.y});
    }
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      re[k1 * C::SA + lane] = a[k1].x;
      im[k1 * C::SA + lane] = a[k1].y;
    }
  }
  slot_sync();
  cx b[N2];
  if (lane < N1) {
#pragma unroll
    for (int j = 0; j < N2; ++j) b[j] = {re[lane * C::SA + j], im[lane * C::SA + j]};
    Dft<N2, -1>::run(b);
  }
  slot_sync();
  if (lane < N1) {
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      re[lane + N1 * k2] = b[k2].x;
      im[lane + N1 * k2] = b[k2].y;
    }
  }
  slot_sync();
}

// Inverse four-step body. On entry lane k < N1 holds b[k2] = Z[k + N1*k2]; on exit lane
// j < N2 holds a[j1] = z[j + N2*j1] (unnormalised inverse DFT).
template <int N1, int N2>
__device__ __forceinline__ void inv_fft_from_regs(cx (&b)[N2], cx (&a)[N1], float* re,
                                                  float* im, int lane, rsrc_t twB, int tz) {
  using C = RowCfg<N1, N2>;
  if (lane < N1) {
    Dft<N2, +1>::run(b);
#pragma unroll
    for (int j2 = 1; j2 < N2; ++j2) {
      const f2b w = bld2(twB, lane * 8, tz + j2 * N1 * 8);
      b[j2] = cmulconj(b[j2], cx{w.x, w.y});
    }
#pragma unroll
    for (int j2 = 0; j2 < N2; ++j2) {
      re[j2 * C::SB + lane] = b[j2].x;
      im[j2 * C::SB + lane] = b[j2].y;
    }
  }
  slot_sync();
  if (lane < N2) {
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) a[k1] = {re[lane * C::SB + k1], im[lane * C::SB + k1]};
    Dft<N1, +1>::run(a);
  }
}

// ---------------------------------------------------------------------------------------
// Forward row pass (divergence + row R2C, eq. (3) and the row half of F(L) in eq. (23)).
// Rows of the block are processed in strips so the previous row's Ey^ stays in registers.
// bx: block of SLOTS strips; b: image of the batch.
template <int N1, int N2, int SLOTS>
__device__ __forceinline__ void row_fwd_body(const RowFwdArgs p, int bx, int b) {
  using C = RowCfg<N1, N2>;
  __shared__ float s_re[SLOTS][C::LDSC];
  __shared__ float s_im[SLOTS][C::LDSC];
  const int slot = threadIdx.x / C::G;
  const int lane = threadIdx.x % C::G;
  float* re = s_re[slot];
  float* im = s_im[slot];
  const int strip = bx * SLOTS + slot;
  const bool strip_ok = strip < p.nstrips;
  const int y0 = strip * p.strip;
  const int K1 = p.KP;
  const rsrc_t rgx = make_buf(p.gx + b * p.img_in, p.img_in * 4);
  const rsrc_t rgy = make_buf(p.gy + b * p.img_in, p.img_in * 4);
  const rsrc_t rT1 = make_buf(p.T1 + b * p.img_t1, p.img_t1 * 8);
  const rsrc_t rSB = make_buf(p.SB + b * p.img_sb, p.img_sb * 8);
  const rsrc_t rtw = make_buf(p.twA, (long long)C::N * 8);
  const rsrc_t rsx = make_buf(p.sx, (long long)C::NH * 8);

  cx prev[C::NI];
#pragma unroll
  for (int i = 0; i < C::NI; ++i) prev[i] = {0.f, 0.f};

  for (int it = 0; it <= p.strip; ++it) {
    const int tz = fresh_zero();
    const int y = y0 - 1 + it;
    const bool row_in = strip_ok && y >= 0 && y < p.H;
    cx a[N1];
    if (lane < N2) {
      const int vo = (y * p.W + lane) * 4;
#pragma unroll
      for (int y1 = 0; y1 < N1; ++y1) {
        // tz keeps the bounds tests inside the row loop (hoisted, their masks spill)
        const int x = N2 * y1 + lane + tz;
        if (row_in && x < p.W) {
          a[y1] = {bld1(rgx, vo, N2 * y1 * 4), bld1(rgy, vo, N2 * y1 * 4)};
        } else {
          a[y1] = {0.f, 0.f};
        }
      }
    }
    fwd_fft_to_lds<N1, N2>(a, re, im, lane, rtw, tz);
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
          const f2b sv = bld2(rsx, lane * 8, tz + C::G * i * 8);
          cx t = cmul(cx{sv.x, sv.y}, ex);
          if (l > p.K) {
            t = cadd(t, csub(ey, prev[i]));
          } else if (y < p.H) {
            bst2(rSB, ey.x, ey.y, (y * K1 + lane) * 8, C::G * i * 8);
          }
          bst2(rT1, t.x, t.y, (y * C::NHP + lane) * 8, C::G * i * 8);
        }
        prev[i] = ey;
      }
    }
    slot_sync();
  }
}

template <int N1, int N2, int SLOTS>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
k_row_fwd(RowFwdArgs p) {
  int bx, by;
  xcd_contiguous(bx, by);
  row_fwd_body<N1, N2, SLOTS>(p, bx, by);
}

// ragged batches: one work item (image, block) per workgroup; pointers rebased per image
template <int N1, int N2, int SLOTS>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
k_row_fwd_rg(RgBase base, const RgRowFwd* tab, const RgItem* items) {
  const RgItem it = items[blockIdx.x];
  const RgRowFwd& e = tab[it.img];
  RowFwdArgs p = e.a;
  p.gx = base.gx + e.in;
  p.gy = base.gy + e.in;
  p.T1 = reinterpret_cast<f2*>(base.ws + e.t);
  p.SB = reinterpret_cast<f2*>(base.ws + e.side);
  row_fwd_body<N1, N2, SLOTS>(p, it.blk, 0);
}

// ---------------------------------------------------------------------------------------
// Inverse row pass (row C2R of eq. (23), real part, crop and Algorithm B's constant).
// Each slot handles p.ppw pairs of rows, two rows per complex inverse FFT.
template <int N1, int N2, int SLOTS>
__device__ __forceinline__ void row_inv_body(const RowInvArgs p, int bx, int b) {
  using C = RowCfg<N1, N2>;
  __shared__ float s_re[SLOTS][C::LDSC];
  __shared__ float s_im[SLOTS][C::LDSC];
  const int slot = threadIdx.x / C::G;
  const int lane = threadIdx.x % C::G;
  float* re = s_re[slot];
  float* im = s_im[slot];
  const rsrc_t rT2 = make_buf(p.T2 + b * p.img_t2, p.img_t2 * 8);
  const rsrc_t ru = make_buf(p.u + b * p.img_u, p.img_u * 4);
  const rsrc_t rtw = make_buf(p.twB, (long long)C::N * 8);

  // v_ref = sum of the column pass's per-tile partials: lane-strided sums, then a fixed-order
  // butterfly across the slot (every lane ends with the same, deterministic total)
  double vr = 0.0;
  for (int j = lane; j < p.nparts; j += C::G) vr += p.partial[(long long)b * p.nparts + j];
#pragma unroll
  for (int off = C::G / 2; off > 0; off >>= 1) vr += __shfl_xor(vr, off, C::G);
  const float vref = float(vr);

  for (int r = 0; r < p.ppw; ++r) {
    const int tz = fresh_zero();
    const int q = (bx * SLOTS + slot) * p.ppw + r;
    const bool ok = q < p.npairs;
    const int y1 = 2 * q, y2 = 2 * q + 1;
    const bool has2 = ok && y2 < p.H;
    cx bz[N2];
    if (lane < N1) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const int kk = lane + N1 * k2;
        const int m = kk < C::NH ? kk : C::N - kk;
        f2b X1 = {0.f, 0.f}, X2 = {0.f, 0.f};
        if (ok) X1 = bld2(rT2, (y1 * C::NHP + m) * 8, 0);
        if (has2) X2 = bld2(rT2, (y2 * C::NHP + m) * 8, 0);
        if (kk < C::NH) bz[k2] = {X1.x - X2.y, X1.y + X2.x};
        else bz[k2] = {X1.x + X2.y, X2.x - X1.y};
      }
    }
    cx a[N1];
    inv_fft_from_regs<N1, N2>(bz, a, re, im, lane, rtw, tz);
    if (lane < N2 && ok) {
      const int v1 = (y1 * p.W + lane) * 4, v2 = (y2 * p.W + lane) * 4;
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) {
        const int x = lane + N2 * j1 + tz;  // tz: bounds tests stay inside the loop
        if (x < p.W) {
          bst1(ru, a[j1].x - vref, v1, N2 * j1 * 4);
          if (has2) bst1(ru, a[j1].y - vref, v2, N2 * j1 * 4);
        }
      }
    }
    slot_sync();
  }
}

template <int N1, int N2, int SLOTS>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
k_row_inv(RowInvArgs p) {
  row_inv_body<N1, N2, SLOTS>(p, blockIdx.x, blockIdx.y);
}

template <int N1, int N2, int SLOTS>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
k_row_inv_rg(RgBase base, const RgRowInv* tab, const RgItem* items) {
  const RgItem it = items[blockIdx.x];
  const RgRowInv& e = tab[it.img];
  RowInvArgs p = e.a;
  p.T2 = reinterpret_cast<const f2*>(base.ws + e.t);
  p.u = base.u + e.out;
  p.partial = reinterpret_cast<const double*>(base.ws + e.red);
  row_inv_body<N1, N2, SLOTS>(p, it.blk, 0);
}

// ---------------------------------------------------------------------------------------
// Backward row pass 1: row R2C of du (two rows per complex FFT) and partial sums of du.
template <int N1, int N2, int SLOTS>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
k_row_bfwd(RowBwdFwdArgs p) {
  using C = RowCfg<N1, N2>;
  __shared__ float s_re[SLOTS][C::LDSC];
  __shared__ float s_im[SLOTS][C::LDSC];
  __shared__ double s_sum[SLOTS];
  const int slot = threadIdx.x / C::G;
  const int lane = threadIdx.x % C::G;
  float* re = s_re[slot];
  float* im = s_im[slot];
  const int b = blockIdx.y;
  const rsrc_t rdu = make_buf(p.du + b * p.img_in, p.img_in * 4);
  const rsrc_t rU = make_buf(p.U + b * p.img_u, p.img_u * 8);
  const rsrc_t rtw = make_buf(p.twA, (long long)C::N * 8);

  double lsum = 0.0;
  for (int r = 0; r < p.ppw; ++r) {
    const int tz = fresh_zero();
    const int q = (blockIdx.x * SLOTS + slot) * p.ppw + r;
    const bool ok = q < p.npairs;
    const int y1 = 2 * q, y2 = 2 * q + 1;
    const bool has2 = ok && y2 < p.H;
    cx a[N1];
    if (lane < N2) {
      const int v1 = (y1 * p.W + lane) * 4, v2 = (y2 * p.W + lane) * 4;
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) {
        const int x = N2 * j1 + lane + tz;  // tz: bounds tests stay inside the loop
        float e1 = 0.f, e2 = 0.f;
        if (ok && x < p.W) e1 = bld1(rdu, v1, N2 * j1 * 4);
        if (has2 && x < p.W) e2 = bld1(rdu, v2, N2 * j1 * 4);
        a[j1] = {e1, e2};
      }
    }
    fwd_fft_to_lds<N1, N2>(a, re, im, lane, rtw, tz);
    // the DC bin of the packed transform is (sum of row y1) + i (sum of row y2)
    if (lane == 0) lsum += double(re[0]) + double(im[0]);
    if (ok) {
#pragma unroll
      for (int i = 0; i < C::NI; ++i) {
        const int l = lane + C::G * i;
        if (l < C::NH) {
          const int m = (l == 0) ? 0 : C::N - l;
          const float ar = re[l], ai = im[l], br = re[m], bi = im[m];
          bst2(rU, 0.5f * (ar + br), 0.5f * (ai - bi), (y1 * C::NHP + lane) * 8, C::G * i * 8);
          if (has2)
            bst2(rU, 0.5f * (ai + bi), 0.5f * (br - ar), (y2 * C::NHP + lane) * 8, C::G * i * 8);
        }
      }
    }
    slot_sync();
  }
  // per-workgroup sum: a fixed-order butterfly within each slot, then the slots in order
#pragma unroll
  for (int off = C::G / 2; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, C::G);
  if (lane == 0) s_sum[slot] = lsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < SLOTS; ++i) t += s_sum[i];
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
  int bx, b;
  xcd_contiguous(bx, b);
  // one row per slot: carrying row y + 1 into the next row's iteration costs more
  // registers than reading it again from cache (the neighbour row's workgroup runs on
  // the same XCD)
  const int y = bx * SLOTS + slot;
  const bool row_ok = y < p.H;
  const int Kb1 = p.KbP;
  const rsrc_t rW = make_buf(p.Wv + b * p.img_w, p.img_w * 8);
  const rsrc_t rSD = make_buf(p.SD + b * p.img_sd, p.img_sd * 8);
  const rsrc_t rgx = make_buf(p.dgx + b * p.img_out, p.img_out * 4);
  const rsrc_t rgy = make_buf(p.dgy + b * p.img_out, p.img_out * 4);
  const rsrc_t rtw = make_buf(p.twB, (long long)C::N * 8);
  const rsrc_t rsxm = make_buf(p.sxm, (long long)C::NH * 8);
  const int tz = fresh_zero();

#pragma unroll
  for (int i = 0; i < C::NI; ++i) {
    const int l = lane + C::G * i;
    if (l < C::NH) {
      cx cur = {0.f, 0.f}, nxt = {0.f, 0.f};
      if (row_ok) {
        const f2b v0 = bld2(rW, (y * C::NHP + lane) * 8, C::G * i * 8);
        const f2b v1 = bld2(rW, ((y + 1) * C::NHP + lane) * 8, C::G * i * 8);
        cur = {v0.x, v0.y};
        nxt = {v1.x, v1.y};
      }
      const f2b sm = bld2(rsxm, lane * 8, tz + C::G * i * 8);
      const cx X1 = cmul(cx{sm.x, sm.y}, cur);
      cx X2;
      if (l <= p.Kb) {
        X2 = {0.f, 0.f};
        if (row_ok) {
          const f2b v = bld2(rSD, (y * Kb1 + lane) * 8, C::G * i * 8);
          X2 = {v.x, v.y};
        }
      } else {
        X2 = csub(cur, nxt);
      }
      // full spectrum of dgx + i dgy at bins l and N - l
      re[l] = X1.x - X2.y;
      im[l] = X1.y + X2.x;
      if (l != 0 && 2 * l != C::N) {
        re[C::N - l] = X1.x + X2.y;
        im[C::N - l] = X2.x - X1.y;
      }
    }
  }
  slot_sync();
  cx bz[N2];
  if (lane < N1) {
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) bz[k2] = {re[lane + N1 * k2], im[lane + N1 * k2]};
  }
  slot_sync();
  cx a[N1];
  inv_fft_from_regs<N1, N2>(bz, a, re, im, lane, rtw, tz);
  if (lane < N2 && row_ok) {
    const int vo = (y * p.W + lane) * 4;
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) {
      const int x = lane + N2 * j1;
      if (x < p.W) {
        bst1(rgx, a[j1].x, vo, N2 * j1 * 4);
        bst1(rgy, a[j1].y, vo, N2 * j1 * 4);
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// launchers

template <int N1, int N2>
struct RowLaunch {
  using C = RowCfg<N1, N2>;
  // 64-lane slots run one wavefront per workgroup; narrower slots fill 256-thread groups
  static constexpr int SLOTS = C::G == 64 ? 1 : 256 / C::G;
  static hipError_t fwd(const RowFwdArgs& a, int B, hipStream_t s) {
    dim3 grid((a.nstrips + SLOTS - 1) / SLOTS, B);
    hipLaunchKernelGGL((k_row_fwd<N1, N2, SLOTS>), grid, dim3(SLOTS * C::G), 0, s, a);
    return hipGetLastError();
  }
  static hipError_t inv(const RowInvArgs& a, int B, hipStream_t s) {
    const int slots_needed = (a.npairs + a.ppw - 1) / a.ppw;
    dim3 grid((slots_needed + SLOTS - 1) / SLOTS, B);
    hipLaunchKernelGGL((k_row_inv<N1, N2, SLOTS>), grid, dim3(SLOTS * C::G), 0, s, a);
    return hipGetLastError();
  }
  static hipError_t bfwd(const RowBwdFwdArgs& a, int B, hipStream_t s) {
    const int slots_needed = (a.npairs + a.ppw - 1) / a.ppw;
    dim3 grid((slots_needed + SLOTS - 1) / SLOTS, B);
    hipLaunchKernelGGL((k_row_bfwd<N1, N2, SLOTS>), grid, dim3(SLOTS * C::G), 0, s, a);
    return hipGetLastError();
  }
  static hipError_t binv(const RowBwdInvArgs& a, int B, hipStream_t s) {
    dim3 grid((a.H + SLOTS - 1) / SLOTS, B);  // one row per slot
    hipLaunchKernelGGL((k_row_binv<N1, N2, SLOTS>), grid, dim3(SLOTS * C::G), 0, s, a);
    return hipGetLastError();
  }
  static hipError_t rg_fwd(const RgBase& base, const RgRowFwd* tab, const RgItem* items,
                           int nitems, hipStream_t s) {
    hipLaunchKernelGGL((k_row_fwd_rg<N1, N2, SLOTS>), dim3(nitems), dim3(SLOTS * C::G), 0, s,
                       base, tab, items);
    return hipGetLastError();
  }
  static hipError_t rg_inv(const RgBase& base, const RgRowInv* tab, const RgItem* items,
                           int nitems, hipStream_t s) {
    hipLaunchKernelGGL((k_row_inv_rg<N1, N2, SLOTS>), dim3(nitems), dim3(SLOTS * C::G), 0, s,
                       base, tab, items);
    return hipGetLastError();
  }
};

#define GFC_ROW_ENTRY(n1, n2)                                                               \
  RowKernels{n1 * n2, n1, n2, RowCfg<n1, n2>::G, RowLaunch<n1, n2>::SLOTS,                   \
             &RowLaunch<n1, n2>::fwd, &RowLaunch<n1, n2>::inv, &RowLaunch<n1, n2>::bfwd,     \
             &RowLaunch<n1, n2>::binv, &RowLaunch<n1, n2>::rg_fwd, &RowLaunch<n1, n2>::rg_inv}

}  // namespace gfc
