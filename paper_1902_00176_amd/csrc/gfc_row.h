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
// Every exchange goes through a single LDS plane per slot, real parts first and then the
// imaginary parts: at N = 2400 that is 9.8 KB instead of 19.7 KB, and together with
// register budgets under 168 it lets three wavefronts share a SIMD instead of two (the row
// passes wait on memory and LDS, and the third wavefront hides those waits: 20-25 % off
// the inverse passes). Spectra are read and written in natural bin order, coalesced.
#pragma once
#include "gfc_buf.h"
#include "gfc_dft.h"
#include "gfc_edit.h"
#include "gfc_internal.h"
#include "gfc_twiddle.h"

#include <utility>

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

// The forward four-step through one LDS plane (real parts, then imaginary parts). On entry
// lane j < N2 holds a[y1] = z[N2*y1 + j]; on exit lane k < N1 holds b[k2] = Z[k + N1*k2]
// and the plane is free (the caller exchanges the spectrum from there).
template <int N1, int N2, bool EXACT_TW = false>
__device__ __forceinline__ void fwd_fft_1p(cx (&a)[N1], cx (&b)[N2], float* pl, int lane,
                                           rsrc_t twA, int tz) {
  using C = RowCfg<N1, N2>;
  if (lane < N2) {
    DftSel<N1, -1>::run(a);
    twiddles<N1, N2, EXACT_TW>(twA, lane, tz, [&](int k1, cx w) { a[k1] = cmul(a[k1], w); });
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) pl[k1 * C::SA + lane] = a[k1].x;
  }
  slot_sync();
  if (lane < N1) {
#pragma unroll
    for (int j = 0; j < N2; ++j) b[j].x = pl[lane * C::SA + j];
  }
  slot_sync();
  if (lane < N2) {
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) pl[k1 * C::SA + lane] = a[k1].y;
  }
  slot_sync();
  if (lane < N1) {
#pragma unroll
    for (int j = 0; j < N2; ++j) b[j].y = pl[lane * C::SA + j];
    // the transform starts once both halves are in: arithmetic on the real parts hoisted
    // above the exchange of the imaginary parts would hold both live
#pragma unroll
    for (int j = 0; j < N2; ++j) asm volatile("" : "+v"(b[j].x), "+v"(b[j].y));
    DftSel<N2, -1>::run(b);
  }
  slot_sync();
}

// Inverse four-step body through one LDS plane (real parts, then imaginary parts). On entry
// lane k < N1 holds b[k2] = Z[k + N1*k2]; on exit lane j < N2 holds a[j1] = z[j + N2*j1]
// (unnormalised inverse DFT).
template <int N1, int N2>
__device__ __forceinline__ void inv_fft_from_regs_1p(cx (&b)[N2], cx (&a)[N1], float* pl,
                                                     int lane, rsrc_t twB, int tz) {
  using C = RowCfg<N1, N2>;
  if (lane < N1) {
    DftSel<N2, +1>::run(b);
    twiddles<N2, N1>(twB, lane, tz, [&](int j2, cx w) { b[j2] = cmulconj(b[j2], w); });
#pragma unroll
    for (int j2 = 0; j2 < N2; ++j2) pl[j2 * C::SB + lane] = b[j2].x;
  }
  slot_sync();
  if (lane < N2) {
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) a[k1].x = pl[lane * C::SB + k1];
  }
  slot_sync();
  if (lane < N1) {
#pragma unroll
    for (int j2 = 0; j2 < N2; ++j2) pl[j2 * C::SB + lane] = b[j2].y;
  }
  slot_sync();
  if (lane < N2) {
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) a[k1].y = pl[lane * C::SB + k1];
    DftSel<N1, +1>::run(a);
  }
}

// ---------------------------------------------------------------------------------------
// Forward row pass (divergence + row R2C, eq. (3) and the row half of F(L) in eq. (23)).
//
// Each slot takes pairs of rows (y, y + 1) of L = div E, formed in float32 from the loaded
// gradient, and transforms them as one complex FFT of L[y] + i L[y + 1]. The bins l <= K go
// to the column pass in the split form (1 - w_N^l) Ex^ and Ey^ instead: those are direct
// sums over the undifferenced rows, because an FFT of L leaves a rounding error of the
// size of |L| in every bin, and the column Green's function amplifies the lowest bins by
// up to 1/lambda(0, 1). In lane j, x = N2 y1 + j and w_N^(l x) = w_N1^(l y1) w_N^(l j): the
// y1 sums take compile-time constants, the lane factor comes from a float64-built table, and
// an LDS transpose sums the lanes.

// acc += v * w_N^E (forward sign) for real v; trivial constants cost one add or nothing
template <int N, int E>
__device__ __forceinline__ void acc_tw(cx& acc, float v) {
  constexpr int e = ((E % N) + N) % N;
  if constexpr (e == 0) {
    acc.x += v;
  } else if constexpr (2 * e == N) {
    acc.x -= v;
  } else if constexpr (4 * e == N) {
    acc.y -= v;
  } else if constexpr (4 * e == 3 * N) {
    acc.y += v;
  } else {
    constexpr float c = float(detail::cs2pi(e, N, 0));
    constexpr float sn = float(-detail::cs2pi(e, N, 1));
    acc.x = __builtin_fmaf(v, c, acc.x);
    acc.y = __builtin_fmaf(v, sn, acc.y);
  }
}

// low-bin partial sums of one y1: Ex bins l = 1..K (index l - 1), Ey bins l = 0..K
template <int N1, int Y1, int... L>
__device__ __forceinline__ void low_acc(cx (&ax)[kLowBins], cx (&ay)[kLowBins + 1], float vx,
                                        float vy, std::integer_sequence<int, L...>) {
  acc_tw<N1, 0>(ay[0], vy);
  (acc_tw<N1, (L + 1) * Y1>(ax[L], vx), ...);
  (acc_tw<N1, (L + 1) * Y1>(ay[L + 1], vy), ...);
}

// low-bin partial sums of one y1 for all bins l = 0..K of one field (volumes: Ez)
template <int N1, int Y1, int... L>
__device__ __forceinline__ void low_acc_all(cx (&az)[kLowBins + 1], float vz,
                                            std::integer_sequence<int, L...>) {
  acc_tw<N1, 0>(az[0], vz);
  (acc_tw<N1, (L + 1) * Y1>(az[L + 1], vz), ...);
}

// Loads of one y1 column of a row pair and its low-bin sums (x = N2 y1 + lane):
// L[y, x] = Ex[y, x] - Ex[y, x-1] + Ey[y, x] - Ey[y-1, x] for rows y0 and y0 + 1. Elements
// outside the image (x >= W, x - 1 < 0, rows outside [0, H), lanes j >= N2) read 0 through
// out-of-range buffer offsets, so the code is straight-line and every load can be in flight
// together.
constexpr int kOOB = 0x70000000;  // a byte offset past every image (plans keep them < 2^30)

// Byte offsets of the bins lane + G i (i = 0, 1, ...) of row y of a tile-major spectrum image
// of R rows (lane < G, G a power of two). Each step of i moves G / kTileBins whole tiles (or,
// for G < kTileBins, part of one), so tile_index's multiply by R is taken once per row and
// the per-i offsets are a scalar product and an add. A row outside the image (ok false)
// gets offsets from kOOB up, which stay below 2^32 since an image is below 2^30 bytes.
template <int G>
struct RowTiles {
  unsigned base, tile;  // offset of bin lane (+ tz); bytes per tile of the image
  __device__ __forceinline__ RowTiles(int y, int lane, int R, bool ok, int tz)
      : base(ok ? unsigned(tile_index(y, lane, R) * 8 + tz) : unsigned(kOOB)),
        tile(unsigned(R) * kTileBins * 8) {}
  __device__ __forceinline__ int operator[](int i) const {
    return int(base + unsigned(i * G / kTileBins) * tile + unsigned(i * G % kTileBins) * 8);
  }
};

// One slot per wavefront: the element x - 1 of lane j is lane j - 1's element x (a DPP
// shift of the whole wavefront by one lane); lane 0 takes `carry`, the previous y1 block's
// element of lane N2 - 1. Saves the x - 1 loads of the divergence.
__device__ __forceinline__ float lane_shift(float v, float carry) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, carry),
                                                               __builtin_bit_cast(int, v),
                                                               0x138 /* wave_shr:1 */, 0xf,
                                                               0xf, false));
}
template <int N2>
__device__ __forceinline__ float lane_last(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), N2 - 1));
}

// One slot per wavefront: the rows are uniform, each row gets its own descriptor whose
// range is that row (empty outside the image), and x >= W falls outside it.
struct PairRowsU {
  rsrc_t x0, x1, ym, y0, y1;
  int vb;  // lane * 4, or kOOB for lanes j >= N2
};
template <int N1, int N2, int Y1>
__device__ __forceinline__ void pair_block(cx (&a)[N1], cx (&ax0)[kLowBins],
                                           cx (&ay0)[kLowBins + 1], cx (&ax1)[kLowBins],
                                           cx (&ay1)[kLowBins + 1], const PairRowsU& r, int W,
                                           float (&cy)[2]) {
  const int v = r.vb + N2 * Y1 * 4;
  const float gx0 = bld1(r.x0, v, 0), gx1 = bld1(r.x1, v, 0);
  const float gym = bld1(r.ym, v, 0), gy0 = bld1(r.y0, v, 0), gy1 = bld1(r.y1, v, 0);
  const float gx0m = lane_shift(gx0, cy[0]), gx1m = lane_shift(gx1, cy[1]);
  cy[0] = lane_last<N2>(gx0);
  cy[1] = lane_last<N2>(gx1);
  a[Y1] = {(gx0 - gx0m) + (gy0 - gym), (gx1 - gx1m) + (gy1 - gy0)};
  low_acc<N1, Y1>(ax0, ay0, gx0, gy0, std::make_integer_sequence<int, kLowBins>{});
  low_acc<N1, Y1>(ax1, ay1, gx1, gy1, std::make_integer_sequence<int, kLowBins>{});
}

// Several slots per wavefront: per-lane row offsets into image-wide descriptors (kOOB for
// rows outside the image and lanes j >= N2), masked per y1 block at x >= W and x - 1 < 0.
struct PairRowsL {
  rsrc_t gx, gy;
  int zm, z0, z1;   // byte offsets of (row, lane) for rows y0 - 1, y0, y0 + 1
  int z0m, z1m;     // x - 1 at y1 = 0: kOOB for lane 0
  int lane;
};
template <int N1, int N2, int Y1>
__device__ __forceinline__ void pair_block(cx (&a)[N1], cx (&ax0)[kLowBins],
                                           cx (&ay0)[kLowBins + 1], cx (&ax1)[kLowBins],
                                           cx (&ay1)[kLowBins + 1], const PairRowsL& r, int W,
                                           float (&)[2]) {
  const int lim = W - N2 * Y1;  // x < W  <=>  lane < lim
  const bool xin = r.lane < lim, xmin = r.lane <= lim;
  constexpr int so = N2 * Y1 * 4, som = Y1 == 0 ? 0 : N2 * Y1 * 4 - 4;
  const int o0 = xin ? r.z0 : kOOB, o1 = xin ? r.z1 : kOOB, om = xin ? r.zm : kOOB;
  const int p0 = xmin ? (Y1 == 0 ? r.z0m : r.z0) : kOOB;
  const int p1 = xmin ? (Y1 == 0 ? r.z1m : r.z1) : kOOB;
  const float gx0 = bld1(r.gx, o0, so), gx0m = bld1(r.gx, p0, som);
  const float gx1 = bld1(r.gx, o1, so), gx1m = bld1(r.gx, p1, som);
  const float gym = bld1(r.gy, om, so), gy0 = bld1(r.gy, o0, so), gy1 = bld1(r.gy, o1, so);
  a[Y1] = {(gx0 - gx0m) + (gy0 - gym), (gx1 - gx1m) + (gy1 - gy0)};
  low_acc<N1, Y1>(ax0, ay0, gx0, gy0, std::make_integer_sequence<int, kLowBins>{});
  low_acc<N1, Y1>(ax1, ay1, gx1, gy1, std::make_integer_sequence<int, kLowBins>{});
}

// Edited variant of one y1 block: both components (and C) at the five pixels the divergence
// of a row pair touches, (y0, x), (y0, x-1), (y0+1, x), (y0+1, x-1), (y0-1, x), each edited
// once. Uniform rows (one slot per wavefront): one descriptor per (field, row).
struct EditRowsU {
  rsrc_t x[3], y[3], c[3];  // rows y0 - 1, y0, y0 + 1
  int vb;
};
template <int N1, int N2, int Y1, int EDIT>
__device__ __forceinline__ void pair_block_edit(cx (&a)[N1], cx (&ax0)[kLowBins],
                                                cx (&ay0)[kLowBins + 1], cx (&ax1)[kLowBins],
                                                cx (&ay1)[kLowBins + 1], const EditRowsU& r,
                                                int W, float tau2, float alpha, float (&cy)[2]) {
  const int v = r.vb + N2 * Y1 * 4;
  auto px = [&](int row, int off, float& ex, float& ey) {
    ex = bld1(r.x[row], off, 0);
    ey = bld1(r.y[row], off, 0);
    const float c = EDIT == kEditGdm ? bld1(r.c[row], off, 0) : 0.f;
    edit_pixel<EDIT>(ex, ey, c, tau2, alpha);
  };
  float x0, y0, x1, y1, xm, ym, x0m, x1m;
  px(1, v, x0, y0);
  px(2, v, x1, y1);
  px(0, v, xm, ym);
  // the edited x - 1 neighbours are the neighbouring lanes' edited values (saves the loads
  // and the edit of two pixels)
  x0m = lane_shift(x0, cy[0]);
  x1m = lane_shift(x1, cy[1]);
  cy[0] = lane_last<N2>(x0);
  cy[1] = lane_last<N2>(x1);
  a[Y1] = {(x0 - x0m) + (y0 - ym), (x1 - x1m) + (y1 - y0)};
  low_acc<N1, Y1>(ax0, ay0, x0, y0, std::make_integer_sequence<int, kLowBins>{});
  low_acc<N1, Y1>(ax1, ay1, x1, y1, std::make_integer_sequence<int, kLowBins>{});
}

// Several slots per wavefront: per-lane row offsets into image-wide descriptors.
struct EditRowsL {
  rsrc_t gx, gy, c;
  int z[3];       // byte offsets of (row, lane) for rows y0 - 1, y0, y0 + 1 (kOOB outside)
  int zm0, zm1;   // x - 1 at y1 = 0 for rows y0, y0 + 1: kOOB for lane 0
  int lane;
};
template <int N1, int N2, int Y1, int EDIT>
__device__ __forceinline__ void pair_block_edit(cx (&a)[N1], cx (&ax0)[kLowBins],
                                                cx (&ay0)[kLowBins + 1], cx (&ax1)[kLowBins],
                                                cx (&ay1)[kLowBins + 1], const EditRowsL& r,
                                                int W, float tau2, float alpha, float (&)[2]) {
  const int lim = W - N2 * Y1;
  const bool xin = r.lane < lim, xmin = r.lane <= lim;
  constexpr int so = N2 * Y1 * 4, som = Y1 == 0 ? 0 : N2 * Y1 * 4 - 4;
  auto px = [&](int off, int soff, float& ex, float& ey) {
    ex = bld1(r.gx, off, soff);
    ey = bld1(r.gy, off, soff);
    const float c = EDIT == kEditGdm ? bld1(r.c, off, soff) : 0.f;
    edit_pixel<EDIT>(ex, ey, c, tau2, alpha);
  };
  float x0, y0, x0m, y0m, x1, y1, x1m, y1m, xm, ym;
  px(xin ? r.z[1] : kOOB, so, x0, y0);
  px(xmin ? (Y1 == 0 ? r.zm0 : r.z[1]) : kOOB, som, x0m, y0m);
  px(xin ? r.z[2] : kOOB, so, x1, y1);
  px(xmin ? (Y1 == 0 ? r.zm1 : r.z[2]) : kOOB, som, x1m, y1m);
  px(xin ? r.z[0] : kOOB, so, xm, ym);
  a[Y1] = {(x0 - x0m) + (y0 - ym), (x1 - x1m) + (y1 - y0)};
  low_acc<N1, Y1>(ax0, ay0, x0, y0, std::make_integer_sequence<int, kLowBins>{});
  low_acc<N1, Y1>(ax1, ay1, x1, y1, std::make_integer_sequence<int, kLowBins>{});
}

// Laplacian input: rows y0 and y0 + 1 of L [H+1][W+1] straight into the FFT input.
struct LapRowsU {
  rsrc_t r0, r1;  // one descriptor per row, range W + 1 elements (empty past row H)
  int vb;
};
template <int N1, int N2, int Y1>
__device__ __forceinline__ void lap_block(cx (&a)[N1], const LapRowsU& r, int W) {
  const int v = r.vb + N2 * Y1 * 4;
  a[Y1] = {bld1(r.r0, v, 0), bld1(r.r1, v, 0)};
}
struct LapRowsL {
  rsrc_t img;
  int z0, z1;  // byte offsets of (row, lane), kOOB past row H or for lanes j >= N2
  int lane;
};
template <int N1, int N2, int Y1>
__device__ __forceinline__ void lap_block(cx (&a)[N1], const LapRowsL& r, int W) {
  const bool xin = r.lane <= W - N2 * Y1;  // x <= W
  constexpr int so = N2 * Y1 * 4;
  a[Y1] = {bld1(r.img, xin ? r.z0 : kOOB, so), bld1(r.img, xin ? r.z1 : kOOB, so)};
}
template <int N1, int N2, int NB, int Y1, class Rows>
__device__ __forceinline__ void lap_load(cx (&a)[N1], const Rows& r, int W) {
  if constexpr (Y1 < N1) {
    if constexpr (Y1 < NB) lap_block<N1, N2, Y1>(a, r, W);
    else a[Y1] = {0.f, 0.f};
    lap_load<N1, N2, NB, Y1 + 1>(a, r, W);
  }
}

// Volumes: slice z of the 7-point divergence, L = dx Ex + dy Ey + (Ez[z] - Ez[z-1]).
// Uniform rows: one descriptor per (field, row); gz of planes z and z - 1.
struct VolRowsU {
  rsrc_t x0, x1, ym, y0, y1, z0, z1, zm0, zm1;
  int vb;
};
// The low-bin sums of the split (bins l <= K) take Ex, Ey and Ez of plane z undifferenced.
struct VolLow {
  cx ax0[kLowBins], ay0[kLowBins + 1], az0[kLowBins + 1];
  cx ax1[kLowBins], ay1[kLowBins + 1], az1[kLowBins + 1];
};
template <int N1, int Y1>
__device__ __forceinline__ void vol_low(VolLow& w, float gx0, float gy0, float gz0, float gx1,
                                        float gy1, float gz1) {
  low_acc<N1, Y1>(w.ax0, w.ay0, gx0, gy0, std::make_integer_sequence<int, kLowBins>{});
  low_acc<N1, Y1>(w.ax1, w.ay1, gx1, gy1, std::make_integer_sequence<int, kLowBins>{});
  low_acc_all<N1, Y1>(w.az0, gz0, std::make_integer_sequence<int, kLowBins>{});
  low_acc_all<N1, Y1>(w.az1, gz1, std::make_integer_sequence<int, kLowBins>{});
}
template <int N1, int N2, int Y1>
__device__ __forceinline__ void vol_block(cx (&a)[N1], VolLow& w, const VolRowsU& r, int W) {
  const int v = r.vb + N2 * Y1 * 4;
  const float gx0 = bld1(r.x0, v, 0), gx0m = bld1(r.x0, v - 4, 0);
  const float gx1 = bld1(r.x1, v, 0), gx1m = bld1(r.x1, v - 4, 0);
  const float gym = bld1(r.ym, v, 0), gy0 = bld1(r.y0, v, 0), gy1 = bld1(r.y1, v, 0);
  const float gz0 = bld1(r.z0, v, 0), gz1 = bld1(r.z1, v, 0);
  const float gzm0 = bld1(r.zm0, v, 0), gzm1 = bld1(r.zm1, v, 0);
  a[Y1] = {((gx0 - gx0m) + (gy0 - gym)) + (gz0 - gzm0),
           ((gx1 - gx1m) + (gy1 - gy0)) + (gz1 - gzm1)};
  vol_low<N1, Y1>(w, gx0, gy0, gz0, gx1, gy1, gz1);
}
// Several slots per wavefront: per-lane offsets into volume-wide descriptors.
struct VolRowsL {
  rsrc_t gx, gy, gz;
  int zm, z0, z1;     // plane z: rows y0 - 1, y0, y0 + 1 (kOOB outside)
  int zz0, zz1;       // plane z - 1: rows y0, y0 + 1 (kOOB outside)
  int z0m, z1m;       // plane z, x - 1 at y1 = 0 (kOOB for lane 0)
  int lane;
};
template <int N1, int N2, int Y1>
__device__ __forceinline__ void vol_block(cx (&a)[N1], VolLow& w, const VolRowsL& r, int W) {
  const int lim = W - N2 * Y1;
  const bool xin = r.lane < lim, xmin = r.lane <= lim;
  constexpr int so = N2 * Y1 * 4, som = Y1 == 0 ? 0 : N2 * Y1 * 4 - 4;
  const int o0 = xin ? r.z0 : kOOB, o1 = xin ? r.z1 : kOOB, om = xin ? r.zm : kOOB;
  const int q0 = xin ? r.zz0 : kOOB, q1 = xin ? r.zz1 : kOOB;
  const int p0 = xmin ? (Y1 == 0 ? r.z0m : r.z0) : kOOB;
  const int p1 = xmin ? (Y1 == 0 ? r.z1m : r.z1) : kOOB;
  const float gx0 = bld1(r.gx, o0, so), gx0m = bld1(r.gx, p0, som);
  const float gx1 = bld1(r.gx, o1, so), gx1m = bld1(r.gx, p1, som);
  const float gym = bld1(r.gy, om, so), gy0 = bld1(r.gy, o0, so), gy1 = bld1(r.gy, o1, so);
  const float gz0 = bld1(r.gz, o0, so), gz1 = bld1(r.gz, o1, so);
  const float gzm0 = bld1(r.gz, q0, so), gzm1 = bld1(r.gz, q1, so);
  a[Y1] = {((gx0 - gx0m) + (gy0 - gym)) + (gz0 - gzm0),
           ((gx1 - gx1m) + (gy1 - gy0)) + (gz1 - gzm1)};
  vol_low<N1, Y1>(w, gx0, gy0, gz0, gx1, gy1, gz1);
}
template <int N1, int N2, int NB, int Y1, class Rows>
__device__ __forceinline__ void vol_load(cx (&a)[N1], VolLow& w, const Rows& r, int W) {
  if constexpr (Y1 < N1) {
    if constexpr (Y1 < NB) vol_block<N1, N2, Y1>(a, w, r, W);
    else a[Y1] = {0.f, 0.f};
    vol_load<N1, N2, NB, Y1 + 1>(a, w, r, W);
  }
}

// blocks y1 < NB carry the support [0, W]; the rest of a[] is zero
template <int N1, int N2, int NB, int Y1, int EDIT = kEditNone, class Rows>
__device__ __forceinline__ void pair_load(cx (&a)[N1], cx (&ax0)[kLowBins],
                                          cx (&ay0)[kLowBins + 1], cx (&ax1)[kLowBins],
                                          cx (&ay1)[kLowBins + 1], const Rows& r, int W,
                                          float (&cy)[2], float tau2 = 0.f, float alpha = 0.f) {
  if constexpr (Y1 < N1) {
    if constexpr (Y1 < NB) {
      if constexpr (EDIT == kEditNone)
        pair_block<N1, N2, Y1>(a, ax0, ay0, ax1, ay1, r, W, cy);
      else
        pair_block_edit<N1, N2, Y1, EDIT>(a, ax0, ay0, ax1, ay1, r, W, tau2, alpha, cy);
    } else {
      a[Y1] = {0.f, 0.f};
    }
    pair_load<N1, N2, NB, Y1 + 1, EDIT>(a, ax0, ay0, ax1, ay1, r, W, cy, tau2, alpha);
  }
}

// Lane factors of the low-bin sums: Ey bins l = 1..K times w_N^(l j) = wp[l]; Ex bins times
// (1 - w_N^l) w_N^(l j), with 1 - w_N^l = 2 sin^2(pi l / N) + i sin(2 pi l / N) folded in as
// compile-time constants (float64-built, rounded once).
template <int N, int... L>
__device__ __forceinline__ void low_lane_factors(cx (&ax0)[kLowBins], cx (&ax1)[kLowBins],
                                                 cx (&ay0)[kLowBins + 1],
                                                 cx (&ay1)[kLowBins + 1],
                                                 const cx (&wp)[kLowBins + 1],
                                                 std::integer_sequence<int, L...>) {
  auto one = [&](auto lc) {
    constexpr int l = decltype(lc)::value + 1;
    constexpr double h = detail::cs2pi(l, 2 * N, 1);  // sin(pi l / N)
    constexpr cx om = {float(2.0 * h * h), float(detail::cs2pi(l, N, 1))};
    const cx wx = cmul(om, wp[l]);
    ax0[l - 1] = cmul(ax0[l - 1], wx);
    ax1[l - 1] = cmul(ax1[l - 1], wx);
    ay0[l] = cmul(ay0[l], wp[l]);
    ay1[l] = cmul(ay1[l], wp[l]);
  };
  (one(std::integral_constant<int, L>{}), ...);
}

// LDS floats of one slot's plane in the forward row pass: the FFT exchange, or the low-bin
// lane sums (NCV complex values per row, both rows, at a stride of G + 1 lanes) when
// larger. Where the sums of both rows would outgrow the exchange they pass through the
// plane one row at a time (kLowRounds = 2), which halves it and holds fewer values live:
// the 256-point volume slice kernel went from 2 to 3 wavefronts per SIMD (128^3 volumes
// 0.31 -> 0.30 ms) and the 1024-point row kernel (32 x 32, slots of 32 lanes) from 176
// registers to 163 and 3 wavefronts (512x512 x 96 0.28 -> 0.27 ms). The 512-point kernel
// (16 x 32) gained no occupancy and lost 2 % to the extra round, and the uneven batch's
// groups of 600-1024 points were no faster: those keep one round.
template <int N1, int N2, int NCV>
constexpr int kLowRounds =
    4 * NCV * (RowCfg<N1, N2>::G + 1) > RowCfg<N1, N2>::LDSC &&
            ((RowCfg<N1, N2>::G == 32 && N1 >= 32) || NCV > 2 * kLowBins + 1)
        ? 2
        : 1;
template <int N1, int N2, int NCV>
constexpr int kFwdPlaneN = cmax(RowCfg<N1, N2>::LDSC, 4 * NCV * (RowCfg<N1, N2>::G + 1) /
                                                        kLowRounds<N1, N2, NCV>);
template <int N1, int N2>
constexpr int kFwdPlane = kFwdPlaneN<N1, N2, 2 * kLowBins + 1>;
// volume slices also sum Ez: 3K + 2 complex low-bin values per row
template <int N1, int N2>
constexpr int kFwdPlane3 = kFwdPlaneN<N1, N2, 3 * kLowBins + 2>;
template <int N1, int N2, int SLOTS, int EDIT = kEditNone>
constexpr int kFwdLds =  // floats per workgroup: one plane per slot
    SLOTS * (EDIT == kIn3D ? kFwdPlane3<N1, N2> : kFwdPlane<N1, N2>);
template <int N1, int N2, int SLOTS>
constexpr int kInvLds = SLOTS * RowCfg<N1, N2>::LDSC;  // one plane per slot

// lds: kFwdLds<N1, N2, SLOTS> floats of the workgroup's LDS
template <int N1, int N2, int SLOTS, int NB, int EDIT = kEditNone>
__device__ __forceinline__ void row_fwd_body(const RowFwdArgs p, int bx, int b, float* lds) {
  using C = RowCfg<N1, N2>;
  constexpr int KL = kLowBins;
  constexpr bool IS3D = EDIT == kIn3D;
  // low-bin complex values per row: Ex bins 1..K, Ey bins 0..K (and Ez bins 0..K, volumes)
  constexpr int NC = 2 * KL + 1 + (IS3D ? KL + 1 : 0);
  constexpr int NV = 4 * NC;             // floats per lane to sum: two rows, re and im
  constexpr int RS = C::G + 1;           // LDS stride of one value over the lanes
  constexpr int PLANE = IS3D ? kFwdPlane3<N1, N2> : kFwdPlane<N1, N2>;
  constexpr int ROUNDS = kLowRounds<N1, N2, NC>;  // rows of low-bin values per pass
  static_assert((NV / ROUNDS) * RS <= PLANE, "the low-bin lane sums fit the slot's plane");
  const int slot = SLOTS == 1 ? 0 : int(threadIdx.x) / C::G;  // uniform with one slot
  const int lane = SLOTS == 1 ? int(threadIdx.x) : int(threadIdx.x) % C::G;
  float* pl = lds + slot * PLANE;
  const float* gxi = p.gx + b * p.img_in;
  const float* gyi = p.gy + b * p.img_in;
  // volumes: b runs over (volume, z <= zd); the T1 plane is z of zp
  const int vz = EDIT == kIn3D ? b % (p.zd + 1) : 0;
  const long long tplane = EDIT == kIn3D ? (long long)(b / (p.zd + 1)) * p.zp + vz : b;
  const long long vplane = EDIT == kIn3D ? (long long)(b / (p.zd + 1)) * p.zd + vz : b;
  if constexpr (EDIT == kIn3D) {
    gxi = p.gx + vplane * p.img_in;
    gyi = p.gy + vplane * p.img_in;
  }
  const rsrc_t rT1 = make_buf(p.T1 + tplane * p.img_t1, p.img_t1 * 8);
  // side arrays: per image, or per (volume, plane z of zp) like T1
  const rsrc_t rSB = make_buf(p.SB + tplane * p.img_sb, p.img_sb * 8);
  const rsrc_t rSZ = make_buf(IS3D ? p.SZ + tplane * p.img_sb : p.SB, IS3D ? p.img_sb * 8 : 0);
  const rsrc_t rtw = make_buf(p.twA, (long long)C::N * 8);
  const rsrc_t rtl = make_buf(p.twL, (long long)2 * (KL + 1) * C::G * 8);
  const rsrc_t rgx = make_buf(gxi, p.img_in * 4);
  const rsrc_t rgy = make_buf(gyi, p.img_in * 4);

  {
    const int tz = fresh_zero();
    const int q = bx * SLOTS + slot;
    const bool ok = q < p.npairs;
    const int y0 = 2 * q;
    cx a[N1];
    cx ax0[KL], ay0[KL + 1], ax1[KL], ay1[KL + 1], az0[KL + 1], az1[KL + 1];
#pragma unroll
    for (int l = 0; l < KL; ++l) ax0[l] = ax1[l] = {0.f, 0.f};
#pragma unroll
    for (int l = 0; l <= KL; ++l) ay0[l] = ay1[l] = az0[l] = az1[l] = {0.f, 0.f};
    // volumes: copy the loader's sums into the arrays above
    auto take = [&](const VolLow& w) {
#pragma unroll
      for (int l = 0; l < KL; ++l) {
        ax0[l] = w.ax0[l];
        ax1[l] = w.ax1[l];
      }
#pragma unroll
      for (int l = 0; l <= KL; ++l) {
        ay0[l] = w.ay0[l];
        ay1[l] = w.ay1[l];
        az0[l] = w.az0[l];
        az1[l] = w.az1[l];
      }
    };
    float cy[2] = {0.f, 0.f};  // x - 1 of the first y1 block: outside the image
    auto row = [&](const float* img, int y) {
      const bool in = ok && y >= 0 && y < p.H;
      return make_buf(img + (in ? (long long)y * p.W : 0), in ? (long long)p.W * 4 : 0);
    };
    auto off = [&](int y) {
      return (ok && lane < N2 && y >= 0 && y < p.H) ? (y * p.W + lane) * 4 : kOOB;
    };
    if constexpr (EDIT == kIn3D && SLOTS == 1) {
      // planes z (z < zd) and z - 1 (z >= 1) of this volume; rows outside read 0
      const bool pz = vz < p.zd, pm = vz >= 1;
      const float* gzi = p.gz + vplane * p.img_in;
      auto prow = [&](const float* img, bool plane_ok, int y) {
        const bool in = plane_ok && ok && y >= 0 && y < p.H;
        return make_buf(img + (in ? (long long)y * p.W : 0), in ? (long long)p.W * 4 : 0);
      };
      const VolRowsU rows{prow(gxi, pz, y0), prow(gxi, pz, y0 + 1), prow(gyi, pz, y0 - 1),
                          prow(gyi, pz, y0), prow(gyi, pz, y0 + 1), prow(gzi, pz, y0),
                          prow(gzi, pz, y0 + 1), prow(gzi - p.img_in, pm, y0),
                          prow(gzi - p.img_in, pm, y0 + 1), (lane < N2 ? lane * 4 : kOOB) + tz};
      VolLow w{};
      vol_load<N1, N2, NB, 0>(a, w, rows, p.W);
      take(w);
    } else if constexpr (EDIT == kIn3D) {
      const bool pz = vz < p.zd, pm = vz >= 1;
      const float* gzi = p.gz + vplane * p.img_in;
      // descriptors from plane z - 1 (when it exists) so both planes are in range
      const long long lo = pm ? p.img_in : 0;
      auto voff = [&](bool plane_ok, int plane, int y) {
        return (plane_ok && ok && lane < N2 && y >= 0 && y < p.H)
                   ? int(plane * p.img_in + y * p.W + lane) * 4 : kOOB;
      };
      const int zp1 = pm ? 1 : 0;  // plane z is the second plane of the descriptors
      const int z0 = voff(pz, zp1, y0), z1 = voff(pz, zp1, y0 + 1);
      const VolRowsL rows{make_buf(gxi - lo, (lo + p.img_in) * 4), make_buf(gyi - lo, (lo + p.img_in) * 4),
                          make_buf(gzi - lo, (lo + p.img_in) * 4), voff(pz, zp1, y0 - 1), z0, z1,
                          voff(pm, 0, y0), voff(pm, 0, y0 + 1),
                          lane > 0 ? z0 - 4 : kOOB, lane > 0 ? z1 - 4 : kOOB, lane};
      VolLow w{};
      vol_load<N1, N2, NB, 0>(a, w, rows, p.W + tz);
      take(w);
    } else if constexpr (EDIT == kInLaplacian && SLOTS == 1) {
      const float* li = p.C + b * (long long)(p.H + 1) * (p.W + 1);
      auto lrow = [&](int y) {
        const bool in = ok && y <= p.H;
        return make_buf(li + (in ? (long long)y * (p.W + 1) : 0), in ? (long long)(p.W + 1) * 4 : 0);
      };
      const LapRowsU rows{lrow(y0), lrow(y0 + 1), (lane < N2 ? lane * 4 : kOOB) + tz};
      lap_load<N1, N2, NB, 0>(a, rows, p.W);
    } else if constexpr (EDIT == kInLaplacian) {
      const float* li = p.C + b * (long long)(p.H + 1) * (p.W + 1);
      auto loff = [&](int y) {
        return (ok && lane < N2 && y <= p.H) ? (y * (p.W + 1) + lane) * 4 : kOOB;
      };
      const LapRowsL rows{make_buf(li, (long long)(p.H + 1) * (p.W + 1) * 4), loff(y0),
                          loff(y0 + 1), lane};
      lap_load<N1, N2, NB, 0>(a, rows, p.W + tz);
    } else if constexpr (EDIT != kEditNone && SLOTS == 1) {
      const float* ci = EDIT == kEditGdm ? p.C + b * p.img_in : gxi;
      const EditRowsU rows{{row(gxi, y0 - 1), row(gxi, y0), row(gxi, y0 + 1)},
                           {row(gyi, y0 - 1), row(gyi, y0), row(gyi, y0 + 1)},
                           {row(ci, y0 - 1), row(ci, y0), row(ci, y0 + 1)},
                           (lane < N2 ? lane * 4 : kOOB) + tz};
      pair_load<N1, N2, NB, 0, EDIT>(a, ax0, ay0, ax1, ay1, rows, p.W, cy, p.tau2, p.alpha);
    } else if constexpr (EDIT != kEditNone) {
      const float* ci = EDIT == kEditGdm ? p.C + b * p.img_in : gxi;
      const int z0 = off(y0), z1 = off(y0 + 1);
      const EditRowsL rows{rgx, rgy, make_buf(ci, p.img_in * 4), {off(y0 - 1), z0, z1},
                           lane > 0 ? z0 - 4 : kOOB, lane > 0 ? z1 - 4 : kOOB, lane};
      pair_load<N1, N2, NB, 0, EDIT>(a, ax0, ay0, ax1, ay1, rows, p.W + tz, cy, p.tau2, p.alpha);
    } else if constexpr (SLOTS == 1) {
      // tz: the per-y1 offsets are formed in the loop, not hoisted and held live
      const PairRowsU rows{row(gxi, y0), row(gxi, y0 + 1), row(gyi, y0 - 1), row(gyi, y0),
                           row(gyi, y0 + 1), (lane < N2 ? lane * 4 : kOOB) + tz};
      pair_load<N1, N2, NB, 0>(a, ax0, ay0, ax1, ay1, rows, p.W, cy);
    } else {
      const int z0 = off(y0), z1 = off(y0 + 1);
      const PairRowsL rows{rgx, rgy, off(y0 - 1), z0, z1,
                           lane > 0 ? z0 - 4 : kOOB, lane > 0 ? z1 - 4 : kOOB, lane};
      pair_load<N1, N2, NB, 0>(a, ax0, ay0, ax1, ay1, rows, p.W + tz, cy);  // tz: masks per row pair
    }

    // lane factors w_N^(l j) (Ex also times 1 - w_N^l), then the sums over the lanes
    // a given Laplacian: every bin comes from the FFT (no split)
    constexpr bool FULLBINS = EDIT == kInLaplacian;
    constexpr int NVL = FULLBINS ? 0 : (NV + C::G - 1) / C::G;
    float lowsum[NVL > 0 ? NVL : 1];
    if constexpr (!FULLBINS) {
    // w_N^(l j) = (w_N^j)^l from one table row (squarings and products: at most three
    // float32 roundings), and the Ex factor 1 - w_N^l = 2 sin^2(pi l / N) + i sin(2 pi l / N)
    // as float64-built compile-time constants: one load instead of 2K
    cx wp[KL + 1];
    {
      const f2b w1 = bld2(rtl, lane * 8, tz + (KL + 2) * C::G * 8);
      wp[1] = {w1.x, w1.y};
    }
#pragma unroll
    for (int l = 2; l <= KL; ++l) wp[l] = (l % 2 == 0) ? cmul(wp[l / 2], wp[l / 2]) : cmul(wp[l - 1], wp[1]);
    low_lane_factors<C::N>(ax0, ax1, ay0, ay1, wp, std::make_integer_sequence<int, KL>{});
    if constexpr (IS3D) {
#pragma unroll
      for (int l = 1; l <= KL; ++l) {
        az0[l] = cmul(az0[l], wp[l]);
        az1[l] = cmul(az1[l], wp[l]);
      }
    }
    // value index: row r of the pair, complex index c < NC (Ex bins 1..K, then Ey bins
    // 0..K, then for volumes Ez bins 0..K); value v = 2 NC r + 2 c (+1 for the imaginary
    // part). With two rounds, row 0's values pass through the plane first, then row 1's.
#pragma unroll
    for (int k = 0; k < NVL; ++k) lowsum[k] = 0.f;
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        constexpr int E2 = 2 * KL + 1;
        const cx v0 = c < KL ? ax0[c < KL ? c : 0]
                             : c < E2 ? ay0[c < E2 ? c - KL : 0] : az0[c < E2 ? 0 : c - E2];
        const cx v1 = c < KL ? ax1[c < KL ? c : 0]
                             : c < E2 ? ay1[c < E2 ? c - KL : 0] : az1[c < E2 ? 0 : c - E2];
        if (ROUNDS == 1 || r == 0) {
          pl[(2 * c) * RS + lane] = v0.x;
          pl[(2 * c + 1) * RS + lane] = v0.y;
        }
        if (ROUNDS == 1) {
          pl[(2 * NC + 2 * c) * RS + lane] = v1.x;
          pl[(2 * NC + 2 * c + 1) * RS + lane] = v1.y;
        } else if (r == 1) {
          pl[(2 * c) * RS + lane] = v1.x;
          pl[(2 * c + 1) * RS + lane] = v1.y;
        }
      }
      slot_sync();
      // lane t sums values t, t + G, ... (of this round) over the N2 lanes that hold elements
      constexpr int VR = NV / ROUNDS;
#pragma unroll
      for (int k = 0; k < NVL; ++k) {
        const int v = lane + C::G * k - VR * r;
        if (v >= 0 && v < VR) {
#pragma unroll
          for (int j = 0; j < N2; ++j) lowsum[k] += pl[v * RS + j];
        }
      }
      slot_sync();
    }
    }  // !FULLBINS

    cx z[N2];
    fwd_fft_1p<N1, N2, FULLBINS || IS3D>(a, z, pl, lane, rtw, tz);

    // Z = FFT(L[y0] + i L[y0+1]): L^[y0, l] = (Z[l] + conj Z[N-l]) / 2,
    // L^[y0+1, l] = (Z[l] - conj Z[N-l]) / 2i; bins l <= K come from the direct sums.
    // Z reaches natural order through the plane, real parts (bins l and N - l of the
    // lane) first, then the imaginary parts, read where they are used.
    float zr[C::NI], zm[C::NI];
    if (lane < N1) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) pl[lane + N1 * k2] = z[k2].x;
    }
    slot_sync();
#pragma unroll
    for (int i = 0; i < C::NI; ++i) {
      const int l = lane + C::G * i;
      const bool inside = C::G * i + C::G - 1 < C::NH ? true : l < C::NH;
      const int m = (i == 0 && lane == 0) || !inside ? 0 : C::N - l;
      zr[i] = pl[inside ? l : 0];
      zm[i] = pl[m];
    }
    slot_sync();
    if (lane < N1) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) pl[lane + N1 * k2] = z[k2].y;
    }
    slot_sync();
    const bool has1 = ok && y0 + 1 <= p.H;
    const int RT = p.H + 1;  // rows of a T1 image (tile_index)
    if constexpr (SLOTS == 1) {
      // uniform rows: a descriptor per T1 row (the image, empty when the row is outside it),
      // so missing rows are dropped by the hardware with no branch; bins in [NH, NHP) land in
      // the padding of the last tile, and bins past NHP past the image
      const f2* t1b = p.T1 + tplane * p.img_t1;
      const rsrc_t w0 = make_buf(t1b, ok ? p.img_t1 * 8 : 0);
      const rsrc_t w1 = make_buf(t1b, has1 ? p.img_t1 * 8 : 0);
      const RowTiles<C::G> rt(y0, lane, RT, true, tz);
#pragma unroll
      for (int i = 0; i < C::NI; ++i) {
        const int l = lane + C::G * i;
        // mirror bin N - l (0 for l = 0, and for lanes past NH whose stores are dropped)
        const bool inside = C::G * i + C::G - 1 < C::NH ? true : l < C::NH;
        const int m = (i == 0 && lane == 0) || !inside ? 0 : C::N - l;
        const float ar = zr[i], ai = pl[inside ? l : 0], br = zm[i], bi = pl[m];
        cx A = {0.5f * (ar + br), 0.5f * (ai - bi)};
        cx B = {0.5f * (ai + bi), 0.5f * (br - ar)};
        int off = rt[i];
        if constexpr (!FULLBINS) {
          if (i == 0) {
            // bins 1..K come from the direct sums; bin 0 of T1 is (1 - w_N^0) Ex^ = 0
            if (lane == 0) A = B = {0.f, 0.f};
            else if (lane <= KL) off = kOOB;
          }
        }
        bst2(w0, A.x, A.y, off, 0);
        bst2(w1, B.x, B.y, off + kTileBins * 8, 0);  // row y0 + 1: the next row of the tile
      }
    } else {
#pragma unroll
    for (int i = 0; i < C::NI; ++i) {
      const int l = lane + C::G * i;
      if constexpr (FULLBINS) {
        // every bin of L^ goes to T1. A given Laplacian's bins l <= K are then replaced by
        // their split form (launch_lap_low); volumes build theirs after the z transform
        if (ok && l < C::NH) {
          const int m = (l == 0) ? 0 : C::N - l;
          const float ar = zr[i], ai = pl[l], br = zm[i], bi = pl[m];
          const cx A = {0.5f * (ar + br), 0.5f * (ai - bi)};
          const cx B = {0.5f * (ai + bi), 0.5f * (br - ar)};
          bst2(rT1, A.x, A.y, tile_index(y0, l, RT) * 8, 0);
          if (has1) bst2(rT1, B.x, B.y, tile_index(y0 + 1, l, RT) * 8, 0);
        }
      } else if (ok && l < C::NH && (l == 0 || l > KL)) {
        const int m = (l == 0) ? 0 : C::N - l;
        const float ar = zr[i], ai = pl[l], br = zm[i], bi = pl[m];
        cx A = {0.5f * (ar + br), 0.5f * (ai - bi)};
        cx B = {0.5f * (ai + bi), 0.5f * (br - ar)};
        if (l == 0) A = B = {0.f, 0.f};  // (1 - w_N^0) Ex^ = 0; Ey^ goes to SB
        bst2(rT1, A.x, A.y, tile_index(y0, l, RT) * 8, 0);
        if (has1) bst2(rT1, B.x, B.y, tile_index(y0 + 1, l, RT) * 8, 0);
      }
    }
    }
#pragma unroll
    for (int k = 0; k < NVL; ++k) {
      const int v = lane + C::G * k;
      if (ok && v < NV) {
        const int rr = v / (2 * NC), c = (v / 2) % NC, comp = v & 1;
        const int y = y0 + rr;
        if (c < KL) {
          if (y <= p.H) bst1(rT1, lowsum[k], tile_index(y, c + 1, RT) * 8 + comp * 4, 0);
        } else if (c < 2 * KL + 1) {
          if (y < p.H) bst1(rSB, lowsum[k], (y * p.KP + c - KL) * 8 + comp * 4, 0);
        } else if (y < p.H) {
          bst1(rSZ, lowsum[k], (y * p.KP + c - 2 * KL - 1) * 8 + comp * 4, 0);
        }
      }
    }
    slot_sync();
  }
}

// Edited loaders hold more values than the plain one; left alone the compiler gives them
// one wavefront per SIMD. With one slot per workgroup (the x - 1 neighbours come by lane
// shifts) two wavefronts (a few spilled registers) measured 1.2-1.6x faster; the
// full-support variants (2 W > N) and the several-slot loaders would spill far more and
// keep the default.
template <int N1, int SLOTS, int NB, int EDIT>
constexpr int kFwdWaves =
    ((EDIT == kEditThreshold || EDIT == kEditGdm) && NB < N1 && SLOTS == 1) ? 2 : 1;

// NB: y1 blocks that can hold the support [0, W] (all N1, or N1/2 + 1 when 2 W <= N)
template <int N1, int N2, int SLOTS, int NB, int EDIT>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
__attribute__((amdgpu_waves_per_eu(kFwdWaves<N1, SLOTS, NB, EDIT>)))
k_row_fwd(RowFwdArgs p) {
  __shared__ float lds[kFwdLds<N1, N2, SLOTS, EDIT>];
  int bx, by;
  xcd_contiguous(bx, by);
  row_fwd_body<N1, N2, SLOTS, NB, EDIT>(p, bx, by, lds);
}

// ragged batches: one work item (image, block) per workgroup; pointers rebased per image
template <int N1, int N2, int SLOTS, int NB>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
k_row_fwd_rg(const RgBase* basep, const RgRowFwd* tab, const RgItem* items) {
  const RgBase base = *basep;  // written by launch_set_base on this stream
  const RgItem it = items[blockIdx.x];
  const RgRowFwd& e = tab[it.img];
  RowFwdArgs p = e.a;
  p.gx = base.gx + e.in;
  p.gy = base.gy + e.in;
  p.T1 = reinterpret_cast<f2*>(base.ws + e.t);
  p.SB = reinterpret_cast<f2*>(base.ws + e.side);
  __shared__ float lds[kFwdLds<N1, N2, SLOTS>];
  row_fwd_body<N1, N2, SLOTS, NB>(p, it.blk, 0, lds);
}

// ---------------------------------------------------------------------------------------
// Inverse row pass (row C2R of eq. (23), real part, crop and Algorithm B's constant).
// Each slot handles one pair of rows, two rows per complex inverse FFT.
// MOM: also the float64 sums of the stored values and their squares, one pair per
// workgroup (fixed summation order), for the colour correction of eq. (25).
// lds: kInvLds<N1, N2, SLOTS> floats of the workgroup's LDS
// Output blocks j1 of the inverse row pass that can hold x = lane + N2 j1 < W when 2 W <= N
template <int N1>
constexpr int kInvHalf = (N1 + 1) / 2;

// Packed spectrum of two real rows, P = F(r1) + i F(r2), from their half spectra X1, X2 at
// the bins l = lane + G q < NH that the lane holds: P[l] = (X1.x - X2.y, X1.y + X2.x) and
// P[N - l] = (X1.x + X2.y, X2.x - X1.y). The bins go through one LDS plane, real parts
// first, and come out in the four-step layout: lane k < N1 gets bz[k2] = P[k + N1 k2].
template <int N1, int N2>
__device__ __forceinline__ void packed_to_bz(const cx (&X1)[RowCfg<N1, N2>::NI],
                                             const cx (&X2)[RowCfg<N1, N2>::NI],
                                             cx (&bz)[N2], float* pl, int lane) {
  using C = RowCfg<N1, N2>;
#pragma unroll
  for (int q = 0; q < C::NI; ++q) {
    const int l = lane + C::G * q;
    if (l < C::NH) {
      pl[l] = X1[q].x - X2[q].y;
      if (l != 0 && 2 * l != C::N) pl[C::N - l] = X1[q].x + X2[q].y;
    }
  }
  slot_sync();
  if (lane < N1) {
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) bz[k2].x = pl[lane + N1 * k2];
  }
  slot_sync();
#pragma unroll
  for (int q = 0; q < C::NI; ++q) {
    const int l = lane + C::G * q;
    if (l < C::NH) {
      pl[l] = X1[q].y + X2[q].x;
      if (l != 0 && 2 * l != C::N) pl[C::N - l] = X2[q].x - X1[q].y;
    }
  }
  slot_sync();
  if (lane < N1) {
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) bz[k2].y = pl[lane + N1 * k2];
  }
  slot_sync();
}

// NBO: output blocks j1 that can hold x < W (N1, or kInvHalf<N1> when 2 W <= N)
template <int N1, int N2, int SLOTS, bool MOM = false, int NBO = N1>
__device__ __forceinline__ void row_inv_body(const RowInvArgs p, int bx, int b, float* lds) {
  using C = RowCfg<N1, N2>;
  __shared__ double s_mom[SLOTS][2];
  double m1 = 0.0, m2 = 0.0;
  const int slot = SLOTS == 1 ? 0 : int(threadIdx.x) / C::G;  // uniform with one slot
  const int lane = SLOTS == 1 ? int(threadIdx.x) : int(threadIdx.x) % C::G;
  float* pl = lds + slot * C::LDSC;
  // image b, or slice z = b % zd of volume b / zd (its spectra are plane z of zp)
  const int vol = b / p.zd;
  const f2* T2i = p.T2 + ((long long)vol * p.zp + b % p.zd) * p.img_t2;
  const rsrc_t ru = make_buf(p.u + b * p.img_u, p.img_u * 4);
  const rsrc_t rtw = make_buf(p.twB, (long long)C::N * 8);

  // v_ref = sum of the column pass's per-tile partials: lane-strided sums, then a fixed-order
  // butterfly across the slot (every lane ends with the same, deterministic total)
  double vr = strided_sum<C::G, 4>(p.partial + (long long)vol * p.nparts, p.nparts, lane);
#pragma unroll
  for (int off = C::G / 2; off > 0; off >>= 1) vr += __shfl_xor(vr, off, C::G);
  const float vref = float(vr);

  {
    const int tz = fresh_zero();
    const int q = bx * SLOTS + slot;
    const bool ok = q < p.npairs;
    const int y1 = 2 * q, y2 = 2 * q + 1;
    const bool has2 = ok && y2 < p.H;
    cx bz[N2];
    const int RT = p.H + 1;  // rows of a T2 image (tile_index)
    if constexpr (SLOTS == 1) {
      // One slot per wavefront: the rows are uniform and each has a descriptor for the image,
      // empty when the row is outside it (its loads read 0). The spectrum bins are read in
      // natural order (bins in [NH, NHP) read the last tile's padding, unused) and reach the
      // four-step layout through LDS.
      const rsrc_t r1 = make_buf(T2i, ok ? p.img_t2 * 8 : 0);
      const rsrc_t r2 = make_buf(T2i, has2 ? p.img_t2 * 8 : 0);
      cx X1[C::NI], X2[C::NI];
      const RowTiles<C::G> rt(y1, lane, RT, true, tz);
#pragma unroll
      for (int i = 0; i < C::NI; ++i) {
        // the whole offset per lane, so that the range check covers it (row y2 = y1 + 1 is
        // the next row of the tile)
        const int o = rt[i];
        const f2b v1 = bld2(r1, o, 0);
        const f2b v2 = bld2(r2, o + kTileBins * 8, 0);
        X1[i] = {v1.x, v1.y};
        X2[i] = {v2.x, v2.y};
      }
      packed_to_bz<N1, N2>(X1, X2, bz, pl, lane);
    } else if (lane < N1) {
      // slots of one wavefront hold different rows: one descriptor for the image, and lane
      // k gathers its bins k + N1 k2 (from the Hermitian mirror past N/2) directly
      const rsrc_t rT2 = make_buf(T2i, p.img_t2 * 8);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const int kk = lane + N1 * k2;
        const int m = kk < C::NH ? kk : C::N - kk;
        f2b X1 = {0.f, 0.f}, X2 = {0.f, 0.f};
        if (ok) X1 = bld2(rT2, tile_index(y1, m, RT) * 8, 0);
        if (has2) X2 = bld2(rT2, tile_index(y2, m, RT) * 8, 0);
        if (kk < C::NH) bz[k2] = {X1.x - X2.y, X1.y + X2.x};
        else bz[k2] = {X1.x + X2.y, X2.x - X1.y};
      }
    }
    cx a[N1];
    inv_fft_from_regs_1p<N1, N2>(bz, a, pl, lane, rtw, tz);
    if constexpr (SLOTS == 1 && !MOM) {
      // output rows with descriptors whose range is the row: stores at x >= W are dropped
      // by the hardware with no branch; blocks j1 >= NBO hold no x < W and are not stored
      const float* ub = p.u + b * p.img_u;
      const rsrc_t u1 = make_buf(ub + (long long)y1 * p.W, ok ? (long long)p.W * 4 : 0);
      const rsrc_t u2 = make_buf(ub + (long long)y2 * p.W, has2 ? (long long)p.W * 4 : 0);
      const int vb = (lane < N2 ? lane * 4 : kOOB) + tz;
#pragma unroll
      for (int j1 = 0; j1 < NBO; ++j1) {
        bst1(u1, a[j1].x - vref, vb + N2 * j1 * 4, 0);
        bst1(u2, a[j1].y - vref, vb + N2 * j1 * 4, 0);
      }
    } else if (lane < N2 && ok) {
      const int v1 = (y1 * p.W + lane) * 4, v2 = (y2 * p.W + lane) * 4;
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) {
        const int x = lane + N2 * j1 + tz;  // tz: bounds tests stay inside the loop
        if (x < p.W) {
          const float o1 = a[j1].x - vref, o2 = a[j1].y - vref;
          bst1(ru, o1, v1, N2 * j1 * 4);
          if (has2) bst1(ru, o2, v2, N2 * j1 * 4);
          if constexpr (MOM) {
            const double d1 = o1, d2 = has2 ? double(o2) : 0.0;
            m1 += d1 + d2;
            m2 = __builtin_fma(d1, d1, __builtin_fma(d2, d2, m2));
          }
        }
      }
    }
    slot_sync();
  }
  if constexpr (MOM) {
#pragma unroll
    for (int off = C::G / 2; off > 0; off >>= 1) {
      m1 += __shfl_xor(m1, off, C::G);
      m2 += __shfl_xor(m2, off, C::G);
    }
    if (lane == 0) {
      s_mom[slot][0] = m1;
      s_mom[slot][1] = m2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double t1 = 0.0, t2 = 0.0;
      for (int i = 0; i < SLOTS; ++i) {
        t1 += s_mom[i][0];
        t2 += s_mom[i][1];
      }
      double* o = p.mom + 2 * ((long long)b * gridDim.x + bx);
      o[0] = t1;
      o[1] = t2;
    }
  }
}

template <int N1, int N2, int SLOTS, bool MOM, int NBO = N1>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
__attribute__((amdgpu_waves_per_eu(3))) k_row_inv(RowInvArgs p) {
  __shared__ float lds[kInvLds<N1, N2, SLOTS>];
  row_inv_body<N1, N2, SLOTS, MOM, NBO>(p, blockIdx.x, blockIdx.y, lds);
}

template <int N1, int N2, int SLOTS, int NBO = N1>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
k_row_inv_rg(const RgBase* basep, const RgRowInv* tab, const RgItem* items) {
  const RgBase base = *basep;  // written by launch_set_base on this stream
  const RgItem it = items[blockIdx.x];
  const RgRowInv& e = tab[it.img];
  RowInvArgs p = e.a;
  p.T2 = reinterpret_cast<const f2*>(base.ws + e.t);
  p.u = base.u + e.out;
  p.partial = reinterpret_cast<const double*>(base.ws + e.red);
  __shared__ float lds[kInvLds<N1, N2, SLOTS>];
  row_inv_body<N1, N2, SLOTS, false, NBO>(p, it.blk, 0, lds);
}

// ---------------------------------------------------------------------------------------
// Backward row pass 1: row R2C of du (two rows per complex FFT) and partial sums of du.
// NB: input blocks j1 that can hold x < W (N1, or kInvHalf<N1> when 2 W <= N)
template <int N1, int N2, int SLOTS, int NB = N1>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
__attribute__((amdgpu_waves_per_eu(3))) k_row_bfwd(RowBwdFwdArgs p) {
  using C = RowCfg<N1, N2>;
  __shared__ float s_pl[SLOTS][C::LDSC];  // one plane: real parts cross, then imaginary
  __shared__ double s_sum[SLOTS];
  const int slot = SLOTS == 1 ? 0 : int(threadIdx.x) / C::G;  // uniform with one slot
  const int lane = SLOTS == 1 ? int(threadIdx.x) : int(threadIdx.x) % C::G;
  float* pl = s_pl[slot];
  const int b = blockIdx.y;
  const rsrc_t rdu = make_buf(p.du + b * p.img_in, p.img_in * 4);
  const rsrc_t rU = make_buf(p.U + b * p.img_u, p.img_u * 8);
  const rsrc_t rtw = make_buf(p.twA, (long long)C::N * 8);

  double lsum = 0.0;
  {
    const int tz = fresh_zero();
    const int q = blockIdx.x * SLOTS + slot;
    const bool ok = q < p.npairs;
    const int y1 = 2 * q, y2 = 2 * q + 1;
    const bool has2 = ok && y2 < p.H;
    cx a[N1];
    if constexpr (SLOTS == 1) {
      // uniform rows: a descriptor per row whose range is that row (empty outside the
      // image), so x >= W and missing rows read 0 with no branch; blocks j1 >= NB are 0
      const float* db = p.du + b * p.img_in;
      const rsrc_t d1 = make_buf(db + (long long)y1 * p.W, ok ? (long long)p.W * 4 : 0);
      const rsrc_t d2 = make_buf(db + (long long)y2 * p.W, has2 ? (long long)p.W * 4 : 0);
      const int vb = (lane < N2 ? lane * 4 : kOOB) + tz;
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1)
        a[j1] = j1 < NB ? cx{bld1(d1, vb + N2 * j1 * 4, 0), bld1(d2, vb + N2 * j1 * 4, 0)}
                        : cx{0.f, 0.f};
    } else if (lane < N2) {
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
    cx z[N2];
    fwd_fft_1p<N1, N2>(a, z, pl, lane, rtw, tz);
    // bins l and m = N - l of the packed transform, real parts first
    float ar[C::NI], br[C::NI];
    if (lane < N1) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) pl[lane + N1 * k2] = z[k2].x;
    }
    slot_sync();
#pragma unroll
    for (int i = 0; i < C::NI; ++i) {
      const int l = lane + C::G * i;
      const int m = (l == 0) ? 0 : C::N - l;
      ar[i] = l < C::NH ? pl[l] : 0.f;
      br[i] = l < C::NH ? pl[m] : 0.f;
    }
    slot_sync();
    if (lane < N1) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) pl[lane + N1 * k2] = z[k2].y;
    }
    slot_sync();
    // the DC bin of the packed transform is (sum of row y1) + i (sum of row y2)
    if (lane == 0) lsum += double(ar[0]) + double(pl[0]);
    if (ok) {
      const RowTiles<C::G> rt(y1, lane, p.H + 1, true, 0);  // U images have H + 1 rows
#pragma unroll
      for (int i = 0; i < C::NI; ++i) {
        const int l = lane + C::G * i;
        if (l < C::NH) {
          const int m = (l == 0) ? 0 : C::N - l;
          const float ai = pl[l], bi = pl[m];
          const int o = rt[i];
          bst2(rU, 0.5f * (ar[i] + br[i]), 0.5f * (ai - bi), o, 0);
          if (has2) bst2(rU, 0.5f * (ai + bi), 0.5f * (br[i] - ar[i]), o + kTileBins * 8, 0);
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

// e^(i pi G q / N) for q < NI, evaluated at compile time
template <int N, int G, int NI>
struct HalfTurns {
  float c[NI], s[NI];
  constexpr HalfTurns() : c(), s() {
    for (int q = 0; q < NI; ++q) {
      c[q] = float(detail::cs2pi(long(G) * q, 2L * N, 0));
      s[q] = float(detail::cs2pi(long(G) * q, 2L * N, 1));
    }
  }
};

// ---------------------------------------------------------------------------------------
// Backward row pass 2: apply -D_x as its symbol, -D_y from the column pass (low columns) or
// as a row difference (other columns), and one complex C2R per row for (dgx, dgy).
// NBO: output blocks j1 that can hold x < W (N1, or kInvHalf<N1> when 2 W <= N)
// One LDS plane per slot (the real parts of each exchange, then the imaginary parts).
template <int N1, int N2, int SLOTS, int NBO = N1>
__global__ void __launch_bounds__((SLOTS * RowCfg<N1, N2>::G))
__attribute__((amdgpu_waves_per_eu(3))) k_row_binv(RowBwdInvArgs p) {
  using C = RowCfg<N1, N2>;
  __shared__ float s_pl[SLOTS][C::LDSC];
  const int slot = SLOTS == 1 ? 0 : int(threadIdx.x) / C::G;  // uniform with one slot
  const int lane = SLOTS == 1 ? int(threadIdx.x) : int(threadIdx.x) % C::G;
  float* pl = s_pl[slot];
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
  const int tz = fresh_zero();

  // All loads first (branch-free: rows outside the image read 0 through an out-of-range
  // offset, bins past NH are loaded and ignored), so they are in flight together.
  constexpr int NID = (kLowBinsB + C::G) / C::G;  // slices that can hold a bin l <= Kb
  cx cur[C::NI], nxt[C::NI], sdv[NID];
  const RowTiles<C::G> rt(y, lane, p.H + 1, row_ok, tz);  // W images have H + 1 rows
#pragma unroll
  for (int i = 0; i < C::NI; ++i) {
    // row y + 1 is the next row of the tile
    const int o = rt[i];
    const f2b v0 = bld2(rW, o, 0);
    const f2b v1 = bld2(rW, o + kTileBins * 8, 0);
    cur[i] = {v0.x, v0.y};
    nxt[i] = {v1.x, v1.y};
  }
#pragma unroll
  for (int i = 0; i < NID; ++i) {
    const int l = lane + C::G * i;
    const f2b v = bld2(rSD, (row_ok && l <= p.Kb) ? (y * Kb1 + l) * 8 : kOOB, 0);
    sdv[i] = {v.x, v.y};
  }
  // -D_x's symbol 1 - w_N^-l = 2 s (s - i c) with (c, s) = e^(i pi l / N), formed from the
  // lane's half-angle and a compile-time step per block of G bins: no cancellation at low l
  float hs, hc;
  sincospif(float(lane) / float(C::N), &hs, &hc);
  constexpr HalfTurns<C::N, C::G, C::NI> ht{};
  // the packed spectrum of dgx + i dgy: X1 = -D_x's part, X2 = -D_y's part
  cx X1[C::NI], X2[C::NI];
#pragma unroll
  for (int i = 0; i < C::NI; ++i) {
    const int l = lane + C::G * i;
    const float cl = hc * ht.c[i] - hs * ht.s[i], sl = hs * ht.c[i] + hc * ht.s[i];
    X1[i] = cmul(cx{2.f * sl * sl, -2.f * sl * cl}, cur[i]);
    X2[i] = (i < NID && l <= p.Kb) ? sdv[i < NID ? i : 0] : csub(cur[i], nxt[i]);
  }
  cx bz[N2];
  packed_to_bz<N1, N2>(X1, X2, bz, pl, lane);
  cx a[N1];
  inv_fft_from_regs_1p<N1, N2>(bz, a, pl, lane, rtw, tz);
  if constexpr (SLOTS == 1) {
    // uniform row: descriptors whose range is that row, so stores at x >= W (and of a row
    // outside the image) are dropped with no branch; blocks j1 >= NBO are not stored
    const long long ro = b * p.img_out + (long long)y * p.W;
    const long long rn = row_ok ? (long long)p.W * 4 : 0;
    const rsrc_t ox = make_buf(p.dgx + ro, rn), oy = make_buf(p.dgy + ro, rn);
    const int vb = (lane < N2 ? lane * 4 : kOOB) + tz;
#pragma unroll
    for (int j1 = 0; j1 < NBO; ++j1) {
      bst1(ox, a[j1].x, vb + N2 * j1 * 4, 0);
      bst1(oy, a[j1].y, vb + N2 * j1 * 4, 0);
    }
  } else if (lane < N2 && row_ok) {
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

// ALL = false: the forward launcher handles the plain solve only (the candidate entries of a
// library built for split tuning, which times the plain passes)
template <int N1, int N2, bool ALL = true>
struct RowLaunch {
  using C = RowCfg<N1, N2>;
  // 64-lane slots run one wavefront per workgroup; narrower slots fill 256-thread groups
  static constexpr int SLOTS = C::G == 64 ? 1 : 256 / C::G;
  // y1 blocks of the forward loads: rows with 2 W <= N have their support in the first
  // N1/2 + 1 of them
  static constexpr int NB_HALF = N1 / 2 + 1 < N1 ? N1 / 2 + 1 : N1;
  static hipError_t fwd(const RowFwdArgs& a, int B, hipStream_t s) {
    const int slots_needed = a.npairs;
    dim3 grid((slots_needed + SLOTS - 1) / SLOTS, B);
    const bool half = 2 * a.W <= N1 * N2;
    const dim3 blk(SLOTS * C::G);
    if constexpr (!ALL) {
      if (a.edit != kEditNone) return hipErrorInvalidValue;
      if (half) hipLaunchKernelGGL((k_row_fwd<N1, N2, SLOTS, NB_HALF, kEditNone>), grid, blk, 0, s, a);
      else hipLaunchKernelGGL((k_row_fwd<N1, N2, SLOTS, N1, kEditNone>), grid, blk, 0, s, a);
      return hipGetLastError();
    } else {
      switch (a.edit) {
        case kEditThreshold:
          if (half) hipLaunchKernelGGL((k_row_fwd<N1, N2, SLOTS, NB_HALF, kEditThreshold>), grid, blk, 0, s, a);
          else hipLaunchKernelGGL((k_row_fwd<N1, N2, SLOTS, N1, kEditThreshold>), grid, blk, 0, s, a);
          break;
        case kEditGdm:
          if (half) hipLaunchKernelGGL((k_row_fwd<N1, N2, SLOTS, NB_HALF, kEditGdm>), grid, blk, 0, s, a);
          else hipLaunchKernelGGL((k_row_fwd<N1, N2, SLOTS, N1, kEditGdm>), grid, blk, 0, s, a);
          break;
        case kInLaplacian:
          if (half) hipLaunchKernelGGL((k_row_fwd<N1, N2, SLOTS, NB_HALF, kInLaplacian>), grid, blk, 0, s, a);
          else hipLaunchKernelGGL((k_row_fwd<N1, N2, SLOTS, N1, kInLaplacian>), grid, blk, 0, s, a);
          break;
        case kIn3D:
          if (half) hipLaunchKernelGGL((k_row_fwd<N1, N2, SLOTS, NB_HALF, kIn3D>), grid, blk, 0, s, a);
          else hipLaunchKernelGGL((k_row_fwd<N1, N2, SLOTS, N1, kIn3D>), grid, blk, 0, s, a);
          break;
        default:
          if (half) hipLaunchKernelGGL((k_row_fwd<N1, N2, SLOTS, NB_HALF, kEditNone>), grid, blk, 0, s, a);
          else hipLaunchKernelGGL((k_row_fwd<N1, N2, SLOTS, N1, kEditNone>), grid, blk, 0, s, a);
      }
      return hipGetLastError();
    }
  }
  static hipError_t inv(const RowInvArgs& a, int B, hipStream_t s) {
    const int slots_needed = a.npairs;
    dim3 grid((slots_needed + SLOTS - 1) / SLOTS, B);
    const bool half = 2 * a.W <= N1 * N2;
    if (a.mom)
      hipLaunchKernelGGL((k_row_inv<N1, N2, SLOTS, true>), grid, dim3(SLOTS * C::G), 0, s, a);
    else if (half)
      hipLaunchKernelGGL((k_row_inv<N1, N2, SLOTS, false, kInvHalf<N1>>), grid,
                         dim3(SLOTS * C::G), 0, s, a);
    else
      hipLaunchKernelGGL((k_row_inv<N1, N2, SLOTS, false>), grid, dim3(SLOTS * C::G), 0, s, a);
    return hipGetLastError();
  }
  static hipError_t bfwd(const RowBwdFwdArgs& a, int B, hipStream_t s) {
    const int slots_needed = a.npairs;
    dim3 grid((slots_needed + SLOTS - 1) / SLOTS, B);
    if (2 * a.W <= N1 * N2)
      hipLaunchKernelGGL((k_row_bfwd<N1, N2, SLOTS, kInvHalf<N1>>), grid, dim3(SLOTS * C::G), 0,
                         s, a);
    else
      hipLaunchKernelGGL((k_row_bfwd<N1, N2, SLOTS>), grid, dim3(SLOTS * C::G), 0, s, a);
    return hipGetLastError();
  }
  static hipError_t binv(const RowBwdInvArgs& a, int B, hipStream_t s) {
    dim3 grid((a.H + SLOTS - 1) / SLOTS, B);  // one row per slot
    if (2 * a.W <= N1 * N2)
      hipLaunchKernelGGL((k_row_binv<N1, N2, SLOTS, kInvHalf<N1>>), grid, dim3(SLOTS * C::G), 0,
                         s, a);
    else
      hipLaunchKernelGGL((k_row_binv<N1, N2, SLOTS>), grid, dim3(SLOTS * C::G), 0, s, a);
    return hipGetLastError();
  }
  // half: every image of the launch has 2 W <= N
  static hipError_t rg_fwd(const RgBase* base, const RgRowFwd* tab, const RgItem* items,
                           int nitems, bool half, hipStream_t s) {
    if (half)
      hipLaunchKernelGGL((k_row_fwd_rg<N1, N2, SLOTS, NB_HALF>), dim3(nitems),
                         dim3(SLOTS * C::G), 0, s, base, tab, items);
    else
      hipLaunchKernelGGL((k_row_fwd_rg<N1, N2, SLOTS, N1>), dim3(nitems), dim3(SLOTS * C::G),
                         0, s, base, tab, items);
    return hipGetLastError();
  }
  static hipError_t rg_inv(const RgBase* base, const RgRowInv* tab, const RgItem* items,
                           int nitems, bool half, hipStream_t s) {
    if (half)
      hipLaunchKernelGGL((k_row_inv_rg<N1, N2, SLOTS, kInvHalf<N1>>), dim3(nitems),
                         dim3(SLOTS * C::G), 0, s, base, tab, items);
    else
      hipLaunchKernelGGL((k_row_inv_rg<N1, N2, SLOTS>), dim3(nitems), dim3(SLOTS * C::G), 0, s,
                         base, tab, items);
    return hipGetLastError();
  }
};

// ---------------------------------------------------------------------------------------
// Ragged batches with many row lengths: one launch runs the items of several lengths, each
// workgroup branching (uniformly) on its image's N to that length's body. A launch costs a
// few microseconds of latency however small it is, so a batch of 49 lengths issued per
// length spends most of its time in launch tails; grouping lengths of one workgroup size
// cuts the launches per row pass to a handful. The LDS is the largest of the lengths'; the
// registers are the most any of them needs. Only the half-support forward variant (2 W <= N,
// every default torus) is grouped.
template <int F1, int F2, int I1, int I2>
struct RowLen {
  // forward row pass with the split F1 x F2, inverse with I1 x I2 (N = F1 F2 = I1 I2)
  static constexpr int N = F1 * F2;
  static_assert(I1 * I2 == N, "one row length per entry");
  static constexpr int FSLOTS = RowLaunch<F1, F2>::SLOTS, ISLOTS = RowLaunch<I1, I2>::SLOTS;
  static constexpr int NBH = RowLaunch<F1, F2>::NB_HALF;
  static constexpr int THREADS = FSLOTS * RowCfg<F1, F2>::G;
  static_assert(ISLOTS * RowCfg<I1, I2>::G == THREADS, "one workgroup size per entry");
  static constexpr int FWD_LDS = kFwdLds<F1, F2, FSLOTS>;
  static constexpr int INV_LDS = kInvLds<I1, I2, ISLOTS>;
  static constexpr int FN1 = F1, FN2 = F2, IN1 = I1, IN2 = I2;
};
constexpr int cmax_n(int a) { return a; }
template <class... T>
constexpr int cmax_n(int a, int b, T... r) { return cmax_n(cmax(a, b), r...); }

// Groups whose forward entries all have N1 <= 40 are held to three wavefronts per SIMD (168
// registers): left alone the compiler took 172-175 for two of them and ran two. The group
// of lengths 1500-2048 then spills 20 bytes per lane and still makes the 200-image uneven
// batch about 1 % faster; groups with larger N1 would spill far more and keep the default.
template <class L0, class... Ls>
constexpr int kRgmFwdWaves = cmax_n(L0::FN1, Ls::FN1...) <= 40 ? 3 : 1;

template <class L0, class... Ls>
__global__ void __launch_bounds__(L0::THREADS)
__attribute__((amdgpu_waves_per_eu(kRgmFwdWaves<L0, Ls...>)))
k_row_fwd_rgm(const RgBase* basep, const RgRowFwd* tab, const RgItem* items) {
  const RgBase base = *basep;  // written by launch_set_base on this stream
  static_assert(((Ls::THREADS == L0::THREADS) && ...), "one workgroup size per launch");
  constexpr int NL = cmax_n(L0::FWD_LDS, Ls::FWD_LDS...);
  __shared__ float lds[NL];
  const RgItem it = items[blockIdx.x];
  const RgRowFwd& e = tab[it.img];
  RowFwdArgs p = e.a;
  p.gx = base.gx + e.in;
  p.gy = base.gy + e.in;
  p.T1 = reinterpret_cast<f2*>(base.ws + e.t);
  p.SB = reinterpret_cast<f2*>(base.ws + e.side);
  const int n = p.N;
  (void)((n == L0::N && (row_fwd_body<L0::FN1, L0::FN2, L0::FSLOTS, L0::NBH>(p, it.blk, 0, lds),
                         true)) ||
         ... ||
         (n == Ls::N && (row_fwd_body<Ls::FN1, Ls::FN2, Ls::FSLOTS, Ls::NBH>(p, it.blk, 0, lds),
                         true)));
}

template <class L0, class... Ls>
__global__ void __launch_bounds__(L0::THREADS)
k_row_inv_rgm(const RgBase* basep, const RgRowInv* tab, const RgItem* items) {
  const RgBase base = *basep;  // written by launch_set_base on this stream
  constexpr int NL = cmax_n(L0::INV_LDS, Ls::INV_LDS...);
  __shared__ float lds[NL];
  const RgItem it = items[blockIdx.x];
  const RgRowInv& e = tab[it.img];
  RowInvArgs p = e.a;
  p.T2 = reinterpret_cast<const f2*>(base.ws + e.t);
  p.u = base.u + e.out;
  p.partial = reinterpret_cast<const double*>(base.ws + e.red);
  const int n = p.N;
  // every image of a group has 2 W <= N: only the output blocks that can hold x < W
  (void)((n == L0::N &&
          (row_inv_body<L0::IN1, L0::IN2, L0::ISLOTS, false, kInvHalf<L0::IN1>>(p, it.blk, 0, lds),
           true)) ||
         ... ||
         (n == Ls::N &&
          (row_inv_body<Ls::IN1, Ls::IN2, Ls::ISLOTS, false, kInvHalf<Ls::IN1>>(p, it.blk, 0, lds),
           true)));
}

template <class L0, class... Ls>
struct RowMulti {
  static hipError_t fwd(const RgBase* base, const RgRowFwd* tab, const RgItem* items,
                        int nitems, hipStream_t s) {
    hipLaunchKernelGGL((k_row_fwd_rgm<L0, Ls...>), dim3(nitems), dim3(L0::THREADS), 0, s, base,
                       tab, items);
    return hipGetLastError();
  }
  static hipError_t inv(const RgBase* base, const RgRowInv* tab, const RgItem* items,
                        int nitems, hipStream_t s) {
    hipLaunchKernelGGL((k_row_inv_rgm<L0, Ls...>), dim3(nitems), dim3(L0::THREADS), 0, s, base,
                       tab, items);
    return hipGetLastError();
  }
};

template <int N1, int N2>
constexpr RowSplit row_split() {
  return RowSplit{N1, N2, RowCfg<N1, N2>::G, RowLaunch<N1, N2>::SLOTS};
}

// The forward row pass: the plain solve with the split F1 x F2, the other input modes
// (gradient edits, a given Laplacian, volume slices) with E1 x E2 (each mode's fastest split
// differs: its loader holds other values through the first FFT stage).
template <int F1, int F2, int E1, int E2>
struct RowFwdModes {
  static hipError_t fwd(const RowFwdArgs& a, int B, hipStream_t s) {
    if (a.edit == kEditNone) return RowLaunch<F1, F2, false>::fwd(a, B, s);
    return RowLaunch<E1, E2>::fwd(a, B, s);
  }
};

// One row length with its own split per pass: plain forward (f1 x f2), the other forward
// modes (e1 x e2), inverse (i1 x i2), backward forward (b1 x b2) and backward inverse
// (c1 x c2) row transforms.
#define GFC_ROW_ENTRY(f1, f2, e1, e2, i1, i2, b1, b2, c1, c2)                                \
  RowKernels{f1 * f2, row_split<f1, f2>(), row_split<e1, e2>(), row_split<i1, i2>(),        \
             row_split<b1, b2>(), row_split<c1, c2>(), &RowFwdModes<f1, f2, e1, e2>::fwd,    \
             &RowLaunch<i1, i2>::inv, &RowLaunch<b1, b2>::bfwd, &RowLaunch<c1, c2>::binv,    \
             &RowLaunch<f1, f2>::rg_fwd, &RowLaunch<i1, i2>::rg_inv}
// A candidate split for the autotuner: every pass with n1 x n2, the plain passes only.
#define GFC_ROW_ENTRY_CANDIDATE(n1, n2)                                                       \
  RowKernels{n1 * n2, row_split<n1, n2>(), row_split<n1, n2>(), row_split<n1, n2>(),        \
             row_split<n1, n2>(), row_split<n1, n2>(), &RowLaunch<n1, n2, false>::fwd,      \
             &RowLaunch<n1, n2, false>::inv, &RowLaunch<n1, n2, false>::bfwd,               \
             &RowLaunch<n1, n2, false>::binv, nullptr, nullptr}

}  // namespace gfc
