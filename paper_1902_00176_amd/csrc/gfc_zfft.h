// gfc_zfft.h - FFTs along z for volumes: the third axis of the n-D solve (eq. (5) holds in
// any dimension). The spectra of a volume are P planes of R x NHP (z, row y, row frequency l),
// each tile-major as the images are (side arrays row-major); the transform runs over z for
// every (y, l). A workgroup takes one row y and TL <= 16 consecutive l, contiguous within
// a tile: coalesced loads of TL * 8 bytes per plane into LDS, one four-step FFT of length
// P = P1 * P2 per slot of G lanes (as the row passes), coalesced stores.
#pragma once
#include "gfc_buf.h"
#include "gfc_dft.h"
#include "gfc_internal.h"
#include "gfc_twiddle.h"

namespace gfc {

// A byte offset past every volume's spectra, which plans keep below 2^31 bytes: loads at it
// return zero.
constexpr int kZOob = 0x7ffffff8;

template <int P1, int P2>
struct ZCfg {
  static constexpr int P = P1 * P2;
  static constexpr int G = P1 > P2 ? (P1 <= 8 ? 8 : P1 <= 16 ? 16 : P1 <= 32 ? 32 : 64)
                                   : (P2 <= 8 ? 8 : P2 <= 16 ? 16 : P2 <= 32 ? 32 : 64);
  static constexpr int SA = (P2 % 2 == 0) ? P2 + 1 : P2;  // odd LDS stride of the transpose
  static constexpr int S = (P1 * SA > P) ? P1 * SA : P;     // floats per plane per slot
  static constexpr int TL = (2 * S * 4 * 16 <= 48 * 1024) ? 16 : 8;  // columns per workgroup
};

// din input planes (the rest are zero) -> dout output planes; SIGN -1 forward, +1 inverse
// (unnormalised). In place: every column is read completely before it is written.
template <int P1, int P2, int SIGN>
__global__ void __launch_bounds__((ZCfg<P1, P2>::TL * ZCfg<P1, P2>::G))
k_zfft(ZfftArgs a) {
  using C = ZCfg<P1, P2>;
  constexpr int P = C::P, G = C::G, TL = C::TL, NT = TL * G;
  // one column per row of s_lds; the odd row length puts the TL columns of one plane in
  // different banks for the coalesced load and store phases
  __shared__ float s_lds[TL][2 * C::S + 1];
  const int t = threadIdx.x;
  const int y = blockIdx.y, vol = blockIdx.z;
  const int l0 = blockIdx.x * TL;
  const rsrc_t rT = make_buf(a.T + vol * a.vol_stride, a.vol_stride * 8);
  const rsrc_t rtw = make_buf(a.tw, (long long)P * 8);

  // 1. coalesced load of the column tile: thread -> (plane z, column c). All of a thread's
  // loads are issued before the first is stored to LDS (a loop of load, wait, store paid a
  // memory latency per plane group).
  constexpr int NLD = (TL * P + NT - 1) / NT;  // elements per thread
  f2b v[NLD];
#pragma unroll
  for (int k = 0; k < NLD; ++k) {
    // element k of every thread lies in planes [k G, k G + G): past din, all read 0
    v[k] = f2b{0.f, 0.f};
    if (k * G < a.din) {
      const int i = t + k * NT;
      const int c = i % TL, z = i / TL;
      const int l = l0 + c;
      const bool in = i < TL * P && z < a.din && l < a.NH;
      const long long e =
          (long long)z * a.plane + (a.tiled ? tile_index(y, l, a.R) : y * a.NHP + l);
      v[k] = bld2(rT, in ? int(e * 8) : kZOob, 0);
    }
  }
#pragma unroll
  for (int k = 0; k < NLD; ++k) {
    const int i = t + k * NT;
    if (i < TL * P) {
      s_lds[i % TL][i / TL] = v[k].x;
      s_lds[i % TL][C::S + i / TL] = v[k].y;
    }
  }
  __syncthreads();

  // 2. one FFT per slot (column c); lane j holds z = P2 * y1 + j, y1 < P1
  const int c = t / G, j = t % G;
  float* re = s_lds[c];
  float* im = s_lds[c] + C::S;
  cx x[P1];
  if (j < P2) {
#pragma unroll
    for (int y1 = 0; y1 < P1; ++y1) x[y1] = {re[P2 * y1 + j], im[P2 * y1 + j]};
  }
  __syncthreads();
  if (j < P2) {
    DftSel<P1, SIGN>::run(x);
    // w_P^(k1 j), forward sign (conjugated for the inverse); the forward transform runs on
    // the divergence, whose lowest frequencies the solve amplifies: exact table twiddles
    twiddles<P1, P2, (SIGN < 0)>(rtw, j, 0, [&](int k1, cx w) {
      x[k1] = SIGN < 0 ? cmul(x[k1], w) : cmulconj(x[k1], w);
    });
#pragma unroll
    for (int k1 = 0; k1 < P1; ++k1) {
      re[k1 * C::SA + j] = x[k1].x;
      im[k1 * C::SA + j] = x[k1].y;
    }
  }
  __syncthreads();
  cx b[P2];
  if (j < P1) {
#pragma unroll
    for (int jj = 0; jj < P2; ++jj) b[jj] = {re[j * C::SA + jj], im[j * C::SA + jj]};
    DftSel<P2, SIGN>::run(b);
  }
  __syncthreads();
  if (j < P1) {
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) {  // output index k = k1 + P1 k2 with k1 = j
      re[j + P1 * k2] = b[k2].x;
      im[j + P1 * k2] = b[k2].y;
    }
  }
  __syncthreads();

  // 3. coalesced store of the first dout planes (dout <= P)
#pragma unroll
  for (int k = 0; k < NLD; ++k) {
    const int i = t + k * NT;
    const int cc = i % TL, z = i / TL;
    const int l = l0 + cc;
    if (i < TL * a.dout && l < a.NH)
      bst2(rT, s_lds[cc][z], s_lds[cc][C::S + z],
           int(((long long)z * a.plane +
                (a.tiled ? tile_index(y, l, a.R) : y * a.NHP + l)) * 8), 0);
  }
}

template <int P1, int P2>
struct ZLaunch {
  using C = ZCfg<P1, P2>;
  static hipError_t run(const ZfftArgs& a, int sign, int B, hipStream_t s) {
    const dim3 grid((a.NH + C::TL - 1) / C::TL, a.R, B), blk(C::TL * C::G);
    if (sign < 0) hipLaunchKernelGGL((k_zfft<P1, P2, -1>), grid, blk, 0, s, a);
    else hipLaunchKernelGGL((k_zfft<P1, P2, +1>), grid, blk, 0, s, a);
    return hipGetLastError();
  }
};

#define GFC_Z_ENTRY(p1, p2) ZKernels{p1 * p2, p1, p2, &ZLaunch<p1, p2>::run}

}  // namespace gfc
