// gfc_col.hip - column pass of the GFC solve.
//
// After the row transforms, each column frequency l is an independent 1-D problem along
// the image's y axis: apply the column slice of the Green's spectrum, 1/lambda(k, l) with
// lambda(k, l) = -4 sin^2(pi k/M) - beta_l, beta_l = 4 sin^2(pi l/N), to a column that is
// nonzero only on the first R rows of the M-periodic axis (eqs. (22)-(23) restricted to
// one column). Because 1/lambda(., l) is the symbol of (D_yy - beta_l)^-1, it factors as
//     -rho (1 - rho S^-1)^-1 (1 - rho S)^-1,   rho + 1/rho = 2 + beta_l,  rho < 1,
// S the unit shift on Z_M. The kernel applies that factorisation exactly: a causal and an
// anticausal first-order recursion in float64 with the periodic wrap-around in closed form.
// Column 0 (beta = 0, where lambda(0,0) = 0) is the pseudo-inverse: a cumulative sum.
//
// Layout: one thread per (column, row segment); a workgroup owns C adjacent columns of one
// image and all of their segments, so consecutive lanes read consecutive columns (C*8
// contiguous bytes per row). Each thread loads its segment once and keeps it in registers:
//   1. causal sweep of the segment from a zero state (float64): end state e_t, moment mu_t;
//   2. every thread derives its own carries from the other segments' (e, mu) in LDS. The
//      carries are sums of terms weighted by rho^distance; terms further than kseg segments
//      away weigh less than 2^-64 and are left out, so for all but the lowest columns this
//      reads a handful of LDS entries and there is no serial scan over the column;
//   3. anticausal sweep over the registers, result stored in place.
// Global accesses go through buffer descriptors whose range is one image: rows past the
// input read as 0 and stores past the output are dropped by the hardware.
#include <algorithm>

#include "gfc_buf.h"
#include "gfc_internal.h"

namespace gfc {

struct dc {
  double x, y;
};

constexpr int kOOB = 0x40000000;  // a per-lane byte offset past every image buffer

__device__ __forceinline__ dc dadd(dc a, dc b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ dc dscale(dc a, double s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ dc dfma(double s, dc a, dc b) {  // s*a + b
  return {__builtin_fma(s, a.x, b.x), __builtin_fma(s, a.y, b.y)};
}
__device__ __forceinline__ dc dsel(bool c, dc a, dc b) { return {c ? a.x : b.x, c ? a.y : b.y}; }
// keeps the compiler from converting all register-held values to float64 at once
__device__ __forceinline__ void pin(f2b& v) { asm volatile("" : "+v"(v.x), "+v"(v.y)); }

// LDS entries loaded together in the carry sums (HC below): the forward pass takes 8; the
// backward pass, which holds more state beside its segment, takes 4 (with 8 it spilled 8
// registers and ran 3 % slower; the forward pass ran 2 % slower with 4)
constexpr int kHornerFwd = 8, kHornerBwd = 4;

// acc <- sum_{t in [t0, t1)} r^(t1-1-t) A[t*C + c] (Horner from t0 upwards); the loads of a
// chunk are issued together so the chain waits on LDS once per chunk, not per entry
template <int HC>
__device__ __forceinline__ dc horner_up(const dc* A, int C, int c, int t0, int t1, double r,
                                        dc acc) {
  int t = t0;
  for (; t + HC <= t1; t += HC) {
    dc e[HC];
#pragma unroll
    for (int q = 0; q < HC; ++q) e[q] = A[(t + q) * C + c];
#pragma unroll
    for (int q = 0; q < HC; ++q) acc = dfma(r, acc, e[q]);
  }
  for (; t < t1; ++t) acc = dfma(r, acc, A[t * C + c]);
  return acc;
}

// acc <- sum_{t in (t0, t1]} r^(t-t0-1) A[t*C + c] + r^(t1-t0) acc (Horner from t1 down)
template <int HC>
__device__ __forceinline__ dc horner_down(const dc* A, int C, int c, int t1, int t0, double r,
                                          dc acc) {
  int t = t1;
  for (; t - HC >= t0; t -= HC) {
    dc e[HC];
#pragma unroll
    for (int q = 0; q < HC; ++q) e[q] = A[(t - q) * C + c];
#pragma unroll
    for (int q = 0; q < HC; ++q) acc = dfma(r, acc, e[q]);
  }
  for (; t > t0; --t) acc = dfma(r, acc, A[t * C + c]);
  return acc;
}

// Carry into segment s from the segments before it: sum over t < s of
// rho^(Lseg (s-1-t)) e_t (every segment before the last is Lseg rows), over at most kseg
// segments. rp returns rho^(Lseg s) when the sum is exact (s <= kseg), else 0.
template <int HC>
__device__ __forceinline__ dc carry_in(const dc* E, int C, int c, int s, int kseg, double rhoL,
                                       double& rp) {
  const int t0 = s > kseg ? s - kseg : 0;
  double r = 1.0;
  for (int t = 0; t < s && t <= kseg; ++t) r *= rhoL;
  rp = s > kseg ? 0.0 : r;
  return horner_up<HC>(E, C, c, t0, s, rhoL, dc{0.0, 0.0});
}

// z at the row after segment s (anticausal carry) from the moments zst_t of the later
// segments and z[Rp] = ZR: Z_s = sum_{t > s} rho^(p_t - p_{s+1}) zst_t + rho^(Rp - p_{s+1}) ZR.
template <int HC>
__device__ __forceinline__ dc carry_out(const dc* U, int C, int c, int s, int last, int kseg,
                                        double rhoL, double rhoLl, dc ZR) {
  if (s == last) return ZR;
  if (s + kseg < last) return horner_down<HC>(U, C, c, s + kseg, s, rhoL, dc{0.0, 0.0});
  const dc acc = dfma(rhoLl, ZR, U[last * C + c]);  // z at the start of the last segment
  return horner_down<HC>(U, C, c, last - 1, s, rhoL, acc);
}

// sum_t rho^(Lseg t) zst_t over the first kseg + 1 segments
template <int HC>
__device__ __forceinline__ dc head_moment(const dc* U, int C, int c, int last, int kseg,
                                          double rhoL) {
  const int tmax = kseg < last ? kseg : last;
  return horner_down<HC>(U, C, c, tmax - 1, -1, rhoL, U[tmax * C + c]);
}

// ---------------------------------------------------------------------------------------
// Forward: input rows [0, R), R = H + 1; outputs rows [0, H) and per-column reference terms.
// Columns l <= K arrive split: T holds a = (1 - w_N^l) Ex^ and SB holds b = Ey^, and the
// column input is a + (1 - S) b. The difference is folded into the causal recursion:
// (1 - rho S)^-1 (1 - S) b = b - (1 - rho) S (1 - rho S)^-1 b, which has no cancellation.
// The recursion constants of columns [l0, l0 + C) into LDS (columns past nh read 0), four
// words in flight per thread; visible after the caller's next barrier. The passes read
// them after their barriers, where each read from global memory (an L2 round trip) would
// stall the workgroup again.
constexpr int kColMaxC = 64;  // widest column tile (plans keep col_c <= 64)
__device__ __forceinline__ void stage_consts(ColConst* dst, const ColConst* tab, int l0, int C,
                                             int nh) {
  constexpr int kW = int(sizeof(ColConst) / 8);
  const int nw = C * kW;
  const int have = (nh - l0 < C ? nh - l0 : C) * kW;
  const rsrc_t r = make_buf(tab + l0, (long long)(have > 0 ? have : 0) * 8);
  double* d = reinterpret_cast<double*>(dst);
  const int nt = int(blockDim.x);
  for (int w0 = 0; w0 < nw; w0 += 4 * nt) {
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      v[k] = __builtin_bit_cast(double, bld2(r, (w0 + int(threadIdx.x) + k * nt) * 8, 0));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int w = w0 + int(threadIdx.x) + k * nt;
      if (w < nw) d[w] = v[k];
    }
  }
}

template <int LMAX, bool LOWTILE, bool TAIL, int CP>
__device__ __forceinline__ void col_fwd_tile(const ColFwdArgs& p, int tile, int b, dc* E,
                                             dc* U, ColConst* s_cc) {
  const int C = p.C;
  const int cl = __builtin_ctz(C);
  const int nseg = p.nseg;
  const int last = nseg - 1;
  const int c = threadIdx.x & (C - 1);
  const int s = threadIdx.x >> cl;
  const bool active = s < nseg;
  const int l = tile * C + c;
  const bool col_ok = active && l < p.NH;
  // volumes: image b is plane kz of a volume; only (kz, l) = (0, 0) is the DC column
  const int kz = p.zp > 1 ? b % p.zp : 0;
  const bool dcol = LOWTILE && col_ok && l == 0 && kz == 0;
  const bool low = LOWTILE && col_ok && l <= p.K;
  const int p0 = s * LMAX;
  const int Ls = (TAIL && s == last) ? p.Llast : LMAX;

  const rsrc_t rT = make_buf(p.T + b * p.img_t, p.img_t * 8);
  // tile-major spectra: a thread's rows are 128 bytes apart; rows past the image's H + 1
  // (the widened last segment) would be the next tile's, so they take out-of-range offsets
  const int RT = p.H + 1;
  const int rowT = kTileBins * 8;
  const int vT = col_ok ? tile_index(p0, l, RT) * 8 : kOOB;
  const int vX = (col_ok && !dcol) ? vT : kOOB;  // column 0 has a = 0
  const int nin = RT - p0;  // rows of the segment inside the image

  // the causal sweep reads its constants from the table; the later phases from the copy in
  // LDS that the loads below overlap
  const ColConst* kg = p.cc + kz * p.NH + (col_ok ? l : 0);
  const ColConst* kp = s_cc + c;
  const double rho = dcol ? 1.0 : kg->rho;

  // ---- 1. load the segment, causal sweep from a zero state ----
  f2b v[LMAX];
#pragma unroll
  for (int j = 0; j < LMAX; ++j) v[j] = bld2<CP>(rT, j < nin ? vX + j * rowT : kOOB, 0);
  stage_consts(s_cc, p.cc + kz * p.NH, tile * C, C, p.NH);
  dc e = {0.0, 0.0}, mu = {0.0, 0.0};
  if (LOWTILE && low) {
    const rsrc_t rS = make_buf(p.SB + b * p.img_sb, p.img_sb * 8);
    const int rowS = p.KP * 8;
    const int vS = (p0 * p.KP + l) * 8;
    const double omr = kg->omr;
    if (dcol) {
      // column 0: the running sum of b; v gets the exclusive prefix
      dc st = {0.0, 0.0};
#pragma unroll
      for (int j = 0; j < LMAX; ++j) {
        const f2b bb = bld2(rS, vS + j * rowS, 0);
        v[j] = f2b{float(st.x), float(st.y)};
        pin(v[j]);
        st = {st.x + bb.x, st.y + bb.y};
      }
      e = st;
    } else {
      // the segment's first row carries -b[p0-1]: seeding the causal state of b with
      // b[p0-1] / (1 - rho) makes (1 - rho) * sbb reproduce it without a cancellation
      dc sbb = {0.0, 0.0};
      if (p0 > 0) {
        const f2b bp = bld2(rS, vS - rowS, 0);
        sbb = {double(bp.x) / omr, double(bp.y) / omr};
      }
      dc sa = {0.0, 0.0}, st = {0.0, 0.0};
      double pw = 1.0;
#pragma unroll
      for (int j = 0; j < LMAX; ++j) {
        const f2b bb = bld2(rS, vS + j * rowS, 0);
        pin(v[j]);
        sa = dfma(rho, sa, dc{v[j].x, v[j].y});
        st = {sa.x + bb.x - omr * sbb.x, sa.y + bb.y - omr * sbb.y};
        sbb = dfma(rho, sbb, dc{bb.x, bb.y});
        v[j] = f2b{float(st.x), float(st.y)};
        pin(v[j]);
        if (TAIL) {
          mu = dfma(j < Ls ? pw : 0.0, st, mu);
          e = dsel(j == Ls - 1, st, e);
        } else {
          mu = dfma(pw, st, mu);
        }
        pw *= rho;
      }
      if (!TAIL) e = st;
    }
  } else {
    dc st = {0.0, 0.0};
    double pw = 1.0;
#pragma unroll
    for (int j = 0; j < LMAX; ++j) {
      pin(v[j]);
      st = dfma(rho, st, dc{v[j].x, v[j].y});
      v[j] = f2b{float(st.x), float(st.y)};
        pin(v[j]);
      if (TAIL) {
        mu = dfma(j < Ls ? pw : 0.0, st, mu);
        e = dsel(j == Ls - 1, st, e);
      } else {
        mu = dfma(pw, st, mu);
      }
      pw *= rho;
    }
    if (!TAIL) e = st;
  }
  if (active) {
    E[s * C + c] = e;
    U[s * C + c] = mu;
  }
  __syncthreads();

  // ---- 2. carries ----
  dc D = {0.0, 0.0};      // column 0: prefix before the segment; else rho C_s + rho^p_s gamma
  dc wR1 = {0.0, 0.0};
  double bbar = 0.0, term = 0.0;
  if (col_ok) {
    if (dcol) {
      double pre = 0.0, tot = 0.0;
#pragma unroll 8
      for (int t = 0; t < nseg; ++t) {
        const double x = E[t * C + c].x;
        pre += t < s ? x : 0.0;
        tot += x;
      }
      bbar = tot / double(p.M);
      D = {pre, 0.0};
      term = (tot - double(p.r0) * bbar) * kp->outs;
    } else {
      const int kseg = kp->kseg;
      const double rhoL = kp->rhoL;
      double rp, rl;
      const dc Cs = carry_in<kHornerFwd>(E, C, c, s, kseg, rhoL, rp);
      const dc Cl = carry_in<kHornerFwd>(E, C, c, last, kseg, rhoL, rl);
      const dc cR1 = dfma(kp->rhoLl, Cl, E[last * C + c]);  // c0[Rp-1]
      const dc gam = dscale(cR1, kp->cg);
      D = dfma(rp, gam, dscale(Cs, rho));
      wR1 = dfma(kp->rhoRm1, gam, cR1);
      const dc zst = dfma(s == last ? kp->gLl : kp->gL, D, mu);
      U[s * C + c] = zst;  // only this thread reads its own mu
    }
  }
  __syncthreads();

  // ---- 3. anticausal sweep from registers ----
  // fresh row offsets (recomputed rather than kept live across the carries)
  int vS3 = vT;
  asm volatile("" : "+v"(vS3));
  if (col_ok) {
    if (dcol) {
      const double outs = kp->outs;
#pragma unroll
      for (int j = 0; j < LMAX; ++j) {
        pin(v[j]);
        const double y = double(p0 + j);
        const double val = (D.x + double(v[j].x) - bbar * y) * outs;
        bst2<CP>(rT, float(val), 0.f, j < nin ? vS3 + j * rowT : kOOB, 0);
      }
    } else {
      const int kseg = kp->kseg;
      const double rhoL = kp->rhoL, rhoLl = kp->rhoLl;
      const dc Sw = head_moment<kHornerFwd>(U, C, c, last, kseg, rhoL);
      const dc ZR = dfma(kp->cT, wR1, dscale(Sw, kp->czR));  // z[Rp]
      dc z = carry_out<kHornerFwd>(U, C, c, s, last, kseg, rhoL, rhoLl, ZR);
      if (s == 0) {
        const dc z0 = dfma(last == 0 ? rhoLl : rhoL, z, U[c]);  // z[0]
        const dc zr0 = dfma(kp->ra, wR1, dscale(z0, kp->rb));
        term = kp->wre * zr0.x - kp->wim * zr0.y;
      }
      const double inv_rho = kp->inv_rho;
      const double outs = kp->outs;
      double pj = rhoL * inv_rho;  // rho^j at row j, from j = LMAX - 1
#pragma unroll
      for (int j = LMAX - 1; j >= 0; --j) {
        pin(v[j]);
        const dc w = dfma(pj, D, dc{v[j].x, v[j].y});
        if (TAIL) z = dsel(j < Ls, dfma(rho, z, w), z);
        else z = dfma(rho, z, w);
        bst2<CP>(rT, float(z.x * outs), float(z.y * outs), j < nin ? vS3 + j * rowT : kOOB, 0);
        pj *= inv_rho;
      }
    }
  }
  // per-tile reference partial: the s == 0 threads are lanes [0, C) of wave 0, every other
  // lane of wave 0 holds 0; a fixed-order butterfly keeps the sum deterministic
  if (threadIdx.x < 64) {
    double t = s == 0 ? term : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    if (threadIdx.x == 0) p.partial[(long long)b * p.nparts + tile] = t;
  }
}

template <int LMAX, bool LOWTILE, bool TAIL, int CP>
__global__ void __launch_bounds__(kColMaxThreads) k_col_fwd(ColFwdArgs p) {
  extern __shared__ dc s_mem[];
  __shared__ ColConst s_cc[kColMaxC];
  col_fwd_tile<LMAX, LOWTILE, TAIL, CP>(p, p.tile0 + blockIdx.x, blockIdx.y, s_mem,
                                    s_mem + p.nseg * p.C, s_cc);
}

// ragged batches: one (image, tile) work item per workgroup, the image's arguments from a
// table with workspace addresses as offsets; the workgroup shape is the largest over the
// images (threads past an image's C * nseg idle through the barriers)
template <int LMAX, bool LOWTILE, bool TAIL>
__global__ void __launch_bounds__(kColMaxThreads)
k_col_fwd_rg(const RgBase* basep, const RgCol* tab, const RgItem* items) {
  const RgBase base = *basep;  // written by launch_set_base on this stream
  extern __shared__ dc s_mem[];
  const RgItem it = items[blockIdx.x];
  const RgCol& e = tab[it.img];
  ColFwdArgs p = e.a;
  p.T = reinterpret_cast<f2*>(base.ws + e.t);
  p.SB = reinterpret_cast<const f2*>(base.ws + e.side);
  p.partial = reinterpret_cast<double*>(base.ws + e.red);
  __shared__ ColConst s_cc[kColMaxC];
  col_fwd_tile<LMAX, LOWTILE, TAIL, kNT>(p, it.blk, 0, s_mem, s_mem + p.nseg * p.C, s_cc);
}

// The same over the low-column items followed by the other items in one launch: the first
// nlow workgroups take the split-input path (a workgroup-uniform branch), so within one
// stream the long low-column carries run beside the other tiles instead of before them.
template <int LMAX, bool TAIL>
__global__ void __launch_bounds__(kColMaxThreads)
k_col_fwd_rg_all(const RgBase* basep, const RgCol* tab, const RgItem* items, int nlow) {
  const RgBase base = *basep;  // written by launch_set_base on this stream
  extern __shared__ dc s_mem[];
  const RgItem it = items[blockIdx.x];
  const RgCol& e = tab[it.img];
  ColFwdArgs p = e.a;
  p.T = reinterpret_cast<f2*>(base.ws + e.t);
  p.SB = reinterpret_cast<const f2*>(base.ws + e.side);
  p.partial = reinterpret_cast<double*>(base.ws + e.red);
  __shared__ ColConst s_cc[kColMaxC];
  if (int(blockIdx.x) < nlow)
    col_fwd_tile<LMAX, true, TAIL, kNT>(p, it.blk, 0, s_mem, s_mem + p.nseg * p.C, s_cc);
  else
    col_fwd_tile<LMAX, false, TAIL, kNT>(p, it.blk, 0, s_mem, s_mem + p.nseg * p.C, s_cc);
}

// ---------------------------------------------------------------------------------------
// Backward: input rows [0, R), R = H, plus a Dirac of weight dv = -sum(du) w_N^(l c0) at
// row r0 (the adjoint of the reference-pixel subtraction). Outputs w rows [0, H] and, for
// l <= Kb, the column derivative (-D_y w)[y] = w_in[y] - (1 - rho) z[y+1] scaled like w.
template <int LMAX, bool LOWTILE, bool TAIL, int CP>
__device__ __forceinline__ void col_bwd_tile(const ColBwdArgs& p, int tile, int b, dc* E,
                                             dc* U, double* s_misc, ColConst* s_cc) {
  const int C = p.C;
  const int cl = __builtin_ctz(C);
  const int nseg = p.nseg;
  const int last = nseg - 1;
  const int c = threadIdx.x & (C - 1);
  const int s = threadIdx.x >> cl;
  const bool active = s < nseg;
  const int l = tile * C + c;
  const bool col_ok = active && l < p.NH;
  const bool dcol = LOWTILE && col_ok && l == 0;
  const bool low = LOWTILE && col_ok && l <= p.Kb;
  const int p0 = s * LMAX;
  const int Ls = (TAIL && s == last) ? p.Llast : LMAX;
  const int R = p.H;

  // tile-major spectra (see the forward pass); loads see the H input rows only (row H of the
  // buffer is an output row), stores the H + 1 output rows
  const rsrc_t rT = make_buf(p.T + b * p.img_t, p.img_t * 8);
  const rsrc_t rD = make_buf(p.SD + b * p.img_sd, p.img_sd * 8);
  const int RT = p.H + 1;
  const int rowT = kTileBins * 8;
  const int nin = R - p0, nout = RT - p0;  // input and output rows of the segment
  const int rowD = p.KbP * 8;
  const int vT = col_ok ? tile_index(p0, l, RT) * 8 : kOOB;
  const int vD = low ? (p0 * p.KbP + l) * 8 : kOOB;

  // the causal sweep reads rho from the table; the later phases their constants from the
  // copy in LDS that the loads below overlap
  const ColConst* kp = s_cc + c;
  const double rho = dcol ? 1.0 : p.cc[col_ok ? l : 0].rho;

  // sum(du) from the row pass's partials: wave 0 reduces them (lane-strided sums, then a
  // fixed-order butterfly) and leaves the total in LDS for after the first barrier
  if (threadIdx.x < 64) {
    double S = strided_sum<64, 8>(p.sums + (long long)b * p.nsums, p.nsums, threadIdx.x);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) S += __shfl_xor(S, off, 64);
    if (threadIdx.x == 0) s_misc[0] = S;
  }

  // ---- 1. load, causal sweep from a zero state ----
  f2b v[LMAX];
#pragma unroll
  for (int j = 0; j < LMAX; ++j) v[j] = bld2<CP>(rT, j < nin ? vT + j * rowT : kOOB, 0);
  stage_consts(s_cc, p.cc, tile * C, C, p.NH);
  dc e = {0.0, 0.0}, mu = {0.0, 0.0};
  if (dcol) {
    // column 0: inclusive prefix sums of x, and the sum of those prefixes over the segment
    dc st = {0.0, 0.0};
    double sumP = 0.0;
#pragma unroll
    for (int j = 0; j < LMAX; ++j) {
      pin(v[j]);
      st = {st.x + v[j].x, st.y + v[j].y};
      if (TAIL) sumP += j < Ls ? st.x : 0.0;
      else sumP += st.x;
      v[j] = f2b{float(st.x), float(st.y)};
        pin(v[j]);
    }
    e = st;
    mu = {sumP, 0.0};
  } else {
    dc st = {0.0, 0.0};
    double pw = 1.0;
#pragma unroll
    for (int j = 0; j < LMAX; ++j) {
      pin(v[j]);
      st = dfma(rho, st, dc{v[j].x, v[j].y});
      v[j] = f2b{float(st.x), float(st.y)};
        pin(v[j]);
      if (TAIL) {
        mu = dfma(j < Ls ? pw : 0.0, st, mu);
        e = dsel(j == Ls - 1, st, e);
      } else {
        mu = dfma(pw, st, mu);
      }
      pw *= rho;
    }
    if (!TAIL) e = st;
  }
  if (active) {
    E[s * C + c] = e;
    U[s * C + c] = mu;
  }
  __syncthreads();

  // weight of the Dirac at r0: -sum(du) * w_N^(l c0)
  dc dv = {0.0, 0.0};
  if (col_ok) {
    const double S = s_misc[0];
    const f2 ph = p.dshift[l];
    dv = {-S * double(ph.x), -S * double(ph.y)};
  }

  // ---- 2. carries ----
  dc D = {0.0, 0.0};
  dc wR1 = {0.0, 0.0};
  double xbar = 0.0, meanP = 0.0;
  if (col_ok) {
    if (dcol) {
      // q = -D_y v with D_yy v = x - mean(x) on Z_M, x = column plus the Dirac:
      // q[y] = -(P[y] - mean(P)), P[y] = sum_{j <= y} (x[j] - xbar). Only q is needed (the
      // x-derivative symbol vanishes at l = 0).
      const int Rp = p.Rp;
      double pre = 0.0, tot = 0.0, sin_ = 0.0;
#pragma unroll 8
      for (int t = 0; t < nseg; ++t) {
        const double x = E[t * C + c].x;
        pre += t < s ? x : 0.0;
        tot += x;
        const int end = (t + 1) * LMAX < Rp ? (t + 1) * LMAX : Rp;
        sin_ += U[t * C + c].x + double(Rp - end) * x;  // sum over the block of the prefixes
      }
      const double Mr = double(p.M);
      xbar = (tot + dv.x) / Mr;
      // rows [Rp, M): the prefix is tot (plus dv from r0 on); minus sum_y xbar (y + 1)
      const double sout = tot * (Mr - double(Rp)) + dv.x * (Mr - double(p.r0));
      meanP = (sin_ + sout - xbar * Mr * (Mr + 1.0) * 0.5) / Mr;
      D = {pre, 0.0};
    } else {
      const int kseg = kp->kseg;
      const double rhoL = kp->rhoL;
      double rp, rl;
      const dc Cs = carry_in<kHornerBwd>(E, C, c, s, kseg, rhoL, rp);
      const dc Cl = carry_in<kHornerBwd>(E, C, c, last, kseg, rhoL, rl);
      const dc cR1 = dfma(kp->rhoLl, Cl, E[last * C + c]);
      const dc gam = dfma(kp->cgd, dv, dscale(cR1, kp->cg));
      D = dfma(rp, gam, dscale(Cs, rho));
      wR1 = dfma(kp->rhoRm1, gam, cR1);
      const dc zst = dfma(s == last ? kp->gLl : kp->gL, D, mu);
      U[s * C + c] = zst;
    }
  }
  __syncthreads();

  // ---- 3. anticausal sweep, outputs ----
  int vS3 = vT, vD3 = vD;
  asm volatile("" : "+v"(vS3), "+v"(vD3));
  if (col_ok) {
    const double outs = kp->outs;
    const int vEnd = Ls < nout ? vS3 + Ls * rowT : kOOB;  // the row after this segment
    if (dcol) {
#pragma unroll
      for (int j = 0; j < LMAX; ++j) {
        pin(v[j]);
        const double P = D.x + double(v[j].x) - xbar * double(p0 + j + 1);
        bst2(rD, float(-(P - meanP) * outs), 0.f, vD3 + j * rowD, 0);
        bst2<CP>(rT, 0.f, 0.f, j < nout ? vS3 + j * rowT : kOOB, 0);
      }
      if (s == last) bst2(rT, 0.f, 0.f, vEnd, 0);
    } else {
      const int kseg = kp->kseg;
      const double rhoL = kp->rhoL, rhoLl = kp->rhoLl;
      const dc Sw = head_moment<kHornerBwd>(U, C, c, last, kseg, rhoL);
      const dc ZR = dfma(kp->cTd, dv, dfma(kp->cT, wR1, dscale(Sw, kp->czR)));  // z[Rp]
      dc z = carry_out<kHornerBwd>(U, C, c, s, last, kseg, rhoL, rhoLl, ZR);
      if (s == last) bst2(rT, float(z.x * outs), float(z.y * outs), vEnd, 0);
      const double inv_rho = kp->inv_rho;
      const double omr = kp->omr;
      double pj = rhoL * inv_rho;
#pragma unroll
      for (int j = LMAX - 1; j >= 0; --j) {
        pin(v[j]);
        const dc w = dfma(pj, D, dc{v[j].x, v[j].y});
        if (low) {
          const dc q = {w.x - omr * z.x, w.y - omr * z.y};
          bst2(rD, float(q.x * outs), float(q.y * outs), vD3 + j * rowD, 0);
        }
        if (TAIL) z = dsel(j < Ls, dfma(rho, z, w), z);
        else z = dfma(rho, z, w);
        bst2<CP>(rT, float(z.x * outs), float(z.y * outs), j < nout ? vS3 + j * rowT : kOOB, 0);
        pj *= inv_rho;
      }
    }
  }
}

// LOWTILE: the launch of the tiles holding columns l <= Kb (the -D_y output and column 0's
// pseudo-inverse); the other tiles are compiled without those paths
template <int LMAX, bool LOWTILE, bool TAIL, int CP>
__global__ void __launch_bounds__(kColMaxThreads) k_col_bwd(ColBwdArgs p) {
  extern __shared__ dc s_mem[];
  dc* E = s_mem;
  dc* U = s_mem + p.nseg * p.C;
  double* s_misc = reinterpret_cast<double*>(s_mem + 2 * p.nseg * p.C);
  __shared__ ColConst s_cc[kColMaxC];
  col_bwd_tile<LMAX, LOWTILE, TAIL, CP>(p, p.tile0 + blockIdx.x, blockIdx.y, E, U, s_misc, s_cc);
}

namespace {
// whole waves, so the wave-0 butterflies never read a lane that does not exist
int col_block(int C, int nseg) { return (C * nseg + 63) / 64 * 64; }

// split: the low tiles on s_low, the others on s; else one launch of the general kernel
template <int LMAX, bool TAIL>
void launch_fwd_tiles(const ColFwdArgs& a, int ntiles, int nlow, int B, size_t shm,
                      hipStream_t s, hipStream_t s_low, bool nt, bool split) {
  const dim3 blk(col_block(a.C, a.nseg));
  ColFwdArgs x = a;
  if (!split) {
    x.tile0 = 0;
    hipLaunchKernelGGL((k_col_fwd<LMAX, true, TAIL, 0>), dim3(ntiles, B), blk, shm, s, x);
    return;
  }
  if (nlow > 0) {
    x.tile0 = 0;
    hipLaunchKernelGGL((k_col_fwd<LMAX, true, TAIL, 0>), dim3(nlow, B), blk, shm, s_low, x);
  }
  if (ntiles > nlow) {
    x.tile0 = nlow;
    if (nt)
      hipLaunchKernelGGL((k_col_fwd<LMAX, false, TAIL, kNT>), dim3(ntiles - nlow, B), blk, shm,
                         s, x);
    else
      hipLaunchKernelGGL((k_col_fwd<LMAX, false, TAIL, 0>), dim3(ntiles - nlow, B), blk, shm,
                         s, x);
  }
}
}  // namespace

// Given a side stream and two events, the tiles that hold columns l <= K are launched
// separately, on the side stream, beside the other tiles (compiled without the split-input
// path, which costs registers), and `s` waits for them: they are a small, latency-bound
// launch that would otherwise run alone. The fork and join cost about 30 us of latency, so
// batches whose spectra are small (under kSideMinBytes) launch all tiles at once on `s`
// with the general kernel: that halved the column pass of a 64x64 solve and took 5 % off a
// 48-image 256x256 batch, while 512x512 x 96 and 801x1200 x 100 keep the side stream (2-3 %
// faster with it).
constexpr long long kSideMinBytes = 100LL << 20;
// The main tiles read and write the spectra with nontemporal accesses when the batch's
// spectra exceed the 256 MB memory-side cache by far (801x1200 x 100: 770 MB): the next
// pass then reads them faster (the forward inverse row pass 0.289 -> 0.270 ms at the time).
// Smaller batches keep them cached between passes (a 48-image 256x256 batch, 28 MB, and
// 128^3 volumes, 272 MB, were 6-7 % slower with nontemporal column passes).
constexpr long long kNtMinBytes = 512LL << 20;
// The backward column pass gains from nontemporal accesses from smaller batches on: the
// backward inverse row pass after it reads W 12-13 % faster (214-346 MB of spectra:
// 512x512 x 96, 640x640 x 64, 1024x1024 x 40; backward step 5-8 % faster), where the
// forward solve changed by under 1 %. The backward pass has no volume form.
constexpr long long kNtMinBytesBwd = 64LL << 20;
hipError_t launch_col_fwd(const ColFwdArgs& a, int B, hipStream_t s, hipStream_t side,
                          hipEvent_t fork, hipEvent_t join) {
  const size_t shm = size_t(2 * a.nseg * a.C) * sizeof(dc);
  const int ntiles = (a.NH + a.C - 1) / a.C;
  const int nlow = std::min(ntiles, (a.K + 1 + a.C - 1) / a.C);
  const bool tail = a.Rp != a.nseg * a.Lseg;
  const bool split = side && fork && join && nlow > 0 && ntiles > nlow &&
                     (long long)B * a.img_t * 8 >= kSideMinBytes;
  const bool nt = (long long)B * a.img_t * 8 >= kNtMinBytes;
  hipStream_t s_low = s;
  if (split) {
    hipError_t e = hipEventRecord(fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
    if (e != hipSuccess) return e;
    s_low = side;
  }
  if (a.Lseg == 16) {
    if (tail) launch_fwd_tiles<16, true>(a, ntiles, nlow, B, shm, s, s_low, nt, split);
    else launch_fwd_tiles<16, false>(a, ntiles, nlow, B, shm, s, s_low, nt, split);
  } else if (a.Lseg == 32) {
    if (tail) launch_fwd_tiles<32, true>(a, ntiles, nlow, B, shm, s, s_low, nt, split);
    else launch_fwd_tiles<32, false>(a, ntiles, nlow, B, shm, s, s_low, nt, split);
  } else {
    return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (split && e == hipSuccess) {
    e = hipEventRecord(join, side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, join, 0);
  }
  return e;
}

namespace {
template <int LMAX, bool TAIL>
void launch_rg_tiles(const RgBase* base, const RgCol* tab, const RgItem* low, int nlow,
                     const RgItem* rest, int nrest, int threads, size_t shm, hipStream_t s) {
  if (nlow > 0 && nrest > 0 && rest == low + nlow) {
    hipLaunchKernelGGL((k_col_fwd_rg_all<LMAX, TAIL>), dim3(nlow + nrest), dim3(threads), shm,
                       s, base, tab, low, nlow);
    return;
  }
  if (nlow > 0)
    hipLaunchKernelGGL((k_col_fwd_rg<LMAX, true, TAIL>), dim3(nlow), dim3(threads), shm, s,
                       base, tab, low);
  if (nrest > 0)
    hipLaunchKernelGGL((k_col_fwd_rg<LMAX, false, TAIL>), dim3(nrest), dim3(threads), shm, s,
                       base, tab, rest);
}
}  // namespace

hipError_t launch_col_fwd_rg(const RgBase* base, const RgCol* tab, const RgItem* low,
                             int nlow, const RgItem* rest, int nrest, int Lseg, bool tail,
                             int threads, size_t shm, hipStream_t s) {
  if (threads < 64 || threads > kColMaxThreads || threads % 64) return hipErrorInvalidValue;
  if (Lseg == 16) {
    if (tail) launch_rg_tiles<16, true>(base, tab, low, nlow, rest, nrest, threads, shm, s);
    else launch_rg_tiles<16, false>(base, tab, low, nlow, rest, nrest, threads, shm, s);
  } else if (Lseg == 32) {
    if (tail) launch_rg_tiles<32, true>(base, tab, low, nlow, rest, nrest, threads, shm, s);
    else launch_rg_tiles<32, false>(base, tab, low, nlow, rest, nrest, threads, shm, s);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

namespace {
// split: the low tiles on s_low, the others on s; else one launch of the general kernel
template <int LMAX, bool TAIL>
void launch_bwd_tiles(const ColBwdArgs& a, int ntiles, int nlow, int B, size_t shm,
                      hipStream_t s, hipStream_t s_low, bool nt, bool split) {
  const dim3 blk(col_block(a.C, a.nseg));
  ColBwdArgs x = a;
  if (!split) {
    x.tile0 = 0;
    hipLaunchKernelGGL((k_col_bwd<LMAX, true, TAIL, 0>), dim3(ntiles, B), blk, shm, s, x);
    return;
  }
  if (nlow > 0) {
    x.tile0 = 0;
    hipLaunchKernelGGL((k_col_bwd<LMAX, true, TAIL, 0>), dim3(nlow, B), blk, shm, s_low, x);
  }
  if (ntiles > nlow) {
    x.tile0 = nlow;
    if (nt)
      hipLaunchKernelGGL((k_col_bwd<LMAX, false, TAIL, kNT>), dim3(ntiles - nlow, B), blk, shm,
                         s, x);
    else
      hipLaunchKernelGGL((k_col_bwd<LMAX, false, TAIL, 0>), dim3(ntiles - nlow, B), blk, shm,
                         s, x);
  }
}
}  // namespace

// As in the forward pass, the tiles with columns l <= Kb are a launch of their own, on the
// side stream when one is given and the batch is large, beside the other tiles.
hipError_t launch_col_bwd(const ColBwdArgs& a, int B, hipStream_t s, hipStream_t side,
                          hipEvent_t fork, hipEvent_t join) {
  const size_t shm = size_t(2 * a.nseg * a.C) * sizeof(dc) + 8 * sizeof(double);
  if (a.nimg != B) return hipErrorInvalidValue;
  const int ntiles = (a.NH + a.C - 1) / a.C;
  const int nlow = std::min(ntiles, (a.Kb + a.C) / a.C);
  const bool tail = a.Rp != a.nseg * a.Lseg;
  const bool split = side && fork && join && nlow > 0 && ntiles > nlow &&
                     (long long)B * a.img_t * 8 >= kSideMinBytes;
  const bool nt = (long long)B * a.img_t * 8 >= kNtMinBytesBwd;
  hipStream_t s_low = s;
  if (split) {
    hipError_t e = hipEventRecord(fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
    if (e != hipSuccess) return e;
    s_low = side;
  }
  if (a.Lseg == 16) {
    if (tail) launch_bwd_tiles<16, true>(a, ntiles, nlow, B, shm, s, s_low, nt, split);
    else launch_bwd_tiles<16, false>(a, ntiles, nlow, B, shm, s, s_low, nt, split);
  } else if (a.Lseg == 32) {
    if (tail) launch_bwd_tiles<32, true>(a, ntiles, nlow, B, shm, s, s_low, nt, split);
    else launch_bwd_tiles<32, false>(a, ntiles, nlow, B, shm, s, s_low, nt, split);
  } else {
    return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (split && e == hipSuccess) {
    e = hipEventRecord(join, side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, join, 0);
  }
  return e;
}

}  // namespace gfc
