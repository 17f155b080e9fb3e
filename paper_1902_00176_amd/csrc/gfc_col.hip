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
// contiguous bytes per row). Each thread keeps its segment in registers; segment states are
// combined in LDS by one thread per column; then every thread finishes its rows. The
// result overwrites the input in place. Global accesses go through buffer descriptors.
#include <algorithm>

#include "gfc_buf.h"
#include "gfc_internal.h"

namespace gfc {

struct dc {
  double x, y;
};

constexpr int kChunk = 8;   // rows loaded per step of a segment sweep
constexpr int kCChunk = 4;  // segments per step of the combine

__device__ __forceinline__ dc dadd(dc a, dc b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ dc dscale(dc a, double s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ dc dfma(double s, dc a, dc b) {  // s*a + b
  return {__builtin_fma(s, a.x, b.x), __builtin_fma(s, a.y, b.y)};
}

// Combine the per-segment causal end states e_t (in A0) and moments mu_t (in A1) of one
// column into, per segment, D_t (-> A0) and the anticausal carry Z_t = z[p_t + L_t] (-> A1).
// Returns z[0] and w[R-1]. dv is the weight of a Dirac at row r0 (0 in the forward pass).
__device__ __forceinline__ void combine_column(dc* A0, dc* A1, int C, int c, int nseg,
                                               const ColConst* __restrict__ kp, double rho,
                                               dc dv, dc& z0, dc& wR1) {
  const double rhoL = kp->rhoL, rhoLl = kp->rhoLl;
  // causal carries: C_t = state before segment t
  dc Cc = {0.0, 0.0};
  for (int t0 = 0; t0 < nseg; t0 += kCChunk) {
    dc e[kCChunk];
#pragma unroll
    for (int q = 0; q < kCChunk; ++q) e[q] = (t0 + q < nseg) ? A0[(t0 + q) * C + c] : dc{0.0, 0.0};
#pragma unroll
    for (int q = 0; q < kCChunk; ++q) {
      const int t = t0 + q;
      if (t < nseg) {
        A0[t * C + c] = Cc;
        Cc = dfma(t == nseg - 1 ? rhoLl : rhoL, Cc, e[q]);
      }
    }
  }
  const dc cR1 = Cc;
  const dc gam = dfma(kp->cgd, dv, dscale(cR1, kp->cg));
  // D_t = rho C_t + rho^(p_t) gamma; zst_t = mu_t + g_t D_t; Sum_w = sum rho^(p_t) zst_t
  const double gL = kp->gL, gLl = kp->gLl;
  dc Sw = {0.0, 0.0};
  double rp = 1.0;
  for (int t0 = 0; t0 < nseg; t0 += kCChunk) {
    dc cin[kCChunk], mu[kCChunk];
#pragma unroll
    for (int q = 0; q < kCChunk; ++q) {
      const bool ok = t0 + q < nseg;
      cin[q] = ok ? A0[(t0 + q) * C + c] : dc{0.0, 0.0};
      mu[q] = ok ? A1[(t0 + q) * C + c] : dc{0.0, 0.0};
    }
#pragma unroll
    for (int q = 0; q < kCChunk; ++q) {
      const int t = t0 + q;
      if (t < nseg) {
        const dc Dt = dfma(rp, gam, dscale(cin[q], rho));
        A0[t * C + c] = Dt;
        const dc zst = dfma(t == nseg - 1 ? gLl : gL, Dt, mu[q]);
        A1[t * C + c] = zst;
        Sw = dfma(rp, zst, Sw);
        rp *= rhoL;
      }
    }
  }
  wR1 = dfma(kp->rhoRm1, gam, cR1);
  dc Z = dfma(kp->cTd, dv, dfma(kp->cT, wR1, dscale(Sw, kp->czR)));  // z[R]
  // anticausal carries, last segment first
  for (int t1 = nseg - 1; t1 >= 0; t1 -= kCChunk) {
    dc zs[kCChunk];
#pragma unroll
    for (int q = 0; q < kCChunk; ++q) zs[q] = (t1 - q >= 0) ? A1[(t1 - q) * C + c] : dc{0.0, 0.0};
#pragma unroll
    for (int q = 0; q < kCChunk; ++q) {
      const int t = t1 - q;
      if (t >= 0) {
        A1[t * C + c] = Z;  // z at the row after segment t
        Z = dfma(t == nseg - 1 ? rhoLl : rhoL, Z, zs[q]);
      }
    }
  }
  z0 = Z;
}

// The segment's first input row of a low column carries -b[p0-1]; seeding the causal state
// of b with b[p0-1] / (1 - rho) makes (1 - rho) * sbb reproduce it without a cancellation.
__device__ __forceinline__ dc sbb_seed(rsrc_t rS, int voS, int rowS, int p0, int H, bool on,
                                       double omr) {
  if (on && p0 > 0 && p0 - 1 < H) {
    const f2b bp = bld2(rS, voS - rowS, 0);
    return {double(bp.x) / omr, double(bp.y) / omr};
  }
  return {0.0, 0.0};
}

// Causal sweep of one segment (forward pass input): returns the end state and the moment
// sum_j rho^j c[p0 + j]; with STORE, also c (float32) into creg. Column 0
// accumulates the running sum of b instead (creg gets the exclusive prefix).
template <int LMAX, bool STORE>
__device__ __forceinline__ void causal_sweep(rsrc_t rT, rsrc_t rS, int voT, int voS, int rowT,
                                             int rowS, int Ls, int p0, int H, bool low,
                                             bool dcol, double rho, double omr, dc sbb, dc& st,
                                             dc& mu, f2 (&creg)[LMAX]) {
  dc sa = {0.0, 0.0};
  double pw = 1.0;
  st = {0.0, 0.0};
  mu = {0.0, 0.0};
#pragma unroll
  for (int j0 = 0; j0 < LMAX; j0 += kChunk) {
    f2b xs[kChunk], bs[kChunk];
#pragma unroll
    for (int jj = 0; jj < kChunk; ++jj) {
      const int j = j0 + jj;
      xs[jj] = (j < Ls && !dcol) ? bld2(rT, voT, j * rowT) : f2b{0.f, 0.f};
      bs[jj] = (low && j < Ls && p0 + j < H) ? bld2(rS, voS, j * rowS) : f2b{0.f, 0.f};
    }
#pragma unroll
    for (int jj = 0; jj < kChunk; ++jj) {
      const int j = j0 + jj;
      if (j < Ls) {
        const f2b x = xs[jj];
        const f2b bb = bs[jj];
        if (low) {
          if (dcol) {
            if constexpr (STORE) creg[j] = f2{float(st.x), float(st.y)};  // exclusive prefix sum
            st = {st.x + bb.x, st.y + bb.y};
          } else {
            sa = dfma(rho, sa, dc{x.x, x.y});
            st = {sa.x + bb.x - omr * sbb.x, sa.y + bb.y - omr * sbb.y};
            sbb = dfma(rho, sbb, dc{bb.x, bb.y});
            if constexpr (STORE) creg[j] = f2{float(st.x), float(st.y)};
            mu = dfma(pw, st, mu);
            pw *= rho;
          }
        } else {
          st = dfma(rho, st, dc{x.x, x.y});
          if constexpr (STORE) creg[j] = f2{float(st.x), float(st.y)};
          mu = dfma(pw, st, mu);
          pw *= rho;
        }
      }
    }
    // with the segment held in registers, keep at most one chunk of loads in flight
    if constexpr (STORE) asm volatile("" ::: "memory");
  }
}

// ---------------------------------------------------------------------------------------
// Forward: input rows [0, R), R = H + 1; outputs rows [0, H) and the reference term.
// Columns l <= K arrive split: T holds a = (1 - w_N^l) Ex^ and SB holds b = Ey^, and the
// column input is a + (1 - S) b. The difference is folded into the causal recursion:
// (1 - rho S)^-1 (1 - S) b = b - (1 - rho) S (1 - rho S)^-1 b, which has no cancellation.
template <int LMAX, bool LOWTILE>
__global__ void __launch_bounds__(kColMaxThreads, 4) k_col_fwd(ColFwdArgs p) {
  extern __shared__ dc s_mem[];
  const int C = p.C;
  const int nseg = p.nseg;
  dc* A0 = s_mem;                  // [nseg][C]
  dc* A1 = s_mem + nseg * C;       // [nseg][C]
  double* s_ref = reinterpret_cast<double*>(s_mem + 2 * nseg * C);  // [C]

  const int c = threadIdx.x % C;
  const int s = threadIdx.x / C;
  const int tile = p.tile0 + blockIdx.x;
  const int l = tile * C + c;
  const int b = blockIdx.y;
  const bool col_ok = l < p.NH;
  const int p0 = s * p.Lseg;
  const int Ls = (s == nseg - 1) ? p.Llast : p.Lseg;
  // tiles holding columns l <= K are launched separately (LOWTILE) so the split-input path
  // costs no registers in the other tiles
  const bool dcol = LOWTILE && (l == 0);
  const bool low = LOWTILE && col_ok && l <= p.K;
  const int K1 = p.KP;

  const rsrc_t rT = make_buf(p.T + b * p.img_t, p.img_t * 8);
  const rsrc_t rS = make_buf(p.SB + b * p.img_sb, p.img_sb * 8);
  const int rowT = p.NHP * 8;
  const int rowS = K1 * 8;
  const int voT = (p0 * p.NHP + l) * 8;
  const int voS = (p0 * K1 + l) * 8;

  double rho = 1.0, omr = 0.0;
  if (col_ok && !dcol) {
    rho = p.cc[l].rho;
    omr = p.cc[l].omr;
  }

  // Phase 1: sweep the segment once, keeping only its causal end state and moment. The
  // segment is read again in phase 3 (from cache), so no register copy is held across the
  // combine and more workgroups fit on a CU.
  dc st = {0.0, 0.0};    // causal state (column 0: running sum of b)
  dc mu = {0.0, 0.0};    // sum_j rho^j c[p0 + j]
  if (col_ok) {
    f2 unused[LMAX];
    causal_sweep<LMAX, false>(rT, rS, voT, voS, rowT, rowS, Ls, p0, p.H, low, dcol, rho, omr,
                              sbb_seed(rS, voS, rowS, p0, p.H, low && !dcol, omr), st, mu,
                              unused);
  }
  A0[s * C + c] = st;
  A1[s * C + c] = mu;
  __syncthreads();

  if (s == 0) {
    double term = 0.0;
    if (col_ok) {
      if (dcol) {
        dc pre = {0.0, 0.0};
        for (int t = 0; t < nseg; ++t) {
          const dc e = A0[t * C + c];
          A0[t * C + c] = pre;
          pre = dadd(pre, e);
        }
        const double bbar = pre.x / double(p.M);
        A1[c] = dc{bbar, 0.0};
        term = (pre.x - double(p.r0) * bbar) * p.cc[0].outs;
      } else {
        const ColConst* kp = p.cc + l;
        dc z0, wR1;
        combine_column(A0, A1, C, c, nseg, kp, rho, dc{0.0, 0.0}, z0, wR1);
        const dc zr0 = dfma(kp->ra, wR1, dscale(z0, kp->rb));
        term = kp->wre * zr0.x - kp->wim * zr0.y;
      }
    }
    s_ref[c] = term;
  }
  __syncthreads();

  if (col_ok) {
    f2 creg[LMAX];
    dc st2 = {0.0, 0.0}, mu2 = {0.0, 0.0};
    causal_sweep<LMAX, true>(rT, rS, voT, voS, rowT, rowS, Ls, p0, p.H, low, dcol, rho, omr,
                             sbb_seed(rS, voS, rowS, p0, p.H, low && !dcol, omr), st2, mu2,
                             creg);
    if (dcol) {
      const dc D = A0[s * C];
      const double bbar = A1[0].x;
      const double outs = p.cc[0].outs;
#pragma unroll
      for (int j = 0; j < LMAX; ++j) {
        const int y = p0 + j;
        if (j < Ls && y < p.H) {
          const double v = (D.x + double(creg[j].x) - bbar * double(y)) * outs;
          bst2(rT, float(v), 0.f, voT, j * rowT);
        }
      }
    } else {
      const dc D = A0[s * C + c];
      dc z = A1[s * C + c];
      const double inv_rho = p.cc[l].inv_rho;
      const double outs = p.cc[l].outs;
      double pj = (s == nseg - 1 ? p.cc[l].rhoLl : p.cc[l].rhoL) * inv_rho;  // rho^(Ls-1)
#pragma unroll
      for (int j = LMAX - 1; j >= 0; --j) {
        if (j < Ls) {
          const int y = p0 + j;
          const dc w = dfma(pj, D, dc{creg[j].x, creg[j].y});
          z = dfma(rho, z, w);
          if (y < p.H) bst2(rT, float(z.x * outs), float(z.y * outs), voT, j * rowT);
          pj *= inv_rho;
        }
      }
    }
  }
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < C; ++i) t += s_ref[i];
    p.partial[(long long)b * p.ntiles + tile] = t;
  }
}

// Causal sweep of one segment of the backward pass input (plain column, no split): end
// state, moment, optional float32 copy. Column 0 keeps the inclusive prefix sum of x and
// the sum of those prefixes.
template <int LMAX, bool STORE>
__device__ __forceinline__ void causal_sweep_plain(rsrc_t rT, int voT, int rowT, int Ls,
                                                   bool dcol, double rho, dc& st, dc& mu,
                                                   double& sumP, f2 (&creg)[LMAX]) {
  double pw = 1.0;
  st = {0.0, 0.0};
  mu = {0.0, 0.0};
  sumP = 0.0;
#pragma unroll
  for (int j0 = 0; j0 < LMAX; j0 += kChunk) {
    f2b xs[kChunk];
#pragma unroll
    for (int jj = 0; jj < kChunk; ++jj) {
      const int j = j0 + jj;
      xs[jj] = (j < Ls) ? bld2(rT, voT, j * rowT) : f2b{0.f, 0.f};
    }
#pragma unroll
    for (int jj = 0; jj < kChunk; ++jj) {
      const int j = j0 + jj;
      if (j < Ls) {
        const f2b x = xs[jj];
        if (dcol) {
          st = {st.x + x.x, st.y + x.y};  // inclusive prefix sum
          sumP += st.x;
          if constexpr (STORE) creg[j] = f2{float(st.x), float(st.y)};
        } else {
          st = dfma(rho, st, dc{x.x, x.y});
          if constexpr (STORE) creg[j] = f2{float(st.x), float(st.y)};
          mu = dfma(pw, st, mu);
          pw *= rho;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// Backward: input rows [0, R), R = H, plus a Dirac of weight dv = -sum(du) w_N^(l c0) at
// row r0 (the adjoint of the reference-pixel subtraction). Outputs w rows [0, H] and, for
// l <= Kb, the column derivative (-D_y w)[y] = w_in[y] - (1 - rho) z[y+1] scaled like w.
template <int LMAX>
__global__ void __launch_bounds__(kColMaxThreads, 4) k_col_bwd(ColBwdArgs p) {
  extern __shared__ dc s_mem[];
  const int C = p.C;
  const int nseg = p.nseg;
  dc* A0 = s_mem;
  dc* A1 = s_mem + nseg * C;
  double* s_misc = reinterpret_cast<double*>(s_mem + 2 * nseg * C);  // column-0 extras

  const int c = threadIdx.x % C;
  const int s = threadIdx.x / C;
  const int l = blockIdx.x * C + c;
  const int b = blockIdx.y;
  const bool col_ok = l < p.NH;
  const int R = p.H;
  const int p0 = s * p.Lseg;
  const int Ls = (s == nseg - 1) ? p.Llast : p.Lseg;
  const bool dcol = (l == 0);
  const bool low = col_ok && l <= p.Kb;
  const int Kb1 = p.KbP;

  const rsrc_t rT = make_buf(p.T + b * p.img_t, p.img_t * 8);
  const rsrc_t rD = make_buf(p.SD + b * p.img_sd, p.img_sd * 8);
  const int rowT = p.NHP * 8;
  const int rowD = Kb1 * 8;
  const int voT = (p0 * p.NHP + l) * 8;
  const int voD = (p0 * Kb1 + l) * 8;

  // sum(du) from the row pass's partials: wave 0 reduces them (lane-strided sums, then a
  // fixed-order butterfly) and leaves the total in LDS for after the first barrier
  if (threadIdx.x < 64) {
    double S = 0.0;
    for (int j = threadIdx.x; j < p.nsums; j += 64) S += p.sums[(long long)b * p.nsums + j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) S += __shfl_xor(S, off, 64);
    if (threadIdx.x == 0) s_misc[4] = S;
  }

  double rho = 1.0;
  if (col_ok && !dcol) rho = p.cc[l].rho;

  // Phase 1: summaries only (see the forward kernel); column 0 also sums its local
  // inclusive prefix sums for the mean used below.
  dc st = {0.0, 0.0};
  dc mu = {0.0, 0.0};
  double sumP = 0.0;
  if (col_ok) {
    f2 unused[LMAX];
    causal_sweep_plain<LMAX, false>(rT, voT, rowT, Ls, dcol, rho, st, mu, sumP, unused);
  }
  A0[s * C + c] = st;
  A1[s * C + c] = mu;
  __syncthreads();
  // weight of the Dirac at r0: -sum(du) * w_N^(l c0)
  dc dv = {0.0, 0.0};
  if (col_ok) {
    const double S = s_misc[4];
    const f2 ph = p.dshift[l];
    dv = {-S * double(ph.x), -S * double(ph.y)};
  }

  if (s == 0 && col_ok && dcol) {
    // Column 0: q = -D_y v with D_yy v = x - mean(x) on Z_M, x = column plus the Dirac;
    // q[y] = -(P[y] - mean(P)), P[y] = sum_{j <= y} (x[j] - xbar). Only q is needed (the
    // x-derivative symbol vanishes at l = 0).
    dc pre = {0.0, 0.0};
    for (int t = 0; t < nseg; ++t) {
      const dc e = A0[t * C + c];
      A0[t * C + c] = pre;
      pre = dadd(pre, e);
    }
    const double tot = pre.x + dv.x;
    s_misc[0] = tot / double(p.M);
    s_misc[1] = pre.x;
    s_misc[2] = dv.x;
  }
  __syncthreads();
  // column 0 needs sum_{y<R} Pin[y] (Pin the inclusive prefix of x): reduce in LDS
  if (dcol) {
    double part = 0.0;
    if (col_ok) part = double(Ls) * A0[s * C + c].x + sumP;
    A1[s * C + c] = dc{part, 0.0};
  }
  __syncthreads();
  if (s == 0 && col_ok) {
    if (dcol) {
      double sin_ = 0.0;
      for (int t = 0; t < nseg; ++t) sin_ += A1[t * C + c].x;
      const double Mr = double(p.M);
      const double xbar = s_misc[0], pre = s_misc[1], dvx = s_misc[2];
      // rows [R, M): Pin = pre (+ dv from r0 on); sum_y xbar (y + 1) over Z_M
      const double sout = pre * (Mr - double(R)) + dvx * (Mr - double(p.r0));
      s_misc[3] = (sin_ + sout - xbar * Mr * (Mr + 1.0) * 0.5) / Mr;
    } else {
      dc z0, wR1;
      combine_column(A0, A1, C, c, nseg, p.cc + l, rho, dv, z0, wR1);
    }
  }
  __syncthreads();

  if (col_ok) {
    f2 creg[LMAX];
    dc st2 = {0.0, 0.0}, mu2 = {0.0, 0.0};
    double sp2 = 0.0;
    causal_sweep_plain<LMAX, true>(rT, voT, rowT, Ls, dcol, rho, st2, mu2, sp2, creg);
    if (dcol) {
      const double xbar = s_misc[0], meanP = s_misc[3];
      const double outs = p.cc[0].outs;
      const double pre_s = A0[s * C].x;
#pragma unroll
      for (int j = 0; j < LMAX; ++j) {
        const int y = p0 + j;
        if (j < Ls) {
          const double P = pre_s + double(creg[j].x) - xbar * double(y + 1);
          bst2(rD, float(-(P - meanP) * outs), 0.f, voD, j * rowD);
          bst2(rT, 0.f, 0.f, voT, j * rowT);
        }
      }
      if (s == nseg - 1) bst2(rT, 0.f, 0.f, voT, Ls * rowT);
    } else {
      const dc D = A0[s * C + c];
      dc z = A1[s * C + c];
      const double inv_rho = p.cc[l].inv_rho;
      const double outs = p.cc[l].outs;
      const double omr = p.cc[l].omr;
      if (s == nseg - 1) bst2(rT, float(z.x * outs), float(z.y * outs), voT, Ls * rowT);
      double pj = (s == nseg - 1 ? p.cc[l].rhoLl : p.cc[l].rhoL) * inv_rho;
#pragma unroll
      for (int j = LMAX - 1; j >= 0; --j) {
        if (j < Ls) {
          const dc w = dfma(pj, D, dc{creg[j].x, creg[j].y});
          if (low) {
            const dc q = {w.x - omr * z.x, w.y - omr * z.y};
            bst2(rD, float(q.x * outs), float(q.y * outs), voD, j * rowD);
          }
          z = dfma(rho, z, w);
          bst2(rT, float(z.x * outs), float(z.y * outs), voT, j * rowT);
          pj *= inv_rho;
        }
      }
    }
  }
}

hipError_t launch_col_fwd(const ColFwdArgs& a0, int B, hipStream_t s) {
  const size_t shm = size_t(2 * a0.nseg * a0.C) * sizeof(dc) + size_t(a0.C) * sizeof(double);
  ColFwdArgs a = a0;
  const int ntiles = (a.NH + a.C - 1) / a.C;
  const int nlow = std::min(ntiles, (a.K + 1 + a.C - 1) / a.C);
  a.ntiles = ntiles;
  const dim3 blk(a.C * a.nseg);
  const bool short_rows = a.Lseg <= 16;
  if (nlow > 0) {
    a.tile0 = 0;
    if (short_rows) hipLaunchKernelGGL((k_col_fwd<16, true>), dim3(nlow, B), blk, shm, s, a);
    else hipLaunchKernelGGL((k_col_fwd<32, true>), dim3(nlow, B), blk, shm, s, a);
  }
  if (ntiles > nlow) {
    a.tile0 = nlow;
    if (short_rows) hipLaunchKernelGGL((k_col_fwd<16, false>), dim3(ntiles - nlow, B), blk, shm, s, a);
    else hipLaunchKernelGGL((k_col_fwd<32, false>), dim3(ntiles - nlow, B), blk, shm, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_col_bwd(const ColBwdArgs& a, int B, hipStream_t s) {
  const size_t shm = size_t(2 * a.nseg * a.C) * sizeof(dc) + size_t(a.C + 8) * sizeof(double);
  dim3 grid((a.NH + a.C - 1) / a.C, B);
  if (a.Lseg <= 16) {
    hipLaunchKernelGGL(k_col_bwd<16>, grid, dim3(a.C * a.nseg), shm, s, a);
  } else {
    hipLaunchKernelGGL(k_col_bwd<32>, grid, dim3(a.C * a.nseg), shm, s, a);
  }
  return hipGetLastError();
}

}  // namespace gfc
