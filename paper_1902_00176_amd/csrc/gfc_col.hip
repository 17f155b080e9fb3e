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
// contiguous bytes per row). Segment states are combined in LDS, then every thread
// finishes its rows; the result overwrites the input in place.
#include "gfc_internal.h"

namespace gfc {

struct dc {
  double x, y;
};

__device__ __forceinline__ dc dadd(dc a, dc b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ dc dscale(dc a, double s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ dc dfma(double s, dc a, dc b) {  // s*a + b
  return {__builtin_fma(s, a.x, b.x), __builtin_fma(s, a.y, b.y)};
}

// ---------------------------------------------------------------------------------------
// Forward: input rows [0, R), R = H + 1; outputs rows [0, H) and the reference term.
// Columns l <= K arrive split: T holds a = (1 - w_N^l) Ex^ and SB holds b = Ey^, and the
// column input is a + (1 - S) b. The difference is folded into the causal recursion:
// (1 - rho S)^-1 (1 - S) b = b - (1 - rho) S (1 - rho S)^-1 b, which has no cancellation.
template <int LMAX>
__global__ void __launch_bounds__(1024) k_col_fwd(ColFwdArgs p) {
  extern __shared__ dc s_mem[];
  const int C = p.C;
  const int nseg = p.nseg;
  dc* A0 = s_mem;                  // [nseg][C]: segment end state -> carry -> D
  dc* A1 = s_mem + nseg * C;       // [nseg][C]: segment moment -> Z carry
  double* s_ref = reinterpret_cast<double*>(s_mem + 2 * nseg * C);  // [C]

  const int c = threadIdx.x % C;
  const int s = threadIdx.x / C;
  const int l = blockIdx.x * C + c;
  const int b = blockIdx.y;
  const bool col_ok = l < p.NH;
  const int R = p.H + 1;
  const int p0 = s * p.Lseg;
  const int Ls = (s == nseg - 1) ? p.Llast : p.Lseg;
  const bool dcol = (l == 0);
  const bool low = col_ok && l <= p.K;
  const int K1 = p.K + 1;

  f2* __restrict__ T = p.T + b * p.img_t + l;
  const f2* __restrict__ SB = p.SB + b * p.img_sb + l;

  double rho = 1.0, omr = 0.0;
  if (col_ok && !dcol) {
    rho = p.cc[l].rho;
    omr = p.cc[l].omr;
  }

  f2 creg[LMAX];
  dc st = {0.0, 0.0};    // causal state (column 0: running sum of b)
  dc sa = {0.0, 0.0};    // low columns: causal state of a
  dc sbb = {0.0, 0.0};   // low columns: causal state of b
  dc mu = {0.0, 0.0};    // sum_j rho^j c[p0 + j]
  double pw = 1.0;
  if (low && !dcol && p0 > 0 && p0 - 1 < p.H) {
    // the segment's first input row carries -b[p0-1]; seeding the causal state of b with
    // b[p0-1] / (1 - rho) makes (1 - rho) * sbb reproduce it without a cancellation
    const f2 bp = SB[(long long)(p0 - 1) * K1];
    sbb = {double(bp.x) / omr, double(bp.y) / omr};
  }
  if (col_ok) {
#pragma unroll
    for (int j = 0; j < LMAX; ++j) {
      if (j < Ls) {
        const int y = p0 + j;
        const f2 x = T[(long long)y * p.NH];
        if (low) {
          f2 bb = {0.f, 0.f};
          if (y < p.H) bb = SB[(long long)y * K1];
          if (dcol) {
            creg[j] = f2{float(st.x), float(st.y)};  // exclusive prefix sum
            st = {st.x + bb.x, st.y + bb.y};
          } else {
            sa = dfma(rho, sa, dc{x.x, x.y});
            st = {sa.x + bb.x - omr * sbb.x, sa.y + bb.y - omr * sbb.y};
            sbb = dfma(rho, sbb, dc{bb.x, bb.y});
            creg[j] = f2{float(st.x), float(st.y)};
            mu = dfma(pw, st, mu);
            pw *= rho;
          }
        } else {
          st = dfma(rho, st, dc{x.x, x.y});
          creg[j] = f2{float(st.x), float(st.y)};
          mu = dfma(pw, st, mu);
          pw *= rho;
        }
      }
    }
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
        const ColConst k = p.cc[l];
        dc Cc = {0.0, 0.0};
        for (int t = 0; t < nseg; ++t) {
          const dc e = A0[t * C + c];
          A0[t * C + c] = Cc;  // state before segment t
          Cc = dfma(t == nseg - 1 ? k.rhoLl : k.rhoL, Cc, e);
        }
        const dc cR1 = Cc;
        const dc gam = dscale(cR1, k.cg);
        dc Sw = {0.0, 0.0};
        double rp = 1.0;
        for (int t = 0; t < nseg; ++t) {
          const dc Dt = dfma(rp, gam, dscale(A0[t * C + c], rho));
          A0[t * C + c] = Dt;
          const dc zst = dfma(t == nseg - 1 ? k.gLl : k.gL, Dt, A1[t * C + c]);
          A1[t * C + c] = zst;
          Sw = dfma(rp, zst, Sw);
          rp *= k.rhoL;
        }
        const dc wR1 = dfma(k.rhoRm1, gam, cR1);
        dc Z = dfma(k.cT, wR1, dscale(Sw, k.czR));
        for (int t = nseg - 1; t >= 0; --t) {
          const dc zst = A1[t * C + c];
          A1[t * C + c] = Z;  // z at the row after segment t
          Z = dfma(t == nseg - 1 ? k.rhoLl : k.rhoL, Z, zst);
        }
        const dc zr0 = dfma(k.ra, wR1, dscale(Z, k.rb));
        term = k.wre * zr0.x - k.wim * zr0.y;
      }
    }
    s_ref[c] = term;
  }
  __syncthreads();

  if (col_ok) {
    if (dcol) {
      const dc D = A0[s * C];
      const double bbar = A1[0].x;
      const double outs = p.cc[0].outs;
#pragma unroll
      for (int j = 0; j < LMAX; ++j) {
        const int y = p0 + j;
        if (j < Ls && y < p.H) {
          const double v = (D.x + double(creg[j].x) - bbar * double(y)) * outs;
          T[(long long)y * p.NH] = f2{float(v), 0.f};
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
          if (y < p.H) T[(long long)y * p.NH] = f2{float(z.x * outs), float(z.y * outs)};
          pj *= inv_rho;
        }
      }
    }
  }
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < C; ++i) t += s_ref[i];
    p.partial[(long long)b * gridDim.x + blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------------------
// Backward: input rows [0, R), R = H, plus a Dirac of weight dv = -sum(du) w_N^(l c0) at
// row r0 (the adjoint of the reference-pixel subtraction). Outputs w rows [0, H] and, for
// l <= Kb, the column derivative (-D_y w)[y] = w_in[y] - (1 - rho) z[y+1] scaled like w.
template <int LMAX>
__global__ void __launch_bounds__(1024) k_col_bwd(ColBwdArgs p) {
  extern __shared__ dc s_mem[];
  const int C = p.C;
  const int nseg = p.nseg;
  dc* A0 = s_mem;
  dc* A1 = s_mem + nseg * C;
  double* s_misc = reinterpret_cast<double*>(s_mem + 2 * nseg * C);  // [C]: column-0 extras

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
  const int Kb1 = p.Kb + 1;

  f2* __restrict__ T = p.T + b * p.img_t + l;
  f2* __restrict__ SD = p.SD + b * p.img_sd + l;

  // weight of the Dirac at r0: -sum(du) * w_N^(l c0)
  double S = 0.0;
  for (int j = 0; j < p.nsums; ++j) S += p.sums[(long long)b * p.nsums + j];
  dc dv = {0.0, 0.0};
  if (col_ok) {
    const f2 ph = p.dshift[l];
    dv = {-S * double(ph.x), -S * double(ph.y)};
  }

  double rho = 1.0;
  if (col_ok && !dcol) rho = p.cc[l].rho;

  f2 creg[LMAX];
  dc st = {0.0, 0.0};
  dc mu = {0.0, 0.0};
  double pw = 1.0;
  if (col_ok) {
#pragma unroll
    for (int j = 0; j < LMAX; ++j) {
      if (j < Ls) {
        const int y = p0 + j;
        const f2 x = T[(long long)y * p.NH];
        if (dcol) {
          st = {st.x + x.x, st.y + x.y};  // inclusive prefix sum
          creg[j] = f2{float(st.x), float(st.y)};
        } else {
          st = dfma(rho, st, dc{x.x, x.y});
          creg[j] = f2{float(st.x), float(st.y)};
          mu = dfma(pw, st, mu);
          pw *= rho;
        }
      }
    }
  }
  A0[s * C + c] = st;
  A1[s * C + c] = mu;
  __syncthreads();

  if (s == 0 && col_ok) {
    if (dcol) {
      // Column 0: q = -D_y v with D_yy v = x - mean(x) on Z_M, x = column plus the Dirac;
      // q[y] = -(P[y] - mean(P)), P[y] = sum_{j <= y} (x[j] - xbar). Only q is needed
      // (the x-derivative symbol vanishes at l = 0).
      dc pre = {0.0, 0.0};
      double sumP = 0.0;  // sum over rows [0, R) of the inclusive prefix (no xbar yet)
      for (int t = 0; t < nseg; ++t) {
        const dc e = A0[t * C + c];
        A0[t * C + c] = pre;
        pre = dadd(pre, e);
      }
      const double Mr = double(p.M);
      const double tot = pre.x + dv.x;  // sum of x over the whole column
      const double xbar = tot / Mr;
      s_misc[0] = xbar;
      s_misc[1] = pre.x;
      s_misc[2] = dv.x;
      // mean of P over Z_M is needed; P = Pin (inclusive prefix of x) - xbar * (y + 1).
      // Rows [R, M): Pin = pre for y < r0, pre + dv for y >= r0.
      // The in-block part sum_{y<R} Pin[y] is reduced after the threads publish it.
      (void)sumP;
    }
  }
  __syncthreads();
  // column 0 needs sum_{y<R} Pin[y]: each thread of column 0 adds its rows, reduce in LDS
  if (dcol) {
    double part = 0.0;
    if (col_ok) {
      const double pre_s = A0[s * C + c].x;
#pragma unroll
      for (int j = 0; j < LMAX; ++j)
        if (j < Ls) part += pre_s + double(creg[j].x);
    }
    A1[s * C + c] = dc{part, 0.0};
  }
  __syncthreads();
  if (s == 0 && col_ok) {
    if (dcol) {
      double sin_ = 0.0;
      for (int t = 0; t < nseg; ++t) sin_ += A1[t * C + c].x;
      const double Mr = double(p.M);
      const double xbar = s_misc[0], pre = s_misc[1], dvx = s_misc[2];
      // rows [R, M): Pin = pre (+ dv from r0 on)
      const double sout = pre * (Mr - double(R)) + dvx * (Mr - double(p.r0));
      // sum_y xbar (y + 1) over y in [0, M) = xbar M (M + 1) / 2
      const double meanP = (sin_ + sout - xbar * Mr * (Mr + 1.0) * 0.5) / Mr;
      s_misc[3] = meanP;
    } else {
      const ColConst k = p.cc[l];
      dc Cc = {0.0, 0.0};
      for (int t = 0; t < nseg; ++t) {
        const dc e = A0[t * C + c];
        A0[t * C + c] = Cc;
        Cc = dfma(t == nseg - 1 ? k.rhoLl : k.rhoL, Cc, e);
      }
      const dc cR1 = Cc;
      const dc gam = dfma(k.cgd, dv, dscale(cR1, k.cg));
      dc Sw = {0.0, 0.0};
      double rp = 1.0;
      for (int t = 0; t < nseg; ++t) {
        const dc Dt = dfma(rp, gam, dscale(A0[t * C + c], rho));
        A0[t * C + c] = Dt;
        const dc zst = dfma(t == nseg - 1 ? k.gLl : k.gL, Dt, A1[t * C + c]);
        A1[t * C + c] = zst;
        Sw = dfma(rp, zst, Sw);
        rp *= k.rhoL;
      }
      const dc wR1 = dfma(k.rhoRm1, gam, cR1);
      dc Z = dfma(k.cTd, dv, dfma(k.cT, wR1, dscale(Sw, k.czR)));
      for (int t = nseg - 1; t >= 0; --t) {
        const dc zst = A1[t * C + c];
        A1[t * C + c] = Z;
        Z = dfma(t == nseg - 1 ? k.rhoLl : k.rhoL, Z, zst);
      }
    }
  }
  __syncthreads();

  if (col_ok) {
    if (dcol) {
      const double xbar = s_misc[0], meanP = s_misc[3];
      const double outs = p.cc[0].outs;
      const double pre_s = A0[s * C].x;
#pragma unroll
      for (int j = 0; j < LMAX; ++j) {
        const int y = p0 + j;
        if (j < Ls) {
          const double P = pre_s + double(creg[j].x) - xbar * double(y + 1);
          SD[(long long)y * Kb1] = f2{float(-(P - meanP) * outs), 0.f};
          T[(long long)y * p.NH] = f2{0.f, 0.f};
        }
      }
      if (s == nseg - 1) T[(long long)R * p.NH] = f2{0.f, 0.f};
    } else {
      const dc D = A0[s * C + c];
      dc z = A1[s * C + c];
      const double inv_rho = p.cc[l].inv_rho;
      const double outs = p.cc[l].outs;
      const double omr = p.cc[l].omr;
      if (s == nseg - 1) T[(long long)R * p.NH] = f2{float(z.x * outs), float(z.y * outs)};
      double pj = (s == nseg - 1 ? p.cc[l].rhoLl : p.cc[l].rhoL) * inv_rho;
#pragma unroll
      for (int j = LMAX - 1; j >= 0; --j) {
        if (j < Ls) {
          const int y = p0 + j;
          const dc w = dfma(pj, D, dc{creg[j].x, creg[j].y});
          if (low) {
            const dc q = {w.x - omr * z.x, w.y - omr * z.y};
            SD[(long long)y * Kb1] = f2{float(q.x * outs), float(q.y * outs)};
          }
          z = dfma(rho, z, w);
          T[(long long)y * p.NH] = f2{float(z.x * outs), float(z.y * outs)};
          pj *= inv_rho;
        }
      }
    }
  }
}

hipError_t launch_col_fwd(const ColFwdArgs& a, int B, hipStream_t s) {
  const size_t shm = size_t(2 * a.nseg * a.C) * sizeof(dc) + size_t(a.C) * sizeof(double);
  dim3 grid((a.NH + a.C - 1) / a.C, B);
  hipLaunchKernelGGL(k_col_fwd<kColLmax>, grid, dim3(a.C * a.nseg), shm, s, a);
  return hipGetLastError();
}

hipError_t launch_col_bwd(const ColBwdArgs& a, int B, hipStream_t s) {
  const size_t shm = size_t(2 * a.nseg * a.C) * sizeof(dc) + size_t(a.C + 4) * sizeof(double);
  dim3 grid((a.NH + a.C - 1) / a.C, B);
  hipLaunchKernelGGL(k_col_bwd<kColLmax>, grid, dim3(a.C * a.nseg), shm, s, a);
  return hipGetLastError();
}

}  // namespace gfc
