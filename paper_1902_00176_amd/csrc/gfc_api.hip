// gfc_api.hip - plan, float64 table construction and the C ABI entry points.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "gfc.h"
#include "gfc_internal.h"
#include "gfc_plan.h"

using namespace gfc;

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

bool smooth235(long n) {
  if (n <= 0) return false;
  for (long p : {2L, 3L, 5L})
    while (n % p == 0) n /= p;
  return n == 1;
}
int smooth_at_least(long n) {
  long m = n < 2 ? 2 : n;
  while (!(m % 2 == 0 && smooth235(m))) ++m;
  return int(m);
}

// (cos, sin) of 2 pi e / n with exact integer reduction of e
void cs2pi(long e, long n, double& c, double& s) {
  e %= n;
  if (e < 0) e += n;
  const double t = 2.0 * kPi * double(e) / double(n);
  c = std::cos(t);
  s = std::sin(t);
}

// Segments of exactly Lseg rows; the block is widened to nseg * Lseg rows when those rows
// and the reference row r0 still fall in the zero part of the torus, else the last
// segment is shorter (tail).
ColGeom col_geometry(int R, int M, int r0, int rows, int C_req) {
  ColGeom g;
  if ((R + rows - 1) / rows > kColMaxThreads) rows = 32;
  g.Lseg = rows;
  g.nseg = (R + rows - 1) / rows;
  const int Rp = g.nseg * rows;
  g.tail = !(Rp < M && r0 >= Rp);
  g.Rp = g.tail ? R : Rp;
  g.Llast = g.Rp - (g.nseg - 1) * rows;
  int C = C_req;
  while (C > 1 && C * g.nseg > kColMaxThreads) C /= 2;
  g.C = C;
  return g;
}

}  // namespace

// Per column (kz, l) of a P x M x N problem (P = 1 for images): the recursion constants for
// beta = 4 sin^2(pi l / N) + 4 sin^2(pi kz / P), the output scale 1 / (N P) (the row and z
// inverse transforms are unnormalised), and the reference weights for the corner at
// (z0, r0, c0). Output [P][NH].
void fill_colconst(const gfc_plan_s& p, const ColGeom& g, bool forward,
                   std::vector<ColConst>& out, int P, int z0) {
  const int R = g.Rp;
  out.assign(size_t(P) * p.NH, ColConst{});
  const double M = p.M, N = p.N;
  for (int kz = 0; kz < P; ++kz)
  for (int l = 0; l < p.NH; ++l) {
    ColConst k{};
    if (l == 0 && kz == 0) {
      k.rho = 1.0;
      k.inv_rho = 1.0;
      k.outs = 1.0 / (N * P);
      k.kseg = g.nseg;
      out[size_t(kz) * p.NH + l] = k;
      continue;
    }
    const double sn = std::sin(kPi * double(l) / N);
    const double sz = std::sin(kPi * double(kz) / double(P));
    const double beta = 4.0 * sn * sn + 4.0 * sz * sz;
    const double sq = std::sqrt(beta + 0.25 * beta * beta);
    const double den = 1.0 + 0.5 * beta + sq;
    const double rho = 1.0 / den;
    const double lr = -std::log1p(0.5 * beta + sq);  // log(rho)
    auto pw = [&](double n) { return n <= 0 ? 1.0 : std::exp(n * lr); };
    auto one_minus_pw = [&](double n) { return n <= 0 ? 0.0 : -std::expm1(n * lr); };
    k.rho = rho;
    k.inv_rho = den;
    k.omr = (0.5 * beta + sq) / den;
    const double one_m_r2 = k.omr * (1.0 + rho);
    const double inv1mrM = 1.0 / one_minus_pw(M);
    k.outs = -rho / (N * P);
    k.rhoL = pw(g.Lseg);
    k.rhoLl = pw(g.Llast);
    // rho^d < 2^-64 for d >= dmax rows; carries from further than that are dropped
    const double dmax = std::ceil(64.0 * std::log(2.0) / -lr);
    const double ks = std::ceil(dmax / g.Lseg) + 1.0;
    k.kseg = ks >= double(g.nseg) ? g.nseg : int(ks);
    k.gL = one_minus_pw(2.0 * g.Lseg) / one_m_r2;
    k.gLl = one_minus_pw(2.0 * g.Llast) / one_m_r2;
    k.cg = pw(M - R + 1) * inv1mrM;
    k.rhoRm1 = pw(R - 1);
    k.cT = rho * one_minus_pw(2.0 * (M - R)) / one_m_r2 * inv1mrM;
    k.czR = pw(M - R) * inv1mrM;
    const double r0 = p.r0;
    k.ra = pw(r0 - R + 1) * one_minus_pw(2.0 * (M - r0)) / one_m_r2;
    k.rb = pw(M - r0);
    k.cgd = pw(M - r0) * inv1mrM;
    k.cTd = pw(r0 - R) * one_minus_pw(2.0 * (M - r0)) / one_m_r2 * inv1mrM;
    if (forward) {
      // angle 2 pi (l c0 / N + kz z0 / P), reduced exactly as one fraction of N P
      double c, s;
      cs2pi(long(l) * p.c0 * P + long(kz) * z0 * p.N, long(p.N) * P, c, s);
      const double wgt = (l == 0 || 2 * l == p.N) ? 1.0 : 2.0;  // Hermitian pairs in l
      k.wre = wgt * k.outs * c;
      k.wim = wgt * k.outs * s;
    }
    out[size_t(kz) * p.NH + l] = k;
  }
}

namespace {

// launch geometry that follows from the sizes and the tunable parameters
// Row bins handed to the column pass in split form. The rounding of the row FFT in bins
// l > K reaches the solution amplified by about N / (K M) (the column frequency 0 carries
// about 1/M of it, the Green's function 1/lambda_l grows as (N / l)^2, the split form's error
// shrinks with l): the smallest K in {4, 8, 16, 32} with N <= 16 K M keeps it near 2e-6
// for float32 input, and only thin, wide tori need more than kLowBins.
int auto_low_bins(int M, int N) {
  int K = kLowBins;
  while (K < kMaxLowBins && (long long)N > 16LL * K * M) K *= 2;
  return std::min(K, std::max(kLowBins, N / 2 - 1));
}

void derive_geometry(gfc_plan_s* p) {
  p->KP = (p->K + 1 + 7) / 8 * 8;
  p->gf = col_geometry(p->H + 1, p->M, p->r0, p->col_rows, p->col_c);
  p->gb = col_geometry(p->H, p->M, p->r0, p->col_rows_b, p->col_c);
  p->nfslots = (p->H + 2) / 2;  // one pair of divergence rows per slot
  p->npairs = (p->H + 1) / 2;
  p->ntiles_f = (p->NH + p->gf.C - 1) / p->gf.C;
  p->ntiles_b = (p->NH + p->gb.C - 1) / p->gb.C;
  p->nsums = (p->npairs + p->rk->bf.slots - 1) / p->rk->bf.slots;
}

}  // namespace

extern "C" {

const char* gfc_status_str(gfc_status s) {
  switch (s) {
    case GFC_OK: return "GFC_OK";
    case GFC_E_ARG: return "GFC_E_ARG";
    case GFC_E_SIZE: return "GFC_E_SIZE";
    case GFC_E_NOT_BUILT: return "GFC_E_NOT_BUILT";
    case GFC_E_WORKSPACE: return "GFC_E_WORKSPACE";
    case GFC_E_HIP: return "GFC_E_HIP";
    case GFC_E_OOM: return "GFC_E_OOM";
  }
  return "GFC_E_UNKNOWN";
}

int gfc_supported_length(int N) { return find_row_kernels(N) != nullptr ? 1 : 0; }

gfc_status gfc_plan_create(gfc_plan_t* out, int H, int W, int M, int N, unsigned flags) {
  if (!out) return GFC_E_ARG;
  *out = nullptr;
  if (H < 1 || W < 1 || M < 0 || N < 0 || flags != GFC_FLAG_NONE) return GFC_E_ARG;
  // the column pass holds a whole column in one workgroup: at most 1024 segments of 32 rows
  if (H >= (1 << 15) || W > (1 << 15)) return GFC_E_SIZE;
  // default torus: the smallest even 2/3/5-smooth M >= 2H and N >= 2W, at least H + 2 and
  // W + 2, and N at least the shortest row FFT (16)
  if (M == 0) M = smooth_at_least(std::max(2L * H, H + 2L));
  if (N == 0) N = smooth_at_least(std::max({2L * W, W + 2L, 16L}));
  if (M < H + 2 || N < W + 2) return GFC_E_SIZE;
  const RowKernels* rk = find_row_kernels(N);
  if (!rk) return GFC_E_SIZE;
  auto* p = new (std::nothrow) gfc_plan_s;
  if (!p) return GFC_E_OOM;
  p->H = H;
  p->W = W;
  p->M = M;
  p->N = N;
  p->NH = N / 2 + 1;
  p->oy = (M - H) / 2;
  p->ox = (N - W) / 2;
  p->r0 = M - p->oy;  // grid corner (0,0) relative to the block at the origin
  p->c0 = N - p->ox;
  p->K = auto_low_bins(M, N);
  p->Kb = std::min(kLowBinsB, p->NH - 1);
  // row strides padded to whole 256-byte lines so column tiles never straddle cache lines
  p->NHP = (p->NH + 31) / 32 * 32;
  // kernels address one image's buffers with 32-bit offsets below 2^30
  if ((long long)(H + 1) * p->NHP * 8 >= (1LL << 30) || (long long)H * W * 4 >= (1LL << 30)) {
    delete p;
    return GFC_E_SIZE;
  }
  p->KbP = (p->Kb + 1 + 31) / 32 * 32;
  p->flags = flags;
  p->rk = rk;
  derive_geometry(p);
  *out = p;
  return GFC_OK;
}

gfc_status gfc_plan_get(gfc_plan_t p, int* H, int* W, int* M, int* N, int* oy, int* ox) {
  if (!p) return GFC_E_ARG;
  if (H) *H = p->H;
  if (W) *W = p->W;
  if (M) *M = p->M;
  if (N) *N = p->N;
  if (oy) *oy = p->oy;
  if (ox) *ox = p->ox;
  return GFC_OK;
}

gfc_status gfc_plan_set_param(gfc_plan_t p, const char* name, int value) {
  if (!p || !name) return GFC_E_ARG;
  if (p->built) return GFC_E_ARG;  // the float64 tables depend on the geometry
  if (!std::strcmp(name, "col_c")) {
    if (value < 1 || value > 64 || (value & (value - 1))) return GFC_E_ARG;
    p->col_c = value;
  } else if (!std::strcmp(name, "col_rows")) {
    if (value != 16 && value != 32) return GFC_E_ARG;
    p->col_rows = value;
  } else if (!std::strcmp(name, "col_rows_b")) {
    if (value != 16 && value != 32) return GFC_E_ARG;
    p->col_rows_b = value;
  } else if (!std::strcmp(name, "low_bins")) {
    if (value < kLowBins || value > kMaxLowBins || 2 * value >= p->N) return GFC_E_ARG;
    p->K = value;
  } else if (!std::strcmp(name, "row_split")) {
    const RowKernels* rk = find_row_kernels_split(p->N, value);
    if (!rk) return GFC_E_ARG;
    p->rk = rk;
  } else {
    return GFC_E_ARG;
  }
  derive_geometry(p);
  return GFC_OK;
}

gfc_status gfc_plan_get_param(gfc_plan_t p, const char* name, int* value) {
  if (!p || !name || !value) return GFC_E_ARG;
  if (!std::strcmp(name, "col_c")) *value = p->gf.C;
  else if (!std::strcmp(name, "col_rows")) *value = p->col_rows;
  else if (!std::strcmp(name, "col_rows_b")) *value = p->col_rows_b;
  else if (!std::strcmp(name, "low_bins")) *value = p->K;
  else if (!std::strcmp(name, "low_bins_b")) *value = p->Kb;
  else if (!std::strcmp(name, "row_split")) *value = p->rk->f.N1;
  else if (!std::strcmp(name, "row_split_fwd")) *value = p->rk->f.N1;
  else if (!std::strcmp(name, "row_split_edit")) *value = p->rk->e.N1;
  else if (!std::strcmp(name, "row_split_inv")) *value = p->rk->i.N1;
  else if (!std::strcmp(name, "row_split_bfwd")) *value = p->rk->bf.N1;
  else if (!std::strcmp(name, "row_split_binv")) *value = p->rk->bi.N1;
  else return GFC_E_ARG;
  return GFC_OK;
}

gfc_status gfc_green_build(gfc_plan_t p, void* stream) {
  if (!p) return GFC_E_ARG;
  if (p->built) return GFC_OK;
  const int N = p->N, NH = p->NH;
  // four-step twiddles w_N^(k1 j) of each pass's split N = N1 N2: [N1][N2] for a forward
  // transform (forward and backward-forward row passes), [N2][N1] for an inverse one
  auto tw_fwd = [&](const RowSplit& q) {
    std::vector<f2> t(size_t(q.N1) * q.N2);
    for (int k1 = 0; k1 < q.N1; ++k1)
      for (int j = 0; j < q.N2; ++j) {
        double c, s;
        cs2pi(long(k1) * j, N, c, s);
        t[size_t(k1) * q.N2 + j] = f2{float(c), float(-s)};
      }
    return t;
  };
  auto tw_inv = [&](const RowSplit& q) {
    std::vector<f2> t(size_t(q.N1) * q.N2);
    for (int k1 = 0; k1 < q.N1; ++k1)
      for (int j = 0; j < q.N2; ++j) {
        double c, s;
        cs2pi(long(k1) * j, N, c, s);
        t[size_t(j) * q.N1 + k1] = f2{float(c), float(-s)};
      }
    return t;
  };
  const std::vector<f2> twA = tw_fwd(p->rk->f), twAe = tw_fwd(p->rk->e);
  const std::vector<f2> twB = tw_inv(p->rk->i);
  const std::vector<f2> twAb = tw_fwd(p->rk->bf), twBb = tw_inv(p->rk->bi);
  std::vector<f2> dsh(NH);
  // low-bin twiddles of a forward row pass, lane j < N2 of a G-lane slot:
  // [0][l][j] = (1 - w_N^l) w_N^(l j) for Ex, [1][l][j] = w_N^(l j) for Ey (0 for j >= N2)
  const int K1 = kLowBins + 1;
  auto tw_low = [&](const RowSplit& q) {
    std::vector<f2> t(size_t(2) * K1 * q.G, f2{0.f, 0.f});
    for (int l = 0; l < K1; ++l) {
      const double h = std::sin(kPi * double(l) / double(N));
      double c, s;
      cs2pi(l, N, c, s);
      const double ar = 2.0 * h * h, ai = s;  // 1 - e^{-i 2 pi l / N}
      for (int j = 0; j < q.N2; ++j) {
        double cj, sj;
        cs2pi(long(l) * j, N, cj, sj);
        const double wr = cj, wi = -sj;  // e^{-i 2 pi l j / N}
        t[size_t(l) * q.G + j] = f2{float(ar * wr - ai * wi), float(ar * wi + ai * wr)};
        t[size_t(K1 + l) * q.G + j] = f2{float(wr), float(wi)};
      }
    }
    return t;
  };
  const std::vector<f2> twL = tw_low(p->rk->f), twLe = tw_low(p->rk->e);
  // direct-sum twiddles of the extra split bins: w_N^m for m < N, then 1 - w_N^l
  std::vector<f2> twX(size_t(N) + kMaxLowBins + 1);
  for (int m = 0; m < N; ++m) {
    double c, s;
    cs2pi(m, N, c, s);
    twX[m] = f2{float(c), float(-s)};
  }
  for (int l = 0; l <= kMaxLowBins; ++l) {
    const double h = std::sin(kPi * double(l) / double(N));
    double c, s;
    cs2pi(l, N, c, s);
    twX[size_t(N) + l] = f2{float(2.0 * h * h), float(s)};
  }
  for (int l = 0; l < NH; ++l) {
    double c, s;
    cs2pi(long(l) * p->c0, N, c, s);
    dsh[l] = f2{float(c), float(-s)};    // e^{-2 pi i l c0 / N}
  }
  // float64 w_N^m = e^{-2 pi i m / N}, m < N: direct sums of a given Laplacian's low bins
  std::vector<double> twD(size_t(2) * N);
  for (int m = 0; m < N; ++m) {
    double c, sn;
    cs2pi(m, N, c, sn);
    twD[2 * size_t(m)] = c;
    twD[2 * size_t(m) + 1] = -sn;
  }
  std::vector<ColConst> ccf, ccb;
  fill_colconst(*p, p->gf, true, ccf, 1, 0);
  fill_colconst(*p, p->gb, false, ccb, 1, 0);

  size_t off = 0;
  const size_t o_twA = off; off = align256(off + twA.size() * sizeof(f2));
  const size_t o_twB = off; off = align256(off + twB.size() * sizeof(f2));
  const size_t o_twAb = off; off = align256(off + twAb.size() * sizeof(f2));
  const size_t o_twBb = off; off = align256(off + twBb.size() * sizeof(f2));
  const size_t o_twL = off; off = align256(off + twL.size() * sizeof(f2));
  const size_t o_twAe = off; off = align256(off + twAe.size() * sizeof(f2));
  const size_t o_twLe = off; off = align256(off + twLe.size() * sizeof(f2));
  const size_t o_twX = off; off = align256(off + twX.size() * sizeof(f2));
  const size_t o_dsh = off; off = align256(off + dsh.size() * sizeof(f2));
  const size_t o_ccf = off; off = align256(off + ccf.size() * sizeof(ColConst));
  const size_t o_ccb = off; off = align256(off + ccb.size() * sizeof(ColConst));
  const size_t o_twD = off; off = align256(off + twD.size() * sizeof(double));
  std::vector<unsigned char> host(off, 0);
  std::memcpy(host.data() + o_twA, twA.data(), twA.size() * sizeof(f2));
  std::memcpy(host.data() + o_twB, twB.data(), twB.size() * sizeof(f2));
  std::memcpy(host.data() + o_twAb, twAb.data(), twAb.size() * sizeof(f2));
  std::memcpy(host.data() + o_twBb, twBb.data(), twBb.size() * sizeof(f2));
  std::memcpy(host.data() + o_twL, twL.data(), twL.size() * sizeof(f2));
  std::memcpy(host.data() + o_twAe, twAe.data(), twAe.size() * sizeof(f2));
  std::memcpy(host.data() + o_twLe, twLe.data(), twLe.size() * sizeof(f2));
  std::memcpy(host.data() + o_twX, twX.data(), twX.size() * sizeof(f2));
  std::memcpy(host.data() + o_dsh, dsh.data(), dsh.size() * sizeof(f2));
  std::memcpy(host.data() + o_ccf, ccf.data(), ccf.size() * sizeof(ColConst));
  std::memcpy(host.data() + o_ccb, ccb.data(), ccb.size() * sizeof(ColConst));
  std::memcpy(host.data() + o_twD, twD.data(), twD.size() * sizeof(double));

  void* d = nullptr;
  if (hipMalloc(&d, off) != hipSuccess) return GFC_E_OOM;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(d, host.data(), off, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    (void)hipFree(d);
    return GFC_E_HIP;
  }
  auto* base = static_cast<unsigned char*>(d);
  p->dmem = d;
  p->twA = reinterpret_cast<f2*>(base + o_twA);
  p->twB = reinterpret_cast<f2*>(base + o_twB);
  p->twAb = reinterpret_cast<f2*>(base + o_twAb);
  p->twBb = reinterpret_cast<f2*>(base + o_twBb);
  p->twL = reinterpret_cast<f2*>(base + o_twL);
  p->twAe = reinterpret_cast<f2*>(base + o_twAe);
  p->twLe = reinterpret_cast<f2*>(base + o_twLe);
  p->twX = reinterpret_cast<f2*>(base + o_twX);
  p->dshift = reinterpret_cast<f2*>(base + o_dsh);
  p->ccf = reinterpret_cast<ColConst*>(base + o_ccf);
  p->ccb = reinterpret_cast<ColConst*>(base + o_ccb);
  p->twD = reinterpret_cast<double*>(base + o_twD);
  (void)hipGetDevice(&p->device);
  if (hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess)
    return GFC_E_HIP;
  p->built = true;
  return GFC_OK;
}

gfc_status gfc_workspace_size(gfc_plan_t p, int B, size_t* bytes) {
  if (!p || !bytes || B < 0) return GFC_E_ARG;
  *bytes = ws_layout(p, B).total;
  return GFC_OK;
}

gfc_status gfc_solve_batch_stage(gfc_plan_t p, int stage, const float* gx, const float* gy,
                                 float* u, int B, void* workspace, size_t ws_bytes,
                                 void* stream) {
  if (!p || B < 0 || stage < 0 || stage > 3) return GFC_E_ARG;
  if (!p->built) return GFC_E_NOT_BUILT;
  if (B == 0) return GFC_OK;
  if (!workspace) return GFC_E_ARG;
  if ((stage == 0 || stage == 1) && (!gx || !gy)) return GFC_E_ARG;
  if ((stage == 0 || stage == 3) && !u) return GFC_E_ARG;
  const WsLayout w = ws_layout(p, B);
  if (ws_bytes < w.total) return GFC_E_WORKSPACE;
  auto* ws = static_cast<unsigned char*>(workspace);
  f2* T = reinterpret_cast<f2*>(ws + w.t);
  f2* SB = reinterpret_cast<f2*>(ws + w.side);
  double* partial = reinterpret_cast<double*>(ws + w.red);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);

  if (stage == 0 || stage == 1) {
    const RowFwdArgs f = row_fwd_args(p, gx, gy, T, SB);
    gfc_status st = hip_status(p->rk->fwd(f, B, s));
    if (st == GFC_OK) st = hip_status(launch_low_ext(f, B, s));
    if (st != GFC_OK) return st;
  }
  if (stage == 0 || stage == 2) {
    std::lock_guard<std::mutex> fork_lock(p->fork_mtx);
    const gfc_status st = hip_status(launch_col_fwd(col_fwd_args(p, T, SB, partial), B, s,
                                                    p->side, p->ev_fork, p->ev_join));
    if (st != GFC_OK) return st;
  }
  if (stage == 0 || stage == 3) {
    const gfc_status st = hip_status(p->rk->inv(row_inv_args(p, T, u, partial), B, s));
    if (st != GFC_OK) return st;
  }
  return GFC_OK;
}

gfc_status gfc_solve_batch(gfc_plan_t p, const float* gx, const float* gy, float* u, int B,
                           void* workspace, size_t ws_bytes, void* stream) {
  if (!p || B < 0) return GFC_E_ARG;
  if (!p->built) return GFC_E_NOT_BUILT;
  if (B == 0) return GFC_OK;
  return gfc_solve_batch_stage(p, 0, gx, gy, u, B, workspace, ws_bytes, stream);
}

// forward solve with an optional gradient edit before the divergence and an optional
// colour correction after the inverse row pass
static gfc_status solve_forward(gfc_plan_t p, const float* gx, const float* gy, const float* C,
                                int edit, float tau2, float alpha, const float* I_mean,
                                const float* I_std, float* u, int B, void* workspace,
                                size_t ws_bytes, void* stream) {
  const WsLayout w = ws_layout(p, B);
  if (ws_bytes < w.total) return GFC_E_WORKSPACE;
  auto* ws = static_cast<unsigned char*>(workspace);
  f2* T = reinterpret_cast<f2*>(ws + w.t);
  f2* SB = reinterpret_cast<f2*>(ws + w.side);
  double* partial = reinterpret_cast<double*>(ws + w.red);
  double* mom = reinterpret_cast<double*>(ws + w.mom);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  RowFwdArgs f = row_fwd_args(p, gx, gy, T, SB);
  f.edit = edit;
  f.C = C;
  f.tau2 = tau2;
  f.alpha = alpha;
  if (edit != kEditNone) {  // the edited and Laplacian forward modes use their own split
    f.twA = p->twAe;
    f.twL = p->twLe;
  }
  gfc_status st = hip_status(p->rk->fwd(f, B, s));
  if (st != GFC_OK) return st;
  if (edit != kInLaplacian) {
    st = hip_status(launch_low_ext(f, B, s));
    if (st != GFC_OK) return st;
  }
  if (edit == kInLaplacian) {
    LapLowArgs la{};
    la.L = C;
    la.twD = p->twD;
    la.Lh = reinterpret_cast<double*>(ws + w.lap);
    la.T1 = T;
    la.SB = SB;
    la.H = p->H;
    la.W = p->W;
    la.N = p->N;
    la.K = p->K;
    la.NHP = p->NHP;
    la.KP = p->KP;
    la.img_L = (long long)(p->H + 1) * (p->W + 1);
    la.img_lh = (long long)(p->H + 1) * (p->K + 1) * 2;
    la.img_t1 = f.img_t1;
    la.img_sb = f.img_sb;
    st = hip_status(launch_lap_low(la, B, s));
    if (st != GFC_OK) return st;
  }
  {
    std::lock_guard<std::mutex> fork_lock(p->fork_mtx);
    st = hip_status(launch_col_fwd(col_fwd_args(p, T, SB, partial), B, s, p->side, p->ev_fork,
                                   p->ev_join));
  }
  if (st != GFC_OK) return st;
  RowInvArgs v = row_inv_args(p, T, u, partial);
  const bool color = I_mean != nullptr;
  v.mom = color ? mom : nullptr;
  st = hip_status(p->rk->inv(v, B, s));
  if (st != GFC_OK || !color) return st;
  return hip_status(launch_color_apply(u, mom, inv_groups(p), I_mean, I_std,
                                       (long long)p->H * p->W, B, s));
}

gfc_status gfc_solve_batch_color(gfc_plan_t p, const float* gx, const float* gy,
                                 const float* I_mean, const float* I_std, float* u, int B,
                                 void* workspace, size_t ws_bytes, void* stream) {
  if (!p || B < 0) return GFC_E_ARG;
  if (!p->built) return GFC_E_NOT_BUILT;
  if (B == 0) return GFC_OK;
  if (!workspace || !gx || !gy || !u || !I_mean || !I_std) return GFC_E_ARG;
  return solve_forward(p, gx, gy, nullptr, kEditNone, 0.f, 0.f, I_mean, I_std, u, B, workspace,
                       ws_bytes, stream);
}

gfc_status gfc_solve_laplacian(gfc_plan_t p, const float* L, float* u, int B, void* workspace,
                               size_t ws_bytes, void* stream) {
  if (!p || B < 0) return GFC_E_ARG;
  if (!p->built) return GFC_E_NOT_BUILT;
  if (B == 0) return GFC_OK;
  if (!workspace || !L || !u) return GFC_E_ARG;
  if ((long long)(p->H + 1) * (p->W + 1) * 4 >= (1LL << 30)) return GFC_E_SIZE;
  return solve_forward(p, nullptr, nullptr, L, kInLaplacian, 0.f, 0.f, nullptr, nullptr, u, B,
                       workspace, ws_bytes, stream);
}

gfc_status gfc_solve_edit(gfc_plan_t p, const float* gx, const float* gy, const float* C,
                          int mode, float param, const float* I_mean, const float* I_std,
                          float* u, int B, void* workspace, size_t ws_bytes, void* stream) {
  if (!p || B < 0) return GFC_E_ARG;
  if (!p->built) return GFC_E_NOT_BUILT;
  if (mode != GFC_EDIT_THRESHOLD && mode != GFC_EDIT_GDM) return GFC_E_ARG;
  if (mode == GFC_EDIT_THRESHOLD && !(param >= 0.f)) return GFC_E_ARG;
  if (mode == GFC_EDIT_GDM && !(param >= 0.f && param <= 1.f)) return GFC_E_ARG;
  if ((I_mean == nullptr) != (I_std == nullptr)) return GFC_E_ARG;
  if (B == 0) return GFC_OK;
  if (!workspace || !gx || !gy || !u || (mode == GFC_EDIT_GDM && !C)) return GFC_E_ARG;
  const float tau2 = mode == GFC_EDIT_THRESHOLD ? param * param : 0.f;  // rounded once
  const float alpha = mode == GFC_EDIT_GDM ? param : 0.f;
  return solve_forward(p, gx, gy, C, mode == GFC_EDIT_THRESHOLD ? kEditThreshold : kEditGdm,
                       tau2, alpha, I_mean, I_std, u, B, workspace, ws_bytes, stream);
}

gfc_status gfc_solve_backward_stage(gfc_plan_t p, int stage, const float* du, float* dgx,
                                    float* dgy, int B, void* workspace, size_t ws_bytes,
                                    void* stream) {
  if (!p || B < 0 || stage < 0 || stage > 3) return GFC_E_ARG;
  if (!p->built) return GFC_E_NOT_BUILT;
  if (B == 0) return GFC_OK;
  if (!workspace) return GFC_E_ARG;
  if ((stage == 0 || stage == 1) && !du) return GFC_E_ARG;
  if ((stage == 0 || stage == 3) && (!dgx || !dgy)) return GFC_E_ARG;
  const WsLayout w = ws_layout(p, B);
  if (ws_bytes < w.total) return GFC_E_WORKSPACE;
  auto* ws = static_cast<unsigned char*>(workspace);
  f2* T = reinterpret_cast<f2*>(ws + w.t);
  f2* SD = reinterpret_cast<f2*>(ws + w.side);
  double* sums = reinterpret_cast<double*>(ws + w.red);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long long img_t = (long long)(p->H + 1) * p->NHP;
  const long long img_sd = (long long)p->H * p->KbP;

  if (stage == 0 || stage == 1) {
    RowBwdFwdArgs a{};
    a.du = du;
    a.U = T;
    a.sums = sums;
    a.twA = p->twAb;
    a.H = p->H;
    a.W = p->W;
    a.npairs = (p->H + 1) / 2;
    a.img_in = (long long)p->H * p->W;
    a.img_u = img_t;
    const gfc_status st = hip_status(p->rk->bfwd(a, B, s));
    if (st != GFC_OK) return st;
  }
  if (stage == 0 || stage == 2) {
    ColBwdArgs c{};
    c.T = T;
    c.SD = SD;
    c.cc = p->ccb;
    c.sums = sums;
    c.dshift = p->dshift;
    c.nsums = p->nsums;
    c.H = p->H;
    c.M = p->M;
    c.NH = p->NH;
    c.NHP = p->NHP;
    c.Kb = p->Kb;
    c.KbP = p->KbP;
    c.r0 = p->r0;
    c.C = p->gb.C;
    c.nseg = p->gb.nseg;
    c.Lseg = p->gb.Lseg;
    c.Llast = p->gb.Llast;
    c.Rp = p->gb.Rp;
    c.img_t = img_t;
    c.img_sd = img_sd;
    c.nimg = B;
    std::lock_guard<std::mutex> fork_lock(p->fork_mtx);
    const gfc_status st =
        hip_status(launch_col_bwd(c, B, s, p->side, p->ev_fork, p->ev_join));
    if (st != GFC_OK) return st;
  }
  if (stage == 0 || stage == 3) {
    RowBwdInvArgs v{};
    v.Wv = T;
    v.SD = SD;
    v.dgx = dgx;
    v.dgy = dgy;
    v.twB = p->twBb;
    v.H = p->H;
    v.W = p->W;
    v.Kb = p->Kb;
    v.KbP = p->KbP;
    v.img_w = img_t;
    v.img_sd = img_sd;
    v.img_out = (long long)p->H * p->W;
    const gfc_status st = hip_status(p->rk->binv(v, B, s));
    if (st != GFC_OK) return st;
  }
  return GFC_OK;
}

gfc_status gfc_solve_backward(gfc_plan_t p, const float* du, float* dgx, float* dgy, int B,
                              void* workspace, size_t ws_bytes, void* stream) {
  if (!p || B < 0) return GFC_E_ARG;
  if (!p->built) return GFC_E_NOT_BUILT;
  if (B == 0) return GFC_OK;
  return gfc_solve_backward_stage(p, 0, du, dgx, dgy, B, workspace, ws_bytes, stream);
}

gfc_status gfc_green_export(gfc_plan_t p, double* out) {
  if (!p || !out) return GFC_E_ARG;
  for (int k = 0; k < p->M; ++k) {
    const double sk = std::sin(kPi * double(k) / double(p->M));
    for (int l = 0; l < p->NH; ++l) {
      const double sl = std::sin(kPi * double(l) / double(p->N));
      const double lam = -4.0 * sk * sk - 4.0 * sl * sl;
      out[size_t(k) * p->NH + l] = (k == 0 && l == 0) ? 0.0 : 1.0 / lam;
    }
  }
  return GFC_OK;
}

void gfc_plan_destroy(gfc_plan_t p) {
  if (!p) return;
  if (p->dmem) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (p->device >= 0 && cur != p->device) (void)hipSetDevice(p->device);
    (void)hipFree(p->dmem);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    if (p->side) (void)hipStreamDestroy(p->side);
    if (cur >= 0 && cur != p->device) (void)hipSetDevice(cur);
  }
  delete p;
}


// ---- volumes (n-D GFC, three dimensions) --------------------------------------------------

}  // extern "C"


struct gfc_plan3_s {
  gfc_plan_s* p2 = nullptr;  // the (y, x) part: H, W, M, N, row kernels, column geometry
  int D = 0, P = 0, oz = 0, z0 = 0;
  const gfc::ZKernels* zk = nullptr;
  bool built = false;
  void* dmem = nullptr;
  gfc::ColConst* cc = nullptr;  // [P][NH]
  gfc::f2* tw = nullptr;        // [P1][P2]
  gfc::f2* omz = nullptr;       // [P]: 1 - w_P^kz, the z difference as its symbol
};

namespace {
struct Ws3 {
  size_t t, side, sz, red, tot, total;  // side: SB, sz: SZ; tot: corner sums per volume
};
Ws3 ws3_layout(const gfc_plan3_s* q, int B) {
  const gfc_plan_s* p = q->p2;
  Ws3 w{};
  const size_t vols = size_t(B) * q->P;
  const size_t side = align256(vols * size_t(p->H) * p->KP * sizeof(f2));
  w.t = 0;
  w.side = align256(vols * size_t(p->H + 1) * p->NHP * sizeof(f2));
  w.sz = w.side + side;
  w.red = w.sz + side;
  w.tot = w.red + align256(vols * size_t(p->ntiles_f) * sizeof(double));
  w.total = w.tot + align256(size_t(B) * sizeof(double));
  return w;
}
}  // namespace

extern "C" {

gfc_status gfc_plan3_create(gfc_plan3_t* out, int D, int H, int W, int P, int M, int N,
                            unsigned flags) {
  if (!out) return GFC_E_ARG;
  *out = nullptr;
  if (D < 1 || P < 0 || flags != GFC_FLAG_NONE) return GFC_E_ARG;
  if (P == 0) P = smooth_at_least(2L * D);
  if (P < D + 2) return GFC_E_SIZE;
  const ZKernels* zk = find_z_kernels(P);
  if (!zk) return GFC_E_SIZE;
  gfc_plan_t p2 = nullptr;
  const gfc_status st = gfc_plan_create(&p2, H, W, M, N, flags);
  if (st != GFC_OK) return st;
  // a volume's (P planes) spectra must stay addressable with 32-bit offsets per plane set
  if ((long long)P * (p2->H + 1) * p2->NHP * 8 >= (1LL << 31) ||
      (long long)D * H * W * 4 >= (1LL << 30)) {
    gfc_plan_destroy(p2);
    return GFC_E_SIZE;
  }
  // the row bins l <= kLowBins take the split input (x-, y- and z-parts apart); the plane
  // extension for thin tori is for images only
  p2->K = kLowBins;
  derive_geometry(p2);
  auto* q = new (std::nothrow) gfc_plan3_s;
  if (!q) {
    gfc_plan_destroy(p2);
    return GFC_E_OOM;
  }
  q->p2 = p2;
  q->D = D;
  q->P = P;
  q->oz = (P - D) / 2;
  q->z0 = P - q->oz;  // grid corner relative to the volume at the origin
  q->zk = zk;
  *out = q;
  return GFC_OK;
}

gfc_status gfc_plan3_get(gfc_plan3_t q, int* D, int* H, int* W, int* P, int* M, int* N) {
  if (!q) return GFC_E_ARG;
  if (D) *D = q->D;
  if (P) *P = q->P;
  return gfc_plan_get(q->p2, H, W, M, N, nullptr, nullptr);
}

gfc_status gfc_green_build3(gfc_plan3_t q, void* stream) {
  if (!q) return GFC_E_ARG;
  if (q->built) return GFC_OK;
  gfc_status st = gfc_green_build(q->p2, stream);
  if (st != GFC_OK) return st;
  const int P = q->P, P1 = q->zk->P1, P2 = q->zk->P2;
  std::vector<ColConst> cc;
  fill_colconst(*q->p2, q->p2->gf, true, cc, P, q->z0);
  std::vector<f2> tw(size_t(P1) * P2);
  for (int k1 = 0; k1 < P1; ++k1)
    for (int j = 0; j < P2; ++j) {
      double c, s;
      cs2pi(long(k1) * j, P, c, s);
      tw[size_t(k1) * P2 + j] = f2{float(c), float(-s)};
    }
  // 1 - w_P^kz = 2 sin^2(pi kz / P) + i sin(2 pi kz / P)
  std::vector<f2> omz(P);
  for (int kz = 0; kz < P; ++kz) {
    const double h = std::sin(kPi * double(kz) / double(P));
    double c, sn;
    cs2pi(kz, P, c, sn);
    omz[kz] = f2{float(2.0 * h * h), float(sn)};
  }
  const size_t o_cc = 0;
  const size_t o_tw = align256(cc.size() * sizeof(ColConst));
  const size_t o_omz = o_tw + align256(tw.size() * sizeof(f2));
  const size_t total = o_omz + align256(omz.size() * sizeof(f2));
  std::vector<unsigned char> host(total, 0);
  std::memcpy(host.data() + o_cc, cc.data(), cc.size() * sizeof(ColConst));
  std::memcpy(host.data() + o_tw, tw.data(), tw.size() * sizeof(f2));
  std::memcpy(host.data() + o_omz, omz.data(), omz.size() * sizeof(f2));
  void* d = nullptr;
  if (hipMalloc(&d, total) != hipSuccess) return GFC_E_OOM;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(d, host.data(), total, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    (void)hipFree(d);
    return GFC_E_HIP;
  }
  q->dmem = d;
  q->cc = reinterpret_cast<ColConst*>(static_cast<unsigned char*>(d) + o_cc);
  q->tw = reinterpret_cast<f2*>(static_cast<unsigned char*>(d) + o_tw);
  q->omz = reinterpret_cast<f2*>(static_cast<unsigned char*>(d) + o_omz);
  q->built = true;
  return GFC_OK;
}

gfc_status gfc_workspace3_size(gfc_plan3_t q, int B, size_t* bytes) {
  if (!q || !bytes || B < 0) return GFC_E_ARG;
  *bytes = ws3_layout(q, B).total;
  return GFC_OK;
}

gfc_status gfc_solve3_batch(gfc_plan3_t q, const float* gx, const float* gy, const float* gz,
                            float* u, int B, void* workspace, size_t ws_bytes, void* stream) {
  if (!q || B < 0) return GFC_E_ARG;
  if (!q->built) return GFC_E_NOT_BUILT;
  if (B == 0) return GFC_OK;
  if (!gx || !gy || !gz || !u || !workspace) return GFC_E_ARG;
  const Ws3 w = ws3_layout(q, B);
  if (ws_bytes < w.total) return GFC_E_WORKSPACE;
  gfc_plan_s* p = q->p2;
  auto* ws = static_cast<unsigned char*>(workspace);
  f2* T = reinterpret_cast<f2*>(ws + w.t);
  f2* SB = reinterpret_cast<f2*>(ws + w.side);
  f2* SZ = reinterpret_cast<f2*>(ws + w.sz);
  double* partial = reinterpret_cast<double*>(ws + w.red);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int D = q->D, P = q->P;
  const long long plane = (long long)(p->H + 1) * p->NHP;
  const long long splane = (long long)p->H * p->KP;
  // 1. rows of the 7-point divergence, every slice z in [0, D] of every volume; bins
  //    l <= K split: T gets (1 - w_N^l) Ex^, SB gets Ey^ and SZ gets Ez^ of planes z < D
  RowFwdArgs f = row_fwd_args(p, gx, gy, T, SB);
  f.edit = kIn3D;
  f.twA = p->twAe;  // volume slices: the forward split of the non-plain modes
  f.twL = p->twLe;
  f.gz = gz;
  f.zd = D;
  f.zp = P;
  f.SZ = SZ;
  gfc_status st = hip_status(p->rk->fwd(f, B * (D + 1), s));
  if (st != GFC_OK) return st;
  // 2. z transforms: T with D + 1 planes in, the side arrays with D, P planes out each
  ZfftArgs z{};
  z.T = T;
  z.tw = q->tw;
  z.R = p->H + 1;
  z.NH = p->NH;
  z.NHP = p->NHP;
  z.plane = plane;
  z.vol_stride = plane * P;
  z.din = D + 1;
  z.dout = P;
  z.tiled = 1;
  st = hip_status(q->zk->run(z, -1, B, s));
  if (st != GFC_OK) return st;
  ZfftArgs zs = z;
  zs.R = p->H;
  zs.NH = p->K + 1;
  zs.NHP = p->KP;
  zs.plane = splane;
  zs.vol_stride = splane * P;
  zs.din = D;
  zs.tiled = 0;
  zs.T = SB;
  st = hip_status(q->zk->run(zs, -1, B, s));
  if (st != GFC_OK) return st;
  zs.T = SZ;
  st = hip_status(q->zk->run(zs, -1, B, s));
  if (st != GFC_OK) return st;
  // 3. the z difference of Ez as its symbol into the split bins; 4. the column pass
  st = hip_status(launch_sz_combine(T, SZ, q->omz, p->H, p->NHP, p->K, p->KP, P, plane,
                                    splane, B, s));
  if (st != GFC_OK) return st;
  ColFwdArgs c = col_fwd_args(p, T, SB, partial);
  c.cc = q->cc;
  c.zp = P;
  {
    std::lock_guard<std::mutex> fork_lock(p->fork_mtx);
    st = hip_status(launch_col_fwd(c, B * P, s, p->side, p->ev_fork, p->ev_join));
  }
  if (st != GFC_OK) return st;
  // 5. inverse z transform: P planes in, the D planes of the volume out
  z.din = P;
  z.dout = D;
  st = hip_status(q->zk->run(z, +1, B, s));
  if (st != GFC_OK) return st;
  // 6. the corner constant of each volume, then the inverse rows of every slice z < D, crop
  double* total = reinterpret_cast<double*>(ws + w.tot);
  st = hip_status(launch_partial_sums(partial, P * p->ntiles_f, total, B, s));
  if (st != GFC_OK) return st;
  RowInvArgs v = row_inv_args(p, T, u, total);
  v.zd = D;
  v.zp = P;
  v.nparts = 1;
  return hip_status(p->rk->inv(v, B * D, s));
}

void gfc_plan3_destroy(gfc_plan3_t q) {
  if (!q) return;
  if (q->dmem) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (q->p2->device >= 0 && cur != q->p2->device) (void)hipSetDevice(q->p2->device);
    (void)hipFree(q->dmem);
    if (cur >= 0 && cur != q->p2->device) (void)hipSetDevice(cur);
  }
  gfc_plan_destroy(q->p2);
  delete q;
}

}  // extern "C"
