// gfc_plan.h - the plan object behind gfc_plan_t and the argument blocks it hands to the
// kernel launchers (shared by the plain and the ragged entry points).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <mutex>

#include "gfc.h"
#include "gfc_internal.h"

namespace gfc {

// Launch geometry defaults; each can be changed per plan with gfc_plan_set_param.
constexpr int kColC = 16;         // "col_c": columns per workgroup in the column pass
constexpr int kColRows = 16;      // "col_rows", "col_rows_b": rows per thread in the forward
                                  // and the backward column pass (16|32)

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

inline gfc_status hip_status(hipError_t e) { return e == hipSuccess ? GFC_OK : GFC_E_HIP; }

}  // namespace gfc

struct gfc_plan_s {
  // sizes (block at the torus origin; r0, c0: the grid corner relative to it)
  int H = 0, W = 0, M = 0, N = 0, NH = 0, NHP = 0, KP = 0, KbP = 0, oy = 0, ox = 0, r0 = 0, c0 = 0, K = 0, Kb = 0;
  unsigned flags = 0;
  const gfc::RowKernels* rk = nullptr;
  gfc::ColGeom gf{}, gb{};
  // launch geometry (gfc_plan_set_param) and what follows from it
  int col_c = gfc::kColC, col_rows = gfc::kColRows, col_rows_b = gfc::kColRows;
  int nfslots = 0, npairs = 0;
  int ntiles_f = 0, ntiles_b = 0, nsums = 0;
  // device tables, one allocation (gfc_green_build)
  bool built = false;
  int device = -1;
  void* dmem = nullptr;
  // four-step twiddles of each row pass's split: twA plain forward, twAe the other forward
  // modes, twB inverse, twAb backward forward, twBb backward inverse; twL / twLe the low-bin
  // lane factors of the two forward splits
  gfc::f2 *twA = nullptr, *twAe = nullptr, *twB = nullptr, *twAb = nullptr, *twBb = nullptr,
          *twL = nullptr, *twLe = nullptr, *twX = nullptr, *dshift = nullptr;
  double* twD = nullptr;  // [N][2] float64 w_N^m (direct sums of a given Laplacian's low bins)
  gfc::ColConst *ccf = nullptr, *ccb = nullptr;
  // a side stream for the forward column pass's low tiles, joined back with two events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // serialises the fork/join enqueue of calls from several host threads on one plan (the
  // events are re-recorded by every call)
  std::mutex fork_mtx;
};

namespace gfc {

// workgroups of the inverse row pass (one moment pair each for the colour correction)
inline int inv_groups(const gfc_plan_s* p) {
  const int slots_needed = (p->H + 1) / 2;  // one row pair per slot
  return (slots_needed + p->rk->i.slots - 1) / p->rk->i.slots;
}

// workspace of a batch: spectra T, side arrays (SB forward / SD backward), reductions,
// moment sums of the colour correction, float64 low-bin row sums of a given Laplacian
struct WsLayout {
  size_t t, side, red, mom, lap, total;
};
inline WsLayout ws_layout(const gfc_plan_s* p, int B) {
  WsLayout w{};
  const size_t Bz = size_t(B);
  const size_t tbytes = Bz * size_t(p->H + 1) * p->NHP * sizeof(f2);
  const size_t sb = Bz * size_t(p->H) * p->KP * sizeof(f2);
  const size_t sd = Bz * size_t(p->H) * p->KbP * sizeof(f2);
  const size_t pf = Bz * size_t(p->ntiles_f) * sizeof(double);
  const size_t ps = Bz * size_t(p->nsums) * sizeof(double);
  const size_t pm = Bz * size_t(inv_groups(p)) * 2 * sizeof(double);
  w.t = 0;
  w.side = align256(tbytes);
  w.red = w.side + align256(std::max(sb, sd));
  const size_t pl = Bz * size_t(p->H + 1) * size_t(p->K + 1) * 2 * sizeof(double);
  w.mom = w.red + align256(std::max(pf, ps));
  w.lap = w.mom + align256(pm);
  w.total = w.lap + align256(pl);
  return w;
}

inline RowFwdArgs row_fwd_args(const gfc_plan_s* p, const float* gx, const float* gy, f2* T,
                               f2* SB) {
  RowFwdArgs a{};
  a.gx = gx;
  a.gy = gy;
  a.C = nullptr;
  a.edit = kEditNone;
  a.tau2 = 0.f;
  a.alpha = 0.f;
  a.T1 = T;
  a.SB = SB;
  a.twA = p->twA;
  a.twL = p->twL;
  a.twX = p->twX;
  a.H = p->H;
  a.W = p->W;
  a.K = p->K;
  a.KP = p->KP;
  a.N = p->N;
  a.NHP = p->NHP;
  a.npairs = (p->H + 2) / 2;
  a.img_in = (long long)p->H * p->W;
  a.img_t1 = (long long)(p->H + 1) * p->NHP;
  a.img_sb = (long long)p->H * p->KP;
  a.gz = nullptr;
  a.SZ = nullptr;
  a.zd = 0;
  a.zp = 1;
  return a;
}

inline ColFwdArgs col_fwd_args(const gfc_plan_s* p, f2* T, const f2* SB, double* partial) {
  ColFwdArgs c{};
  c.T = T;
  c.SB = SB;
  c.cc = p->ccf;
  c.partial = partial;
  c.H = p->H;
  c.M = p->M;
  c.NH = p->NH;
  c.NHP = p->NHP;
  c.K = p->K;
  c.KP = p->KP;
  c.r0 = p->r0;
  c.C = p->gf.C;
  c.nseg = p->gf.nseg;
  c.Lseg = p->gf.Lseg;
  c.Llast = p->gf.Llast;
  c.Rp = p->gf.Rp;
  c.nparts = p->ntiles_f;
  c.img_t = (long long)(p->H + 1) * p->NHP;
  c.img_sb = (long long)p->H * p->KP;
  c.zp = 1;
  return c;
}

inline RowInvArgs row_inv_args(const gfc_plan_s* p, const f2* T, float* u,
                               const double* partial) {
  RowInvArgs v{};
  v.T2 = T;
  v.u = u;
  v.partial = partial;
  v.nparts = p->ntiles_f;
  v.twB = p->twB;
  v.H = p->H;
  v.W = p->W;
  v.npairs = (p->H + 1) / 2;
  v.img_t2 = (long long)(p->H + 1) * p->NHP;
  v.img_u = (long long)p->H * p->W;
  v.mom = nullptr;
  v.zd = 1;
  v.zp = 1;
  v.N = p->N;
  return v;
}

}  // namespace gfc
