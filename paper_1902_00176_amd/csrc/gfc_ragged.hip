// gfc_ragged.hip - ragged batches: many images of different sizes in one solve.
//
// Each image keeps its own plan (its torus, float64 column tables and row twiddles; images
// with the same sizes share one). The three passes run over all images at once:
//   row pass      one launch per distinct row length N (the FFT code is specialised on N),
//                 spread over four streams, each workgroup one (image, strip block) item;
//                 then one launch of the extra split row bins of thin images (K > 4);
//   column pass   one launch for the tiles holding columns l <= K and one for the rest,
//                 covering every image, each workgroup one (image, column tile) item;
//   inverse row   as the row pass.
// Work items are ordered largest image first so the small ones fill the tail of a launch.
// The whole sequence is captured once into a HIP graph and replayed by every later call
// with the same buffers. Per image the arithmetic is the plain path's, so a ragged solve
// equals solving each image with its plan (gfc_ragged_solve_sequential).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "gfc.h"
#include "gfc_internal.h"
#include "gfc_plan.h"

using namespace gfc;

namespace {
constexpr int kRgStreams = 4;       // streams the per-length row launches are spread over
constexpr int kRgColThreads = 512;  // target workgroup size of the ragged column pass
constexpr int kRgColRows = 16;      // rows per column-pass thread for every image

int pow2_floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}
}  // namespace

struct gfc_ragged_s {
  int B = 0;
  unsigned flags = 0;
  std::vector<int> H, W, M, N;
  std::vector<long long> off;      // B + 1 element offsets of the packed [H_i][W_i] arrays
  std::vector<gfc_plan_t> plans;   // distinct plans
  std::vector<int> plan_of;        // image -> plan
  std::vector<size_t> ws_off;      // image -> byte offset of its workspace region
  std::vector<size_t> ws_len;      // image -> bytes of that region (its plan at B = 1)
  size_t ws_total = 0;
  bool built = false;
  int device = -1;

  // device tables (one allocation)
  void* dmem = nullptr;
  RgRowFwd* tab_f = nullptr;
  RgCol* tab_c = nullptr;
  RgRowInv* tab_i = nullptr;
  RgItem* items = nullptr;
  struct Group {
    const RowKernels* rk;
    int f_off, f_n, i_off, i_n;
    bool half;  // every image of the group has 2 W <= N
  };
  std::vector<Group> groups;  // one per distinct N
  int x_off = 0, x_n = 0;  // low-bin extension items (image, row) of images with K > kLowBins
  int c_low_off = 0, c_low_n = 0, c_rest_off = 0, c_rest_n = 0;
  int c_threads = 64;
  size_t c_shm = 0;
  bool c_tail = false;

  // launch machinery
  hipStream_t side[kRgStreams - 1] = {};
  hipEvent_t ev[4 * kRgStreams] = {};
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  RgBase cached{};
};

namespace {

void release(gfc_ragged_s* r) {
  if (r->exec) (void)hipGraphExecDestroy(r->exec);
  for (auto& e : r->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& s : r->side)
    if (s) (void)hipStreamDestroy(s);
  if (r->cap) (void)hipStreamDestroy(r->cap);
  if (r->dmem) (void)hipFree(r->dmem);
  for (gfc_plan_t p : r->plans) gfc_plan_destroy(p);
  r->plans.clear();
}

// Enqueue the three passes on `main` (and the side streams, joined back to `main`).
gfc_status enqueue(gfc_ragged_s* r, const RgBase& base, hipStream_t main) {
  hipStream_t st[kRgStreams] = {main, r->side[0], r->side[1], r->side[2]};
  auto fork = [&](int k) -> bool {  // side streams wait for main
    if (hipEventRecord(r->ev[k], main) != hipSuccess) return false;
    for (int i = 1; i < kRgStreams; ++i)
      if (hipStreamWaitEvent(st[i], r->ev[k], 0) != hipSuccess) return false;
    return true;
  };
  auto join = [&](int k) -> bool {  // main waits for the side streams
    for (int i = 1; i < kRgStreams; ++i) {
      if (hipEventRecord(r->ev[k + i], st[i]) != hipSuccess) return false;
      if (hipStreamWaitEvent(main, r->ev[k + i], 0) != hipSuccess) return false;
    }
    return true;
  };
  if (!fork(0)) return GFC_E_HIP;
  for (size_t g = 0; g < r->groups.size(); ++g) {
    const auto& G = r->groups[g];
    if (G.f_n > 0 &&
        G.rk->rg_fwd(base, r->tab_f, r->items + G.f_off, G.f_n, G.half, st[g % kRgStreams]) != hipSuccess)
      return GFC_E_HIP;
  }
  if (!join(kRgStreams)) return GFC_E_HIP;
  if (launch_low_ext_rg(base, r->tab_f, r->items + r->x_off, r->x_n, main) != hipSuccess)
    return GFC_E_HIP;
  if (launch_col_fwd_rg(base, r->tab_c, r->items + r->c_low_off, r->c_low_n,
                        r->items + r->c_rest_off, r->c_rest_n, kRgColRows, r->c_tail,
                        r->c_threads, r->c_shm, main) != hipSuccess)
    return GFC_E_HIP;
  if (!fork(2 * kRgStreams)) return GFC_E_HIP;
  for (size_t g = 0; g < r->groups.size(); ++g) {
    const auto& G = r->groups[g];
    if (G.i_n > 0 &&
        G.rk->rg_inv(base, r->tab_i, r->items + G.i_off, G.i_n, st[g % kRgStreams]) != hipSuccess)
      return GFC_E_HIP;
  }
  if (!join(3 * kRgStreams)) return GFC_E_HIP;
  return GFC_OK;
}

gfc_status check_solve(gfc_ragged_s* r, const float* gx, const float* gy, float* u, void* ws,
                       size_t ws_bytes) {
  if (!r) return GFC_E_ARG;
  if (!r->built) return GFC_E_NOT_BUILT;
  if (r->B == 0) return GFC_OK;
  if (!gx || !gy || !u || !ws) return GFC_E_ARG;
  if (ws_bytes < r->ws_total) return GFC_E_WORKSPACE;
  return GFC_OK;
}

}  // namespace

extern "C" {

gfc_status gfc_ragged_create(gfc_ragged_t* out, int B, const int* H, const int* W,
                             const int* M, const int* N, unsigned flags) {
  if (!out) return GFC_E_ARG;
  *out = nullptr;
  if (B < 0 || (B > 0 && (!H || !W)) || (flags & ~GFC_RAGGED_NO_GRAPH)) return GFC_E_ARG;
  auto* r = new (std::nothrow) gfc_ragged_s;
  if (!r) return GFC_E_OOM;
  r->B = B;
  r->flags = flags;
  r->off.assign(size_t(B) + 1, 0);
  std::map<std::tuple<int, int, int, int, int>, int> cache;
  for (int i = 0; i < B; ++i) {
    gfc_plan_t p = nullptr;
    gfc_status st = gfc_plan_create(&p, H[i], W[i], M ? M[i] : 0, N ? N[i] : 0, GFC_FLAG_NONE);
    if (st != GFC_OK) {
      release(r);
      delete r;
      return st;
    }
    // every image uses segments of kRgColRows rows; C fills a workgroup of about
    // kRgColThreads threads
    const int nseg = (p->H + 1 + kRgColRows - 1) / kRgColRows;
    const int C = std::max(1, std::min(64, pow2_floor(std::max(1, kRgColThreads / nseg))));
    const auto key = std::make_tuple(p->H, p->W, p->M, p->N, C);
    auto it = cache.find(key);
    if (it != cache.end()) {
      gfc_plan_destroy(p);
      r->plan_of.push_back(it->second);
    } else {
      if (gfc_plan_set_param(p, "col_rows", kRgColRows) != GFC_OK ||
          gfc_plan_set_param(p, "col_c", C) != GFC_OK) {
        gfc_plan_destroy(p);
        release(r);
        delete r;
        return GFC_E_ARG;
      }
      cache[key] = int(r->plans.size());
      r->plan_of.push_back(int(r->plans.size()));
      r->plans.push_back(p);
    }
    const gfc_plan_s* q = r->plans[r->plan_of.back()];
    r->H.push_back(q->H);
    r->W.push_back(q->W);
    r->M.push_back(q->M);
    r->N.push_back(q->N);
    r->off[i + 1] = r->off[i] + (long long)q->H * q->W;
  }
  *out = r;
  return GFC_OK;
}

gfc_status gfc_ragged_build(gfc_ragged_t r, void* stream) {
  if (!r) return GFC_E_ARG;
  if (r->built) return GFC_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (gfc_plan_t p : r->plans) {
    const gfc_status st = gfc_green_build(p, stream);
    if (st != GFC_OK) return st;
  }
  const int B = r->B;
  // workspace regions: each image's plan layout at B = 1
  r->ws_off.assign(B, 0);
  r->ws_len.assign(B, 0);
  size_t tot = 0;
  for (int i = 0; i < B; ++i) {
    const WsLayout w = ws_layout(r->plans[r->plan_of[i]], 1);
    r->ws_off[i] = tot;
    r->ws_len[i] = w.total;
    tot += align256(w.total);
  }
  r->ws_total = tot;

  // argument tables
  std::vector<RgRowFwd> tf(B);
  std::vector<RgCol> tc(B);
  std::vector<RgRowInv> ti(B);
  for (int i = 0; i < B; ++i) {
    const gfc_plan_s* p = r->plans[r->plan_of[i]];
    const WsLayout w = ws_layout(p, 1);
    const long long t = (long long)(r->ws_off[i] + w.t);
    const long long side = (long long)(r->ws_off[i] + w.side);
    const long long red = (long long)(r->ws_off[i] + w.red);
    tf[i] = RgRowFwd{row_fwd_args(p, nullptr, nullptr, nullptr, nullptr), r->off[i], t, side};
    tc[i] = RgCol{col_fwd_args(p, nullptr, nullptr, nullptr), t, side, red};
    ti[i] = RgRowInv{row_inv_args(p, nullptr, nullptr, nullptr), r->off[i], t, red};
  }

  // work items: images by row length, largest first within each list
  std::vector<int> order(B);
  for (int i = 0; i < B; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const long long sa = (long long)r->H[a] * r->N[a], sb = (long long)r->H[b] * r->N[b];
    return sa > sb;
  });
  std::vector<RgItem> items;
  r->groups.clear();
  std::vector<int> lengths;
  for (int i : order)
    if (std::find(lengths.begin(), lengths.end(), r->N[i]) == lengths.end())
      lengths.push_back(r->N[i]);
  for (int n : lengths) {
    gfc_ragged_s::Group g{};
    const int first = *std::find_if(order.begin(), order.end(), [&](int i) { return r->N[i] == n; });
    g.rk = r->plans[r->plan_of[first]]->rk;
    const int slots = g.rk->slots;
    g.f_off = int(items.size());
    g.half = true;
    for (int i : order) {
      if (r->N[i] != n) continue;
      g.half = g.half && 2 * r->W[i] <= n;
      const gfc_plan_s* p = r->plans[r->plan_of[i]];
      const int nb = (p->nfslots + slots - 1) / slots;
      for (int k = 0; k < nb; ++k) items.push_back(RgItem{i, k});
    }
    g.f_n = int(items.size()) - g.f_off;
    g.i_off = int(items.size());
    for (int i : order) {
      if (r->N[i] != n) continue;
      const gfc_plan_s* p = r->plans[r->plan_of[i]];
      const int need = (p->npairs + p->row_ppw - 1) / p->row_ppw;
      const int nb = (need + slots - 1) / slots;
      for (int k = 0; k < nb; ++k) items.push_back(RgItem{i, k});
    }
    g.i_n = int(items.size()) - g.i_off;
    r->groups.push_back(g);
  }
  r->x_off = int(items.size());
  for (int i : order) {
    const gfc_plan_s* p = r->plans[r->plan_of[i]];
    if (p->K > kLowBins)
      for (int y = 0; y <= p->H; ++y) items.push_back(RgItem{i, y});
  }
  r->x_n = int(items.size()) - r->x_off;
  int threads = 64;
  size_t shm = 0;
  bool tail = false;
  r->c_low_off = int(items.size());
  for (int i : order) {
    const gfc_plan_s* p = r->plans[r->plan_of[i]];
    const int nlow = std::min(p->ntiles_f, (p->K + 1 + p->gf.C - 1) / p->gf.C);
    for (int k = 0; k < nlow; ++k) items.push_back(RgItem{i, k});
  }
  r->c_low_n = int(items.size()) - r->c_low_off;
  r->c_rest_off = int(items.size());
  for (int i : order) {
    const gfc_plan_s* p = r->plans[r->plan_of[i]];
    const int nlow = std::min(p->ntiles_f, (p->K + 1 + p->gf.C - 1) / p->gf.C);
    for (int k = nlow; k < p->ntiles_f; ++k) items.push_back(RgItem{i, k});
  }
  r->c_rest_n = int(items.size()) - r->c_rest_off;
  for (const gfc_plan_s* p : r->plans) {
    if (p->gf.Lseg != kRgColRows) return GFC_E_SIZE;
    threads = std::max(threads, (p->gf.C * p->gf.nseg + 63) / 64 * 64);
    shm = std::max(shm, size_t(2 * p->gf.nseg * p->gf.C) * 2 * sizeof(double));
    tail = tail || p->gf.tail;
  }
  r->c_threads = threads;
  r->c_shm = shm;
  r->c_tail = tail;

  // one device allocation for the tables and the item list
  size_t o = 0;
  const size_t o_f = o;
  o = align256(o + tf.size() * sizeof(RgRowFwd));
  const size_t o_c = o;
  o = align256(o + tc.size() * sizeof(RgCol));
  const size_t o_i = o;
  o = align256(o + ti.size() * sizeof(RgRowInv));
  const size_t o_it = o;
  o = align256(o + items.size() * sizeof(RgItem));
  std::vector<unsigned char> host(std::max<size_t>(o, 256), 0);
  if (!tf.empty()) std::memcpy(host.data() + o_f, tf.data(), tf.size() * sizeof(RgRowFwd));
  if (!tc.empty()) std::memcpy(host.data() + o_c, tc.data(), tc.size() * sizeof(RgCol));
  if (!ti.empty()) std::memcpy(host.data() + o_i, ti.data(), ti.size() * sizeof(RgRowInv));
  if (!items.empty())
    std::memcpy(host.data() + o_it, items.data(), items.size() * sizeof(RgItem));
  void* d = nullptr;
  if (hipMalloc(&d, host.size()) != hipSuccess) return GFC_E_OOM;
  if (hipMemcpyAsync(d, host.data(), host.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    (void)hipFree(d);
    return GFC_E_HIP;
  }
  auto* base = static_cast<unsigned char*>(d);
  r->dmem = d;
  r->tab_f = reinterpret_cast<RgRowFwd*>(base + o_f);
  r->tab_c = reinterpret_cast<RgCol*>(base + o_c);
  r->tab_i = reinterpret_cast<RgRowInv*>(base + o_i);
  r->items = reinterpret_cast<RgItem*>(base + o_it);

  for (auto& st : r->side)
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return GFC_E_HIP;
  if (hipStreamCreateWithFlags(&r->cap, hipStreamNonBlocking) != hipSuccess) return GFC_E_HIP;
  for (auto& e : r->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return GFC_E_HIP;
  (void)hipGetDevice(&r->device);
  r->built = true;
  return GFC_OK;
}

gfc_status gfc_ragged_image(gfc_ragged_t r, int i, int* H, int* W, int* M, int* N) {
  if (!r || i < 0 || i >= r->B) return GFC_E_ARG;
  if (H) *H = r->H[i];
  if (W) *W = r->W[i];
  if (M) *M = r->M[i];
  if (N) *N = r->N[i];
  return GFC_OK;
}

gfc_status gfc_ragged_offsets(gfc_ragged_t r, int64_t* offsets) {
  if (!r || !offsets) return GFC_E_ARG;
  for (int i = 0; i <= r->B; ++i) offsets[i] = r->off[i];
  return GFC_OK;
}

gfc_status gfc_ragged_workspace_size(gfc_ragged_t r, size_t* bytes) {
  if (!r || !bytes) return GFC_E_ARG;
  if (!r->built) return GFC_E_NOT_BUILT;
  *bytes = r->ws_total;
  return GFC_OK;
}

gfc_status gfc_ragged_solve(gfc_ragged_t r, const float* gx, const float* gy, float* u,
                            void* workspace, size_t ws_bytes, void* stream) {
  gfc_status st = check_solve(r, gx, gy, u, workspace, ws_bytes);
  if (st != GFC_OK || r->B == 0) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const RgBase base{gx, gy, u, static_cast<unsigned char*>(workspace)};
  if (r->flags & GFC_RAGGED_NO_GRAPH) return enqueue(r, base, s);
  const bool same = r->exec && r->cached.gx == gx && r->cached.gy == gy && r->cached.u == u &&
                    r->cached.ws == base.ws;
  if (!same) {
    if (r->exec) {
      // the previous graph may still be running on the caller's stream
      if (hipStreamSynchronize(s) != hipSuccess) return GFC_E_HIP;
      (void)hipGraphExecDestroy(r->exec);
      r->exec = nullptr;
    }
    if (hipStreamBeginCapture(r->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return GFC_E_HIP;
    st = enqueue(r, base, r->cap);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(r->cap, &graph);
    if (st != GFC_OK || e != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return GFC_E_HIP;
    }
    const hipError_t ei = hipGraphInstantiate(&r->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      r->exec = nullptr;
      return GFC_E_HIP;
    }
    r->cached = base;
  }
  return hip_status(hipGraphLaunch(r->exec, s));
}

gfc_status gfc_ragged_solve_sequential(gfc_ragged_t r, const float* gx, const float* gy,
                                       float* u, void* workspace, size_t ws_bytes,
                                       void* stream) {
  gfc_status st = check_solve(r, gx, gy, u, workspace, ws_bytes);
  if (st != GFC_OK || r->B == 0) return st;
  auto* ws = static_cast<unsigned char*>(workspace);
  for (int i = 0; i < r->B; ++i) {
    st = gfc_solve_batch(r->plans[r->plan_of[i]], gx + r->off[i], gy + r->off[i], u + r->off[i],
                         1, ws + r->ws_off[i], r->ws_len[i], stream);
    if (st != GFC_OK) return st;
  }
  return GFC_OK;
}

void gfc_ragged_destroy(gfc_ragged_t r) {
  if (!r) return;
  release(r);
  delete r;
}

}  // extern "C"
