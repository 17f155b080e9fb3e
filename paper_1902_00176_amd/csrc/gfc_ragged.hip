// gfc_ragged.hip - ragged batches: many images of different sizes in one solve.
//
// Each image keeps its own plan (its torus, float64 column tables and row twiddles; images
// with the same sizes share one). The three passes run over all images at once:
//   row pass      the FFT code is specialised on the row length N; one launch covers the
//                 lengths of one group of about 12 (one workgroup size, half support
//                 2 W <= N), else one launch per length; each workgroup one (image, strip block)
//                 item; then one launch of the extra split row bins of thin images (K > 4);
//   column pass   one launch per stream, each workgroup one (image, column tile) item,
//                 the tiles holding columns l <= K first (they take the split-input path);
//   inverse row   as the row pass.
// Each group or length is one launch over all its images. The launches are dealt to four
// streams (largest estimated bytes first, each to the least loaded stream), and every
// stream runs the three passes for its own images: the
// streams never wait for each other, so one stream's column pass overlaps another's row
// launches. Work items are ordered largest image first so the small ones fill the tail of
// a launch.
// The whole sequence is captured once into a HIP graph and replayed by every later call: the
// kernels read the buffer bases from a device slot that each call fills first (a one-thread
// kernel on the caller's stream), so new addresses need no new graph. Per image the arithmetic is the plain path's, so a ragged solve
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
constexpr int kRgColRows = 32;      // rows per column-pass thread for every image

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
    const RowKernels* rk;  // one row length, or
    const RgMulti* mk;     // several lengths of one workgroup size (half support)
    int f_off, f_n, i_off, i_n;
    bool half;  // every image of the group has 2 W <= N
  };
  std::vector<Group> groups;  // one per multi-length launch, or per row length
  struct Lane {                // the work of one stream
    std::vector<int> groups;   // its row lengths
    int x_off = 0, x_n = 0;    // low-bin extension items (image, row) of images with K > 4
    int c_low_off = 0, c_low_n = 0, c_rest_off = 0, c_rest_n = 0;
    int c_threads = 64;
    size_t c_shm = 0;
    bool c_tail = false;
  };
  Lane lanes[4];

  // launch machinery
  hipStream_t side[kRgStreams - 1] = {};
  hipEvent_t ev[4 * kRgStreams] = {};
  hipStream_t cap = nullptr;
  RgBase* dbase = nullptr;  // device slot the kernels read the buffer bases from
  // the launch sequence, captured once: it reads the bases from dbase, so it serves every
  // call; `done` is recorded after each launch (destroy waits for it)
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
};

namespace {

__global__ void k_set_base(RgBase* slot, RgBase v) {
  if (threadIdx.x == 0) *slot = v;
}

void release(gfc_ragged_s* r) {
  // the graph may still run on a caller's stream: wait for its last launch first
  if (r->done) (void)hipEventSynchronize(r->done);
  if (r->exec) (void)hipGraphExecDestroy(r->exec);
  if (r->done) (void)hipEventDestroy(r->done);
  for (auto& e : r->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& s : r->side)
    if (s) (void)hipStreamDestroy(s);
  if (r->cap) (void)hipStreamDestroy(r->cap);
  if (r->dmem) (void)hipFree(r->dmem);
  for (gfc_plan_t p : r->plans) gfc_plan_destroy(p);
  r->plans.clear();
}

// Enqueue the three passes of every stream's images on `main` and the side streams, joined
// back to `main`.
gfc_status enqueue(gfc_ragged_s* r, const RgBase* base, hipStream_t main) {
  static_assert(kRgStreams == 4, "one Lane per stream");
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
  for (int k = 0; k < kRgStreams; ++k) {
    const auto& Ln = r->lanes[k];
    if (Ln.groups.empty()) continue;
    for (int g : Ln.groups) {
      const auto& G = r->groups[g];
      if (G.f_n == 0) continue;
      const hipError_t e =
          G.mk ? G.mk->fwd(base, r->tab_f, r->items + G.f_off, G.f_n, st[k])
               : G.rk->rg_fwd(base, r->tab_f, r->items + G.f_off, G.f_n, G.half, st[k]);
      if (e != hipSuccess) return GFC_E_HIP;
    }
    if (launch_low_ext_rg(base, r->tab_f, r->items + Ln.x_off, Ln.x_n, st[k]) != hipSuccess)
      return GFC_E_HIP;
    if (launch_col_fwd_rg(base, r->tab_c, r->items + Ln.c_low_off, Ln.c_low_n,
                          r->items + Ln.c_rest_off, Ln.c_rest_n, kRgColRows, Ln.c_tail,
                          Ln.c_threads, Ln.c_shm, st[k]) != hipSuccess)
      return GFC_E_HIP;
    for (int g : Ln.groups) {
      const auto& G = r->groups[g];
      if (G.i_n == 0) continue;
      const hipError_t e = G.mk ? G.mk->inv(base, r->tab_i, r->items + G.i_off, G.i_n, st[k])
                                : G.rk->rg_inv(base, r->tab_i, r->items + G.i_off, G.i_n,
                                               G.half, st[k]);
      if (e != hipSuccess) return GFC_E_HIP;
    }
  }
  if (!join(kRgStreams)) return GFC_E_HIP;
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
  // launch key of an image: its multi-length group (half support) or its row length
  auto key_of = [&](int i) -> long long {
    const RgMulti* m = 2 * r->W[i] <= r->N[i] ? find_rg_multi(r->N[i]) : nullptr;
    return m ? -1 - (long long)m->id : (long long)r->N[i];
  };
  auto bytes_of = [&](int i) {
    return 12.0 * r->H[i] * r->W[i] + 32.0 * (r->H[i] + 1) * (r->N[i] / 2 + 1);
  };
  // launches: the images of one key, largest first, in one launch (cutting them into
  // chunks of at most an eighth of the batch's bytes, to balance the streams, took 4 % more
  // time on the 200-image batch: more, smaller launches)
  std::vector<long long> keys;
  for (int i : order)
    if (std::find(keys.begin(), keys.end(), key_of(i)) == keys.end()) keys.push_back(key_of(i));
  std::vector<std::vector<int>> chunks;
  std::vector<double> gbytes;
  for (long long key : keys) {
    std::vector<int> cur;
    double cb = 0.0;
    for (int i : order) {
      if (key_of(i) != key) continue;
      cur.push_back(i);
      cb += bytes_of(i);
    }
    chunks.push_back(cur);
    gbytes.push_back(cb);
  }
  for (const auto& ch : chunks) {
    gfc_ragged_s::Group g{};
    const int first = ch.front();
    g.rk = r->plans[r->plan_of[first]]->rk;
    g.mk = key_of(first) < 0 ? find_rg_multi(r->N[first]) : nullptr;
    g.f_off = int(items.size());
    g.half = true;
    for (int i : ch) {
      g.half = g.half && 2 * r->W[i] <= r->N[i];
      const gfc_plan_s* p = r->plans[r->plan_of[i]];
      const int slots = p->rk->f.slots;
      const int nb = (p->nfslots + slots - 1) / slots;
      for (int k = 0; k < nb; ++k) items.push_back(RgItem{i, k});
    }
    g.f_n = int(items.size()) - g.f_off;
    g.i_off = int(items.size());
    for (int i : ch) {
      const gfc_plan_s* p = r->plans[r->plan_of[i]];
      const int slots = p->rk->i.slots;
      const int nb = (p->npairs + slots - 1) / slots;
      for (int k = 0; k < nb; ++k) items.push_back(RgItem{i, k});
    }
    g.i_n = int(items.size()) - g.i_off;
    r->groups.push_back(g);
  }
  // launches to streams: largest first, each to the least loaded stream
  std::vector<int> gorder(chunks.size());
  for (size_t g = 0; g < gorder.size(); ++g) gorder[g] = int(g);
  std::stable_sort(gorder.begin(), gorder.end(), [&](int a, int b) { return gbytes[a] > gbytes[b]; });
  double load[kRgStreams] = {};
  std::vector<int> lane_img(B, 0);
  for (auto& Ln : r->lanes) Ln = gfc_ragged_s::Lane{};
  for (int g : gorder) {
    const int k = int(std::min_element(load, load + kRgStreams) - load);
    load[k] += gbytes[g];
    r->lanes[k].groups.push_back(g);
    for (int i : chunks[g]) lane_img[i] = k;
  }
  auto lane_of = [&](int i) { return lane_img[i]; };
  // per stream: extension items, column items (low tiles, then the rest), workgroup shape
  for (int k = 0; k < kRgStreams; ++k) {
    auto& Ln = r->lanes[k];
    Ln.x_off = int(items.size());
    for (int i : order) {
      const gfc_plan_s* p = r->plans[r->plan_of[i]];
      if (lane_of(i) == k && p->K > kLowBins)
        for (int y = 0; y <= p->H; ++y) items.push_back(RgItem{i, y});
    }
    Ln.x_n = int(items.size()) - Ln.x_off;
    Ln.c_low_off = int(items.size());
    for (int i : order) {
      if (lane_of(i) != k) continue;
      const gfc_plan_s* p = r->plans[r->plan_of[i]];
      const int nlow = std::min(p->ntiles_f, (p->K + 1 + p->gf.C - 1) / p->gf.C);
      for (int t = 0; t < nlow; ++t) items.push_back(RgItem{i, t});
    }
    Ln.c_low_n = int(items.size()) - Ln.c_low_off;
    Ln.c_rest_off = int(items.size());
    for (int i : order) {
      if (lane_of(i) != k) continue;
      const gfc_plan_s* p = r->plans[r->plan_of[i]];
      const int nlow = std::min(p->ntiles_f, (p->K + 1 + p->gf.C - 1) / p->gf.C);
      for (int t = nlow; t < p->ntiles_f; ++t) items.push_back(RgItem{i, t});
    }
    Ln.c_rest_n = int(items.size()) - Ln.c_rest_off;
    Ln.c_threads = 64;
    Ln.c_shm = 0;
    Ln.c_tail = false;
    for (int i = 0; i < B; ++i) {
      if (lane_of(i) != k) continue;
      const gfc_plan_s* p = r->plans[r->plan_of[i]];
      if (p->gf.Lseg != kRgColRows) return GFC_E_SIZE;
      Ln.c_threads = std::max(Ln.c_threads, (p->gf.C * p->gf.nseg + 63) / 64 * 64);
      Ln.c_shm = std::max(Ln.c_shm, size_t(2 * p->gf.nseg * p->gf.C) * 2 * sizeof(double));
      Ln.c_tail = Ln.c_tail || p->gf.tail;
    }
  }

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
  const size_t o_base = o;
  o = align256(o + sizeof(RgBase));
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
  r->dbase = reinterpret_cast<RgBase*>(base + o_base);

  for (auto& st : r->side)
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return GFC_E_HIP;
  if (hipStreamCreateWithFlags(&r->cap, hipStreamNonBlocking) != hipSuccess) return GFC_E_HIP;
  for (auto& e : r->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return GFC_E_HIP;
  if (hipEventCreateWithFlags(&r->done, hipEventDisableTiming) != hipSuccess) return GFC_E_HIP;
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
  // the bases of this call into the device slot, ahead of the passes on the same stream
  hipLaunchKernelGGL(k_set_base, dim3(1), dim3(64), 0, s, r->dbase, base);
  if (hipGetLastError() != hipSuccess) return GFC_E_HIP;
  if (r->flags & GFC_RAGGED_NO_GRAPH) return enqueue(r, r->dbase, s);
  if (!r->exec) {
    // first call: capture the launch sequence (it reads the bases from the slot)
    if (hipStreamBeginCapture(r->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return GFC_E_HIP;
    st = enqueue(r, r->dbase, r->cap);
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
  }
  if (hipGraphLaunch(r->exec, s) != hipSuccess) return GFC_E_HIP;
  return hip_status(hipEventRecord(r->done, s));
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
