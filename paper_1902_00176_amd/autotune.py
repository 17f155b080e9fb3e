"""Autotuner for the GFC launch geometry.

For each image size and torus it times every pass of the forward and backward solve on
the GPU (HIP events on the launch stream, median of several repetitions) over a grid of
launch parameters, picks the fastest setting per parameter group and records it in
tuning.json, which Plan() reads. Parameters only change speed, never results:

  col_c      columns per workgroup in the column pass
  col_rows   most rows per thread in the forward column pass (16 | 32)
  col_rows_b most rows per thread in the backward column pass (16 | 32)

    python -m paper_1902_00176_amd.autotune --size 801 1200 1620 2400 100 [--write]
    python -m paper_1902_00176_amd.autotune --workloads [--write]

Row-transform splits (--splits): each row length N = N1 * N2 can be transformed with several
splits (both factors <= 64, the fewest lanes per slot, either order), and which is fastest
differs between the passes (holding N1 values per lane in one stage and N2 in the other
moves register pressure between the forward and the inverse transform). The candidate
library, built with `python paper_1902_00176_amd/build_lib.py --tune`, holds every candidate
of every length as its own entry; this mode times the four row passes of each candidate
(selected with the plan parameter "row_split") and records the fastest split per pass and
length under "row_splits" in tuning.json. The default build compiles those splits.

    python paper_1902_00176_amd/build_lib.py --tune
    GFC_LIBRARY=paper_1902_00176_amd/_build_tune/libgfc_tune.so \
        python -m paper_1902_00176_amd.autotune --splits [--lengths 2400 2048] [--write]
"""
from __future__ import annotations

import argparse
import ctypes
import itertools
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import paper_1902_00176_amd as gfc  # noqa: E402

DEFAULT = {"col_c": 16, "col_rows": 16, "col_rows_b": 16}
GRID = {
    "col": [(c, r) for c in (4, 8, 16, 32) for r in (16, 32)],
}
# the standard workloads: (H, W, M, N, B)
WORKLOADS = [(801, 1200, 1620, 2400, 100), (512, 512, 1024, 1024, 96),
             (256, 256, 512, 512, 48), (64, 64, 128, 128, 1)]


def time_stages(plan, B, reps=7, torch=None):
    """Median ms of each forward and backward stage for a batch of B images."""
    dev = torch.device("cuda:0")
    H, W = plan.H, plan.W
    g = torch.randn((B, H, W), device=dev) * 0.1
    g2 = torch.randn((B, H, W), device=dev) * 0.1  # gy: its own buffer, as in a real solve
    u = torch.empty_like(g)
    d2 = torch.empty_like(g)
    ws = torch.empty(plan.workspace_size(B), dtype=torch.uint8, device=dev)
    L = gfc.lib()
    st = torch.cuda.current_stream(dev)
    sp = ctypes.c_void_p(st.cuda_stream)
    h = plan.handle

    def f(k):
        r = L.gfc_solve_batch_stage(h, k, g.data_ptr(), g2.data_ptr(), u.data_ptr(), B,
                                    ws.data_ptr(), ws.numel(), sp)
        if r:
            raise gfc.GFCError(r, "gfc_solve_batch_stage")

    def bw(k):
        r = L.gfc_solve_backward_stage(h, k, g.data_ptr(), u.data_ptr(), d2.data_ptr(), B,
                                       ws.data_ptr(), ws.numel(), sp)
        if r:
            raise gfc.GFCError(r, "gfc_solve_backward_stage")

    times = {n: [] for n in ("fwd1", "fwd2", "fwd3", "bwd1", "bwd2", "bwd3")}
    for rep in range(reps + 2):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
        ev[0].record(st)
        for k in (1, 2, 3):
            f(k)
            ev[k].record(st)
        for k in (1, 2, 3):
            bw(k)
            ev[3 + k].record(st)
        torch.cuda.synchronize()
        if rep >= 2:
            names = list(times)
            for i, n in enumerate(names):
                times[n].append(ev[i].elapsed_time(ev[i + 1]))
    return {n: statistics.median(v) for n, v in times.items()}


def tune_size(H, W, M, N, B, torch, verbose=True):
    def run(params):
        p = gfc.Plan(H, W, M, N, params=params, tuned=False).build()
        t = time_stages(p, B, torch=torch)
        del p
        return t

    best = dict(DEFAULT)
    log = []
    # column pass
    res = []
    # columns per workgroup (shared) and rows per thread (forward and backward separately)
    for c, r in GRID["col"]:
        t = run({**DEFAULT, "col_c": c, "col_rows": r, "col_rows_b": r})
        res.append((c, r, t))
        log.append({"col_c": c, "col_rows": r, **t})
    best_fb = None
    for c in sorted({c for c, _, _ in res}):
        f = min((t["fwd2"], r) for cc, r, t in res if cc == c)
        b = min((t["bwd2"], r) for cc, r, t in res if cc == c)
        if best_fb is None or f[0] + b[0] < best_fb[0]:
            best_fb = (f[0] + b[0], c, f[1], b[1])
    _, best["col_c"], best["col_rows"], best["col_rows_b"] = best_fb
    final = run(best)
    if verbose:
        for e in log:
            print(json.dumps({k: (round(v, 4) if isinstance(v, float) else v) for k, v in e.items()}),
                  flush=True)
        print(json.dumps({"size": [H, W, M, N, B], "best": best,
                          "ms": {k: round(v, 4) for k, v in final.items()}}), flush=True)
    return best, final


# row passes among the timed stages
ROW_PASSES = {"fwd": "fwd1", "inv": "fwd3", "bfwd": "bwd1", "binv": "bwd3"}


def split_shape(N):
    """A batch whose row passes take long enough to time: the 801 x 1200 workload for its
    2400-point rows, else 256-row images of width N / 2 (their default torus is N wide) and
    enough of them for about 2e7 spectrum bins."""
    if N == 2400:
        return 801, 1200, 1620, 2400, 100
    H, W = 256, N // 2
    B = max(1, min(256, int(2e7 // (H * (N // 2 + 1)))))
    return H, W, 0, N, B


def tune_splits(lengths, torch, verbose=True):
    """{N: {pass: [N1, N2], "ms": {pass: {"N1xN2": ms}}}} for the given row lengths."""
    sys.path.insert(0, HERE)
    import build_lib
    out = {}
    for N in lengths:
        H, W, M, NN, B = split_shape(N)
        ms = {ps: {} for ps in ROW_PASSES}
        for n1, n2 in build_lib.candidate_splits(N):
            p = gfc.Plan(H, W, M, NN, params={"row_split": n1}, tuned=False).build()
            t = time_stages(p, B, torch=torch)
            del p
            for ps, st in ROW_PASSES.items():
                ms[ps][f"{n1}x{n2}"] = round(t[st], 5)
        best = {ps: [int(x) for x in min(v, key=v.get).split("x")] for ps, v in ms.items()}
        out[str(N)] = {**best, "ms": ms, "shape": [H, W, M, NN, B]}
        if verbose:
            print(json.dumps({"N": N, **best,
                              "ms": {ps: min(v.values()) for ps, v in ms.items()}}), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--splits", action="store_true",
                    help="time the candidate row splits (GFC_LIBRARY = the candidate library)")
    ap.add_argument("--lengths", type=int, nargs="*", help="row lengths for --splits (default: all)")
    ap.add_argument("--size", type=int, nargs=5, action="append", metavar=("H", "W", "M", "N", "B"))
    ap.add_argument("--workloads", action="store_true")
    ap.add_argument("--write", action="store_true", help="update tuning.json beside this file")
    ap.add_argument("--out", help="also write the resulting database to this path")
    args = ap.parse_args()
    import torch
    sizes = [tuple(s) for s in (args.size or [])]
    if args.workloads:
        sizes += WORKLOADS
    db_path = os.path.join(HERE, "tuning.json")
    try:
        with open(db_path) as f:
            db = json.load(f)
    except (OSError, ValueError):
        db = {"plans": {}}
    for H, W, M, N, B in sizes:
        best, final = tune_size(H, W, M, N, B, torch)
        db["plans"][gfc.tuning_key(H, W, M, N)] = {**best, "tuned_batch": B,
                                                   "ms": {k: round(v, 4) for k, v in final.items()}}
    if args.splits:
        if not os.environ.get("GFC_LIBRARY"):
            raise SystemExit("--splits times the candidate library: set GFC_LIBRARY to "
                             "paper_1902_00176_amd/_build_tune/libgfc_tune.so")
        lengths = args.lengths or [n for n in range(2, 4097, 2) if gfc.supported_length(n)]
        rs = db.setdefault("row_splits", {})
        for n, ent in tune_splits(lengths, torch).items():
            for keep in ("edit", "edit_ms"):  # hand-measured split of the edit modes
                if keep in rs.get(n, {}):
                    ent[keep] = rs[n][keep]
            rs[n] = ent
    for path in ([db_path] if args.write else []) + ([args.out] if args.out else []):
        with open(path, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
