"""Benchmark of the GFC batched solve on one MI355X.

A step is one forward solve of the 100-image 801x1200 batch on its 1620x2400 torus
(row pass, column pass, inverse row pass), inputs already resident in HBM. Prints one JSON
line: solves/s, per-kernel times from HIP events recorded between the passes on the launch
stream, the roofline of the dominant kernel, forward+backward pairs/s, and the float64 CPU
oracle timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 20] [--warmup 30] [--no-cpu] [--no-bwd]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s
CLOCK_SETTLE_S = 0.5       # untimed work before the warmup steps (GPU clock ramp)
FP32_VALU_PEAK = 78.6e12   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz, packed FP32 off
METRIC = "solves/s at 801x1200 B=100 FP32; fwd+bwd & ragged vs plain; % peak HBM BW"
CSRC = "paper_1902_00176_amd/csrc"
# files that decide what the kernels do and how they are launched: every kernel source, the
# plan and launch code, the build recipe and the tuned launch parameters
EXTRA_SOURCES = ["paper_1902_00176_amd/build_lib.py", "paper_1902_00176_amd/tuning.json",
                 "include/gfc.h"]


# The paper's own timings of the same solve (Sec. 3.1.3 and Fig. 2), on other hardware and
# an unstated torus: context for the figures above, not a baseline they are divided by.
PAPER_CONTEXT = {
    "batch_100_ms": 1.0, "single_solve_ms": 0.9,
    "framework": "PyTorch, float32, 100 images of 801x1200",
    "hardware": "NVIDIA GTX 1080 Ti (the one GPU the paper names)",
    "torus": "not stated (the paper's padding recipe pads by 4 pixels; this benchmark's "
             "default torus is 1620x2400, about 4x the points)",
    "timing_method": "not stated",
}


def kernel_source_hash() -> str:
    """Hash of every file under csrc/ and of the build recipe, header and tuning database:
    byte counters recorded under another hash no longer describe these kernels."""
    h = hashlib.sha256()
    rels = sorted(os.path.join(CSRC, f) for f in os.listdir(os.path.join(ROOT, CSRC))
                  if f.endswith((".h", ".hip")))
    for rel in rels + EXTRA_SOURCES:
        path = os.path.join(ROOT, rel)
        if os.path.exists(path):
            h.update(rel.encode())
            with open(path, "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def stage_model(H, W, N, K, Kb, kind):
    """Algorithmic HBM bytes and nominal FLOPs (5 n log2 n per complex FFT) per image."""
    import math
    NH = N // 2 + 1
    fft = 5.0 * N * math.log2(N)
    if kind == "fwd":
        # row pass: two divergence rows per complex FFT, plus direct sums of the K + 1
        # lowest bins of Ex and Ey (2K + 1 complex bins, W real samples, 4 flops each)
        return {
            "k_row_fwd": (8.0 * H * W + 8.0 * (H + 1) * NH + 8.0 * H * (K + 1),
                          math.ceil((H + 1) / 2) * fft + 4.0 * H * W * (2 * K + 1)),
            "k_col_fwd": (8.0 * (H + 1) * NH + 8.0 * H * (K + 1) + 8.0 * H * NH, 0.0),
            "k_row_inv": (8.0 * H * NH + 4.0 * H * W, math.ceil(H / 2) * fft),
        }
    return {
        "k_row_bfwd": (4.0 * H * W + 8.0 * H * NH, math.ceil(H / 2) * fft),
        "k_col_bwd": (8.0 * H * NH + 8.0 * (H + 1) * NH + 8.0 * H * (Kb + 1), 0.0),
        "k_row_binv": (8.0 * (H + 1) * NH + 8.0 * H * (Kb + 1) + 8.0 * H * W, H * fft),
    }


def load_traffic(kernel: str):
    """HBM bytes per image of one pass, from rocprofv3 PMC runs over a batch
    (profiles/traffic.json), or None when absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k or not t.get("batch"):
        return None
    return (k.get("fetch_bytes", 0) + k.get("write_bytes", 0)) / t["batch"]


def cpu_baseline(w, budget_s=15.0):
    """The float64 oracle on a bounded sample: images of the batch in order (cycling if the
    budget outlasts it), one solve at a time, until budget_s of wall time has passed."""
    import oracle as O
    n = 0
    t0 = time.perf_counter()
    while n < 2 or time.perf_counter() - t0 < budget_s:
        i = n % w.B
        O.solve_fft(w.gx[i], w.gy[i], w.M, w.N)
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "solves/s", "cores": O.cpu_workers(), "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{n} solves of the 801x1200 images (batch order, cycling) on the 1620x2400 "
                      f"torus, float64 scipy.fft oracle, one image at a time, {dt:.1f} s"}


def pmc_summarize(fetch_csv, write_csv, out_path, batch=100):
    """Turn two rocprofv3 --pmc runs of `bench.py --pmc-pass` (FETCH_SIZE, then WRITE_SIZE;
    KiB per dispatch) into HBM bytes per launch of each GFC kernel. Each counter is scaled by
    what it reads for the 256 MiB device copy in the same run."""
    import csv

    def read(path, counter):
        rows = []
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0))
        return rows

    copy_bytes = float(64 << 20) * 4
    out = {"source_hash": kernel_source_hash(), "batch": batch, "kernels": {}, "scale": {}}
    for key, path, counter in (("fetch_bytes", fetch_csv, "FETCH_SIZE"),
                               ("write_bytes", write_csv, "WRITE_SIZE")):
        rows = read(path, counter)
        cp = [v for k, v in rows if "copyBuffer" in k]
        if not cp:
            raise SystemExit(f"{path}: no device copy dispatch to scale {counter} by")
        scale = copy_bytes / cp[0]
        out["scale"][counter] = scale
        for k, v in rows:
            if "gfc::" not in k:
                continue
            name = k.split("gfc::", 1)[1].split("<", 1)[0].split("(", 1)[0]
            ent = out["kernels"].setdefault(name, {"fetch_bytes": 0.0, "write_bytes": 0.0})
            ent[key] += v * scale
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps(out), flush=True)


def ragged_bench(torch, gfc, synth, dev, stream, reps):
    """The uneven-size batch (200 images, H, W ~ U{64..1024}, default tori): ragged solves
    (graph replays) against the plain path, one single-image solve per image on the same
    stream. Both produce identical outputs. Throughput is timed as the headline step is:
    `reps` calls back to back between two events (median of 5 such runs); the latency of
    one call, from an event recorded before the host call to one after it with the stream
    idle before, is reported beside it."""
    import statistics
    sizes = synth.ragged_sizes()
    pairs = synth.make_ragged(sizes=sizes)
    r = gfc.Ragged(sizes).build(dev)
    gx = r.pack([p[0] for p in pairs], dev)
    gy = r.pack([p[1] for p in pairs], dev)
    u = torch.empty_like(gx)
    ws = torch.empty(r.workspace_size(), dtype=torch.uint8, device=dev)

    def timed(fn, n):
        for _ in range(3):
            fn(gx, gy, out=u, workspace=ws)
        torch.cuda.synchronize()
        runs = []
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(n):
                fn(gx, gy, out=u, workspace=ws)
            e1.record(stream)
            torch.cuda.synchronize()
            runs.append(e0.elapsed_time(e1) / n)
        return statistics.median(runs)

    def latency(fn):
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn(gx, gy, out=u, workspace=ws)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return statistics.median(ts)

    ms_r = timed(r.solve, reps)
    lat_r = latency(r.solve)
    ms_p = timed(r.solve_sequential, 2)
    pbytes = 0.0
    for H, W, M, N in r.sizes:
        NH = N // 2 + 1
        pbytes += 12.0 * H * W + 4 * 8.0 * (H + 1) * NH + 2 * 2 * 8.0 * (H + 1) * 17
    B = len(sizes)
    return {"workload": "ragged200_64to1024", "images": B,
            "distinct_row_lengths": len({s[3] for s in r.sizes}),
            "ragged_solves_per_s": B / (ms_r / 1e3), "ragged_ms": ms_r,
            "ragged_latency_ms": lat_r,
            "plain_solves_per_s": B / (ms_p / 1e3), "plain_ms": ms_p,
            "ragged_over_plain": ms_p / ms_r,
            "ragged_hbm_frac": pbytes / (ms_r / 1e3) / HBM_PEAK,
            "timing": "ragged_ms, plain_ms: calls back to back between two events; "
                      "ragged_latency_ms: one call on an idle stream"}


def volume_bench(torch, gfc, dev, stream, reps, D=128, B=4):
    """Three-dimensional solve of B volumes D^3 on the default (2D)^3 torus: volumes/s and
    the algorithmic HBM rate of the five passes."""
    import math
    plan = gfc.Plan3(D, D, D).build(dev)
    g = [torch.randn((B, D, D, D), device=dev) * 0.1 for _ in range(3)]
    u = torch.empty_like(g[0])
    ws = torch.empty(plan.workspace_size(B), dtype=torch.uint8, device=dev)
    for _ in range(3):
        plan.solve(*g, out=u, workspace=ws)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(reps):
        plan.solve(*g, out=u, workspace=ws)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    H = W = D
    P, N = plan.P, plan.N
    NH = N // 2 + 1
    R = H + 1
    vox = D * H * W
    bytes_vol = (12.0 * vox + 8.0 * (D + 1) * R * NH          # rows: gx, gy, gz -> T
                 + 8.0 * (D + 1) * R * NH + 8.0 * P * R * NH  # z forward
                 + 8.0 * P * R * NH + 8.0 * P * H * NH        # column recursion
                 + 8.0 * P * R * NH + 8.0 * D * R * NH        # z inverse
                 + 8.0 * D * H * NH + 4.0 * vox)              # inverse rows -> u
    return {"workload": f"volume{D}^3_b{B}", "torus": [plan.P, plan.M, plan.N],
            "volumes_per_s": B / (ms / 1e3), "ms": ms,
            "hbm_frac": bytes_vol * B / (ms / 1e3) / HBM_PEAK,
            "bytes_per_volume": bytes_vol}


def small_configs_bench(torch, gfc, dev, stream, reps):
    """The two smaller batch shapes: 96 solves of 512x512 on 1024x1024 (3 channels of 32
    merged pairs), forward; and 48 solves of 256x256 on 512x512 (16 x 3 channels, a
    differentiable layer), forward plus backward. Random float32 gradients of that shape
    (the timing does not depend on the values)."""
    out = {}
    for name, B, H, M, bwd in (("merge512_b96", 96, 512, 1024, False),
                               ("layer256_b48", 48, 256, 512, True)):
        plan = gfc.Plan(H, H, M, M).build(dev)
        gx = torch.randn((B, H, H), device=dev) * 0.1
        gy = torch.randn((B, H, H), device=dev) * 0.1
        u = torch.empty_like(gx)
        ws = torch.empty(plan.workspace_size(B), dtype=torch.uint8, device=dev)

        def step():
            plan.solve(gx, gy, out=u, workspace=ws)
            if bwd:
                plan.backward(u, workspace=ws)

        for _ in range(3):
            step()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(reps):
            step()
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        NH = M // 2 + 1
        per = 12.0 * H * H + 4 * 8.0 * (H + 1) * NH  # plain-path bytes per solve (one way)
        key = "pairs_per_s" if bwd else "solves_per_s"
        out[name] = {"torus": [M, M], "batch": B, key: B / (ms / 1e3), "ms_per_step": ms,
                     "hbm_frac": per * (2 if bwd else 1) * B / (ms / 1e3) / HBM_PEAK}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-bwd", action="store_true")
    ap.add_argument("--no-color", action="store_true")
    ap.add_argument("--no-edit", action="store_true")
    ap.add_argument("--no-laplacian", action="store_true")
    ap.add_argument("--no-volume", action="store_true")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--batch", type=int, default=100)
    ap.add_argument("--pmc-summarize", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two counter runs of --pmc-pass")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="for rocprofv3 counter runs: one 256 MiB device copy (the scale "
                         "reference for byte counters), one forward and one backward step")
    args = ap.parse_args()
    if args.pmc_summarize:
        pmc_summarize(*args.pmc_summarize, os.path.join(ROOT, "profiles", "traffic.json"))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X "
              "(a batch shards by image across GPUs with no exchange).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gfc_synth as synth
    import paper_1902_00176_amd as gfc

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = synth.make_workload("batch801x1200", B=args.batch)
    B, H, W_ = w.B, w.H, w.W
    plan = gfc.Plan(H, W_, w.M, w.N).build(dev)
    gx = torch.from_numpy(w.gx).to(dev)
    gy = torch.from_numpy(w.gy).to(dev)
    u = torch.empty_like(gx)
    ws = torch.empty(plan.workspace_size(B), dtype=torch.uint8, device=dev)
    L = gfc.lib()
    stream = torch.cuda.current_stream(dev)
    sp = __import__("ctypes").c_void_p(stream.cuda_stream)
    hp = plan.handle

    def stage_fwd(k):
        st = L.gfc_solve_batch_stage(hp, k, gx.data_ptr(), gy.data_ptr(), u.data_ptr(), B,
                                     ws.data_ptr(), ws.numel(), sp)
        if st != 0:
            raise gfc.GFCError(st, f"gfc_solve_batch_stage({k})")

    if args.pmc_pass:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        for k in (1, 2, 3):
            stage_fwd(k)
        du = torch.randn_like(gx) * 0.1
        dgx = torch.empty_like(gx)
        dgy = torch.empty_like(gx)
        for k in (1, 2, 3):
            st = L.gfc_solve_backward_stage(hp, k, du.data_ptr(), dgx.data_ptr(), dgy.data_ptr(),
                                            B, ws.data_ptr(), ws.numel(), sp)
            if st != 0:
                raise gfc.GFCError(st, f"gfc_solve_backward_stage({k})")
        torch.cuda.synchronize()
        print("pmc pass done", flush=True)
        return

    # The GPU raises its clocks over the first few hundred milliseconds of work: steps timed
    # after 5 warmup steps ran 3.5 % slower than after 30. So the same step first runs
    # untimed for CLOCK_SETTLE_S of wall time, then the W warmup steps, then the K timed ones.
    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < CLOCK_SETTLE_S:
        for _ in range(10):
            for k in (1, 2, 3):
                stage_fwd(k)
        torch.cuda.synchronize()
    settle_s = time.perf_counter() - t_settle
    for _ in range(args.warmup):
        for k in (1, 2, 3):
            stage_fwd(k)
    torch.cuda.synchronize()

    # The K timed steps run back to back with nothing between the passes; the stage times
    # come from K more steps with an event after each pass.
    names = ["k_row_fwd", "k_col_fwd", "k_row_inv"]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for i in range(args.steps):
        for k in (1, 2, 3):
            stage_fwd(k)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    t_start.record(stream)
    for i in range(args.steps):
        ev[i][0].record(stream)
        for k in (1, 2, 3):
            stage_fwd(k)
            ev[i][k].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_step_ev = t_start.elapsed_time(t_end) / args.steps
    stage_ms = {n: sum(ev[i][k].elapsed_time(ev[i][k + 1]) for i in range(args.steps)) / args.steps
                for k, n in enumerate(names)}

    K, Kb = plan.get_param("low_bins"), plan.get_param("low_bins_b")
    model = stage_model(H, W_, w.N, K, Kb, "fwd")
    dom = max(stage_ms, key=stage_ms.get)
    bytes_dom = model[dom][0] * B
    flops_dom = model[dom][1] * B
    t_dom = stage_ms[dom] / 1e3
    hbm_ach = bytes_dom / t_dom
    alu_ach = flops_dom / t_dom
    if flops_dom > 0 and alu_ach / FP32_VALU_PEAK > hbm_ach / HBM_PEAK:
        roof = {"bound": "alu", "achieved": alu_ach / 1e12, "peak": FP32_VALU_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": alu_ach / FP32_VALU_PEAK}
    else:
        roof = {"bound": "hbm", "achieved": hbm_ach / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": hbm_ach / HBM_PEAK}
    traffic = load_traffic(dom)
    roof["traffic"] = traffic * B if traffic is not None else None
    roof["kernel"] = dom
    roof["hbm_frac"] = hbm_ach / HBM_PEAK
    roof["alu_frac"] = alu_ach / FP32_VALU_PEAK

    total_bytes = sum(v[0] for v in model.values()) * B
    result = {
        "metric": METRIC, "value": B / (ms_step / 1e3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "H": H, "W": W_, "M": w.M, "N": w.N, "batch": B},
        "stages_ms": {k: round(v, 5) for k, v in stage_ms.items()},
        "ms_per_step_with_stage_events": ms_step_ev,
        "path_hbm_frac": total_bytes / (ms_step / 1e3) / HBM_PEAK,
        "clock_settle_s": round(settle_s, 3),
        "roofline": roof,
    }

    # the plain per-image path on the same images: one single-image solve per image, in
    # order on one stream, inputs resident
    plan1 = gfc.Plan(H, W_, w.M, w.N).build(dev)
    ws1 = torch.empty(plan1.workspace_size(1), dtype=torch.uint8, device=dev)
    hp1 = plan1.handle

    def per_image_pass():
        for i in range(B):
            st = L.gfc_solve_batch(hp1, gx[i].data_ptr(), gy[i].data_ptr(), u[i].data_ptr(), 1,
                                   ws1.data_ptr(), ws1.numel(), sp)
            if st != 0:
                raise gfc.GFCError(st, "gfc_solve_batch(B=1)")

    per_image_pass()
    torch.cuda.synchronize()
    reps1 = max(args.steps // 4, 3)
    p0 = torch.cuda.Event(enable_timing=True)
    p1 = torch.cuda.Event(enable_timing=True)
    p0.record(stream)
    for _ in range(reps1):
        per_image_pass()
    p1.record(stream)
    torch.cuda.synchronize()
    ms_plain = p0.elapsed_time(p1) / reps1
    result["plain_per_image"] = {"solves_per_s": B / (ms_plain / 1e3), "ms_per_100": ms_plain,
                                 "batched_over_plain": ms_plain / ms_step,
                                 "what": f"{B} gfc_solve_batch calls with B = 1 on one stream"}

    if not args.no_color:
        # forward solve + colour correction of eq. (25): one more read and write of u
        means = torch.full((B,), 0.5, device=dev)
        stds = torch.full((B,), 0.2, device=dev)

        def color_step():
            st = L.gfc_solve_batch_color(hp, gx.data_ptr(), gy.data_ptr(), means.data_ptr(),
                                         stds.data_ptr(), u.data_ptr(), B, ws.data_ptr(),
                                         ws.numel(), sp)
            if st != 0:
                raise gfc.GFCError(st, "gfc_solve_batch_color")

        for _ in range(args.warmup):
            color_step()
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        c0.record(stream)
        for _ in range(args.steps):
            color_step()
        c1.record(stream)
        torch.cuda.synchronize()
        ms_c = c0.elapsed_time(c1) / args.steps
        result["color"] = {"solves_per_s": B / (ms_c / 1e3), "ms_per_step": ms_c,
                           "over_plain": ms_c / ms_step,
                           "statistics": "source mean 0.5 and std 0.2 for every image"}

    if not args.no_edit:
        # gradient edits fused into the row pass (Sec. 3.2.3 thresholding, eq. (26) merging)
        C = torch.rand_like(gx)
        mag = torch.sqrt(gx[:4] * gx[:4] + gy[:4] * gy[:4])
        tau = float(torch.quantile(mag.flatten()[::97], 0.5))

        def edit_step(mode, param, cp):
            st = L.gfc_solve_edit(hp, gx.data_ptr(), gy.data_ptr(), cp, mode,
                                  __import__("ctypes").c_float(param), None, None, u.data_ptr(),
                                  B, ws.data_ptr(), ws.numel(), sp)
            if st != 0:
                raise gfc.GFCError(st, "gfc_solve_edit")

        edits = {}
        for name, mode, param, cp in (("threshold", gfc.EDIT_THRESHOLD, tau, None),
                                      ("gdm", gfc.EDIT_GDM, 0.5, C.data_ptr())):
            for _ in range(args.warmup):
                edit_step(mode, param, cp)
            c0 = torch.cuda.Event(enable_timing=True)
            c1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            c0.record(stream)
            for _ in range(args.steps):
                edit_step(mode, param, cp)
            c1.record(stream)
            torch.cuda.synchronize()
            ms_e = c0.elapsed_time(c1) / args.steps
            edits[name] = {"solves_per_s": B / (ms_e / 1e3), "ms_per_step": ms_e,
                           "over_plain": ms_e / ms_step}
        edits["params"] = f"threshold at the median gradient magnitude; gdm alpha 0.5, C ~ U[0,1]"
        result["edit"] = edits
        del C

    if not args.no_laplacian:
        # Algorithm B's own input: the solve from a given Laplacian on the support of div E
        # (rows of H + 1 by W + 1), its row bins l <= K summed in float64
        Lap = torch.randn((B, H + 1, W_ + 1), device=dev)
        Lap -= Lap.mean(dim=(1, 2), keepdim=True)

        def lap_step():
            st = L.gfc_solve_laplacian(hp, Lap.data_ptr(), u.data_ptr(), B, ws.data_ptr(),
                                       ws.numel(), sp)
            if st != 0:
                raise gfc.GFCError(st, "gfc_solve_laplacian")

        for _ in range(args.warmup):
            lap_step()
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        c0.record(stream)
        for _ in range(args.steps):
            lap_step()
        c1.record(stream)
        torch.cuda.synchronize()
        ms_l = c0.elapsed_time(c1) / args.steps
        result["laplacian"] = {"solves_per_s": B / (ms_l / 1e3), "ms_per_step": ms_l,
                               "over_plain": ms_l / ms_step,
                               "input": "L ~ N(0, 1) minus its mean, [B][H+1][W+1]"}
        del Lap

    if not args.no_volume:
        result["volume"] = volume_bench(torch, gfc, dev, stream, max(args.steps // 2, 3))

    if not args.no_bwd:
        du = torch.randn_like(gx) * 0.1
        dgx = torch.empty_like(gx)
        dgy = torch.empty_like(gx)
        names_b = ["k_row_bfwd", "k_col_bwd", "k_row_binv"]

        def stage_bwd(k):
            st = L.gfc_solve_backward_stage(hp, k, du.data_ptr(), dgx.data_ptr(), dgy.data_ptr(),
                                            B, ws.data_ptr(), ws.numel(), sp)
            if st != 0:
                raise gfc.GFCError(st, f"gfc_solve_backward_stage({k})")

        for _ in range(2):
            for k in (1, 2, 3):
                stage_fwd(k)
            for k in (1, 2, 3):
                stage_bwd(k)
        torch.cuda.synchronize()
        nb = max(args.steps // 2, 3)
        evb = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(nb)]
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for i in range(nb):
            for k in (1, 2, 3):
                stage_fwd(k)
            for k in (1, 2, 3):
                stage_bwd(k)
        t1.record(stream)
        torch.cuda.synchronize()
        ms_pair = t0.elapsed_time(t1) / nb
        for i in range(nb):  # stage times, as for the forward steps
            for k in (1, 2, 3):
                stage_fwd(k)
            evb[i][0].record(stream)
            for k in (1, 2, 3):
                stage_bwd(k)
                evb[i][k].record(stream)
        torch.cuda.synchronize()
        bms = {n: sum(evb[i][k].elapsed_time(evb[i][k + 1]) for i in range(nb)) / nb
               for k, n in enumerate(names_b)}
        mb = stage_model(H, W_, w.N, K, Kb, "bwd")
        result["fwd_bwd"] = {"pairs_per_s": B / (ms_pair / 1e3), "ms_per_pair_step": ms_pair,
                             "stages_ms": {k: round(v, 5) for k, v in bms.items()},
                             "bwd_hbm_frac": sum(v[0] for v in mb.values()) * B /
                             (sum(bms.values()) / 1e3) / HBM_PEAK}

    if not args.no_ragged:
        result["ragged"] = ragged_bench(torch, gfc, synth, dev, stream, max(args.steps // 2, 3))

    if not args.no_small:
        result["small_configs"] = small_configs_bench(torch, gfc, dev, stream, max(args.steps, 5))

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(w)
    result["paper_context"] = PAPER_CONTEXT
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
