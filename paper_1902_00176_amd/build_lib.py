"""Build libgfc.so (HIP, gfx950) in-tree.

The row-pass kernels are templates on the two factors N = N1 * N2 of the row length; one
translation unit is generated per supported length so they compile in parallel, plus a
table TU that maps N to its launchers. Output: paper_1902_00176_amd/libgfc.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
GEN = os.path.join(BUILD, "gen")
LIB = os.path.join(HERE, "libgfc.so")
# the autotuner's library of candidate row splits (built on demand, never shipped)
BUILD_TUNE = os.path.join(HERE, "_build_tune")
LIB_TUNE = os.path.join(BUILD_TUNE, "libgfc_tune.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", f"-I{INCLUDE}", f"-I{CSRC}"]


def smooth235(n: int) -> bool:
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def _pow2ceil(v: int) -> int:
    return 8 if v <= 8 else 16 if v <= 16 else 32 if v <= 32 else 64


def choose_factors(N: int):
    """(N1, N2) with N1*N2 = N, both 2/3/5-smooth and <= 64: fewest lanes per FFT, then
    the most balanced split, with N2 (the lane count of the load step) the larger."""
    best = None
    for n1 in range(2, 65):
        if N % n1:
            continue
        n2 = N // n1
        if n2 < 2 or n2 > 64 or not smooth235(n1) or not smooth235(n2) or n2 < n1:
            continue
        key = (_pow2ceil(max(n1, n2)), n2 - n1)
        if best is None or key < best[0]:
            best = (key, n1, n2)
    return None if best is None else (best[1], best[2])


MAX_ROW_LENGTH = 4096  # 64 x 64: one wavefront of 64 lanes holding 64 values each


def default_lengths():
    """Row lengths compiled into the library: every even 2/3/5-smooth N in [16, 4096] that
    splits into two factors <= 64 (so the default torus of every image up to 2047 pixels
    wide, and 2048 on a 4096-point row, is supported)."""
    return [n for n in range(16, MAX_ROW_LENGTH + 1, 2)
            if smooth235(n) and choose_factors(n) is not None]


def z_lengths():
    """Volume depths P (the torus along z) compiled into the library: every even
    2/3/5-smooth P in [4, 512] that splits into two factors <= 64."""
    return [p for p in range(4, 513, 2) if smooth235(p) and choose_factors(p) is not None]


TUNING = os.path.join(HERE, "tuning.json")
PASSES = ("fwd", "inv", "bfwd", "binv")


def candidate_splits(N: int):
    """Splits N = N1 * N2 the autotuner compares: both factors 2/3/5-smooth and <= 64, with
    the fewest lanes per slot (the smallest power of two >= max(N1, N2)), both orders."""
    out = []
    for n1 in range(2, 65):
        if N % n1:
            continue
        n2 = N // n1
        if 2 <= n2 <= 64 and smooth235(n1) and smooth235(n2):
            out.append((n1, n2))
    if not out:
        return []
    g = min(_pow2ceil(max(a, b)) for a, b in out)
    return [(a, b) for a, b in out if _pow2ceil(max(a, b)) == g]


def tuned_splits():
    """Per row length and pass, the split the autotuner chose (tuning.json "row_splits"),
    {N: {pass: (N1, N2)}}; lengths or passes it does not hold take choose_factors."""
    import json
    try:
        with open(os.environ.get("GFC_TUNING_DB", TUNING)) as f:
            raw = json.load(f).get("row_splits", {})
    except (OSError, ValueError):
        return {}
    out = {}
    for n, d in raw.items():
        N = int(n)
        ent = {}
        for ps in PASSES + ("edit",):
            v = d.get(ps)
            if v and len(v) == 2 and v[0] * v[1] == N and tuple(v) in candidate_splits(N):
                ent[ps] = (int(v[0]), int(v[1]))
        out[N] = ent
    return out


def pass_splits(N: int, tuned=None):
    """The split of each row pass of length N: tuned where tuning.json holds one, else the
    default (fewest lanes, most balanced)."""
    tuned = tuned_splits() if tuned is None else tuned
    d = choose_factors(N)
    t = tuned.get(N, {})
    return {ps: t.get(ps, d) for ps in PASSES}


def _z_split(P: int):
    """(P1, P2) for the z transform: choose_factors where it applies, else 2 x P/2."""
    f = choose_factors(P)
    return f if f is not None else (2, P // 2)


def _lengths_from_env():
    v = os.environ.get("GFC_ROW_LENGTHS")
    if not v:
        return default_lengths()
    return sorted({int(t) for t in v.replace(",", " ").split()})


RGM_BUCKET = 24  # row lengths per multi-length ragged launch


def rg_buckets(lengths):
    """Groups of row lengths that share one ragged launch: lengths of one workgroup size
    (64 threads for 64-lane slots, else 256) and of one side of 2048, in order, split into
    near-equal groups of at most RGM_BUCKET."""
    cls = {}
    for n in lengths:
        n1, n2 = choose_factors(n)
        # class: workgroup size, and rows beyond 2048 points apart (images wider than 1024
        # pixels), so their larger LDS and registers do not lower the occupancy of the rest
        cls.setdefault((64 if _pow2ceil(max(n1, n2)) == 64 else 256, n > 2048), []).append(n)
    out = []
    for t in sorted(cls):
        ns = sorted(cls[t])
        k = -(-len(ns) // RGM_BUCKET)
        size = -(-len(ns) // k)
        out += [ns[i:i + size] for i in range(0, len(ns), size)]
    return out


def generate(lengths, tune=False):
    """Translation units: one per row length (its entry with the split of each pass), the
    multi-length ragged groups, the table of entries and the z transforms. tune=True: every
    candidate split of every length as its own entry (plain passes only), for the autotuner."""
    os.makedirs(GEN, exist_ok=True)
    srcs = []
    tuned = tuned_splits()
    entries = []  # (symbol, N)
    for n in lengths:
        path = os.path.join(GEN, f"row_{n}.hip")
        body = ""
        if tune:
            for n1, n2 in candidate_splits(n):
                sym = f"gfc_row_entry_{n}_{n1}"
                body += (f"const RowKernels* {sym}() {{\n"
                         f"  static const RowKernels k = GFC_ROW_ENTRY_CANDIDATE({n1}, {n2});\n"
                         f"  return &k;\n}}\n")
                entries.append((sym, n))
        else:
            sp = pass_splits(n, tuned)
            # the forward modes other than the plain solve (gradient edits, a given Laplacian,
            # volume slices) take the "edit" split where tuning.json names one (measured by
            # hand: the autotuner times the plain passes only), else the default split
            e_sp = tuned.get(n, {}).get("edit", choose_factors(n))
            order = [sp["fwd"], e_sp, sp["inv"], sp["bfwd"], sp["binv"]]
            args = ", ".join(f"{a}, {b}" for a, b in order)
            sym = f"gfc_row_entry_{n}"
            body = (f"const RowKernels* {sym}() {{\n"
                    f"  static const RowKernels k = GFC_ROW_ENTRY({args});\n"
                    f"  return &k;\n}}\n")
            entries.append((sym, n))
        text = f'#include "gfc_row.h"\nnamespace gfc {{\n{body}}}  // namespace gfc\n'
        _write_if_changed(path, text)
        srcs.append(path)
    buckets = [] if tune else rg_buckets(lengths)
    for k, ns in enumerate(buckets):
        def rl(n):
            sp = pass_splits(n, tuned)
            return f"RowLen<{sp['fwd'][0]}, {sp['fwd'][1]}, {sp['inv'][0]}, {sp['inv'][1]}>"
        lens = ", ".join(rl(n) for n in ns)
        path = os.path.join(GEN, f"row_rgm_{k}.hip")
        text = (f'#include "gfc_row.h"\n'
                f"namespace gfc {{\n"
                f"using RgmK{k} = RowMulti<{lens}>;\n"
                f"const RgMulti* gfc_rgm_entry_{k}() {{\n"
                f"  static const RgMulti m{{{k}, &RgmK{k}::fwd, &RgmK{k}::inv}};\n"
                f"  return &m;\n}}\n}}  // namespace gfc\n")
        _write_if_changed(path, text)
        srcs.append(path)
    rgm_decl = "".join(f"const RgMulti* gfc_rgm_entry_{k}();\n" for k in range(len(buckets)))
    rgm_cases = "".join(f"    case {n}: return gfc_rgm_entry_{k}();\n"
                        for k, ns in enumerate(buckets) for n in ns)
    decl = rgm_decl + "".join(f"const RowKernels* {sym}();\n" for sym, _ in entries)
    calls = ",\n      ".join(f"{sym}()" for sym, _ in entries)
    ne = len(entries)
    table = (f'#include "gfc_internal.h"\nnamespace gfc {{\n{decl}'
             f"static const RowKernels* const* table() {{\n"
             f"  static const RowKernels* const t[] = {{\n      {calls}}};\n  return t;\n}}\n"
             f"int row_kernel_count() {{ return {ne}; }}\n"
             f"const RowKernels* row_kernel_at(int i) {{ return table()[i]; }}\n"
             f"const RowKernels* find_row_kernels(int N) {{\n"
             f"  for (int i = 0; i < {ne}; ++i)\n"
             f"    if (table()[i]->N == N) return table()[i];\n"
             f"  return nullptr;\n}}\n"
             f"const RowKernels* find_row_kernels_split(int N, int N1) {{\n"
             f"  for (int i = 0; i < {ne}; ++i)\n"
             f"    if (table()[i]->N == N && table()[i]->f.N1 == N1) return table()[i];\n"
             f"  return nullptr;\n}}\n"
             f"const RgMulti* find_rg_multi(int N) {{\n  switch (N) {{\n{rgm_cases}"
             f"    default: return nullptr;\n  }}\n}}\n}}  // namespace gfc\n")
    tpath = os.path.join(GEN, "row_table.hip")
    _write_if_changed(tpath, table)
    # z transforms of volumes: one unit for all depths (small kernels)
    zl = z_lengths()
    zt = ('#include "gfc_zfft.h"\nnamespace gfc {\n'
          "static const ZKernels kZ[] = {\n    "
          + ",\n    ".join(f"GFC_Z_ENTRY({_z_split(p)[0]}, {_z_split(p)[1]})" for p in zl)
          + "};\n"
          f"const ZKernels* find_z_kernels(int P) {{\n  for (int i = 0; i < {len(zl)}; ++i)\n"
          "    if (kZ[i].P == P) return &kZ[i];\n  return nullptr;\n}\n}  // namespace gfc\n")
    zpath = os.path.join(GEN, "z_table.hip")
    _write_if_changed(zpath, zt)
    return srcs + [tpath, zpath]


def _write_if_changed(path, text):
    if os.path.exists(path):
        with open(path) as f:
            if f.read() == text:
                return
    with open(path, "w") as f:
        f.write(text)


def _compile(src, obj):
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    return obj


def build(lengths=None, jobs=None, verbose=True, force=False, tune=False):
    """Compile the library. tune=True builds the autotuner's candidate library instead:
    every candidate split of every row length, plain passes only, written to LIB_TUNE in a
    build folder of its own (the default library is not touched)."""
    global BUILD, GEN, LIB
    if tune:
        BUILD, GEN, LIB = BUILD_TUNE, os.path.join(BUILD_TUNE, "gen"), LIB_TUNE
    lengths = lengths or _lengths_from_env()
    if os.path.isdir(BUILD) and force:
        shutil.rmtree(BUILD)
    os.makedirs(BUILD, exist_ok=True)
    units = ("gfc_api.hip", "gfc_col.hip", "gfc_ragged.hip", "gfc_color.hip", "gfc_lowext.hip",
             "gfc_noalloc.hip")
    srcs = [os.path.join(CSRC, f) for f in units] + generate(lengths, tune=tune)
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    headers.append(os.path.join(INCLUDE, "gfc.h"))
    newest_hdr = max(os.path.getmtime(h) for h in headers)
    jobs = jobs or min(16, os.cpu_count() or 4)
    todo = []
    objs = []
    for s in srcs:
        o = os.path.join(BUILD, os.path.basename(s).replace(".hip", ".o"))
        objs.append(o)
        if force or not os.path.exists(o) or os.path.getmtime(o) < max(os.path.getmtime(s), newest_hdr):
            todo.append((s, o))
    if verbose:
        print(f"[gfc build] {len(lengths)} row lengths, compiling {len(todo)}/{len(srcs)} units "
              f"with {jobs} jobs", flush=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, s, o) for s, o in todo]
        for f in cf.as_completed(futs):
            f.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"[gfc build] wrote {LIB}", flush=True)
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv, tune="--tune" in sys.argv)
