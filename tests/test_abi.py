"""CPU-side checks of the C ABI: the library loads, exports every function the header
declares, validates arguments on the host and builds the same Green's spectrum (eq. (22))
as the oracle. No kernel is launched here."""
import ctypes
import os

import numpy as np
import pytest

import oracle as O

gfc = pytest.importorskip("paper_1902_00176_amd")
if not os.path.exists(gfc.lib_path()):
    pytest.skip("libgfc.so not built", allow_module_level=True)


def test_library_exports_every_header_function():
    L = gfc.lib()
    names = gfc.header_functions()
    assert "gfc_solve_batch" in names and "gfc_solve_backward" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings():
    L = gfc.lib()
    assert L.gfc_status_str(0) == b"GFC_OK"
    assert L.gfc_status_str(4) == b"GFC_E_WORKSPACE"


@pytest.mark.parametrize("H,W,M,N,status", [
    (0, 5, 0, 0, 1), (5, -1, 0, 0, 1), (10, 10, 11, 24, 2), (10, 10, 24, 11, 2),
    (10, 10, 24, 22, 2),   # 22 = 2 * 11 is not 2/3/5-smooth: no row FFT
    (10, 10, 12, 24, 0), (801, 1200, 0, 0, 0), (64, 64, 128, 128, 0),
    (1, 1, 0, 0, 0), (4, 4, 0, 0, 0), (32767, 4, 0, 0, 0),  # tiny and tallest default tori
    (1 << 15, 4, 0, 0, 2), (4, (1 << 15) + 1, 0, 0, 2),    # past the height / width limits
    (10, 1300, 0, 0, 0), (10, 1100, 0, 0, 0), (10, 1920, 0, 0, 0),  # default N 2700, 2250, 3840
    (10, 2047, 0, 0, 0),   # the widest default torus: N = 4096
    (10, 2049, 0, 0, 2),   # default N = 4320 has no row FFT (longest: 4096)
    (10, 2399, 0, 2400, 2),  # N < W + 2
])
def test_plan_create_validation(H, W, M, N, status):
    L = gfc.lib()
    h = ctypes.c_void_p()
    st = L.gfc_plan_create(ctypes.byref(h), H, W, M, N, 0)
    assert st == status
    if st == 0:
        L.gfc_plan_destroy(h)
    L.gfc_plan_destroy(None)  # destroying NULL is a no-op


def test_default_grid_and_offsets():
    p = gfc.Plan(801, 1200)
    assert (p.M, p.N) == (1620, 2400)
    assert (p.oy, p.ox) == O.block_offset(801, 1200, 1620, 2400)
    p = gfc.Plan(512, 512)
    assert (p.M, p.N) == (1024, 1024)
    p = gfc.Plan(256, 256)
    assert (p.M, p.N) == (512, 512)


def test_solve_without_build_is_an_error_code():
    L = gfc.lib()
    p = gfc.Plan(16, 16, 40, 40)
    st = L.gfc_solve_batch(p.handle, None, None, None, 1, None, 0, None)
    assert st == 3  # GFC_E_NOT_BUILT: no device touched
    n = ctypes.c_size_t()
    assert L.gfc_workspace_size(p.handle, -1, ctypes.byref(n)) == 1


def test_workspace_grows_linearly_with_batch():
    p = gfc.Plan(801, 1200)
    w1, w2, w100 = p.workspace_size(1), p.workspace_size(2), p.workspace_size(100)
    assert p.workspace_size(0) == 0
    assert w2 > w1 and w100 >= 50 * w2 * 0.99
    # the big term is one [H+1][N/2+1] complex64 array per image
    assert w100 >= 100 * 802 * 1201 * 8


@pytest.mark.parametrize("H,W,M,N", [(5, 6, 12, 16), (64, 64, 128, 128), (100, 37, 210, 80)])
def test_exported_green_spectrum_matches_oracle(H, W, M, N):
    p = gfc.Plan(H, W, M, N)
    G = p.green_spectrum()
    ref = O.green_spectrum(M, N)[:, : N // 2 + 1]
    assert G.shape == ref.shape
    assert np.max(np.abs(G - ref)) <= 1e-15 * np.max(np.abs(ref))


def test_supported_lengths_cover_the_workloads():
    for n in (64, 128, 512, 1024, 2048, 2400, 1620, 1200, 2250, 2560, 3840, 4096):
        assert gfc.supported_length(n), n
    for n in (22, 4100, 4320, 4608):
        assert not gfc.supported_length(n), n


def test_ragged_create_host_logic():
    """Ragged objects are created on the host: sizes resolve to each image's default torus,
    offsets are the packed prefix sums, bad sizes or flags are rejected."""
    import gfc_synth as synth
    sizes = [(64, 64), (37, 45), (801, 1200), (5, 3, 16, 16)]
    r = gfc.Ragged(sizes)
    assert r.B == 4
    for (H, W, *mn), (h, w, M, N) in zip(sizes, r.sizes):
        assert (h, w) == (H, W)
        assert (M, N) == (tuple(mn) if mn else synth.default_grid(H, W))
    assert list(r.offsets) == [0, 4096, 4096 + 37 * 45, 4096 + 37 * 45 + 801 * 1200,
                               4096 + 37 * 45 + 801 * 1200 + 15]
    L = gfc.lib()
    h = ctypes.c_void_p()
    H = (ctypes.c_int * 2)(10, 10)
    W = (ctypes.c_int * 2)(10, 10)
    N = (ctypes.c_int * 2)(0, 22)  # 22 has no row FFT
    assert L.gfc_ragged_create(ctypes.byref(h), 2, H, W, None, N, 0) == 2
    assert L.gfc_ragged_create(ctypes.byref(h), 2, H, W, None, None, 8) == 1
    assert L.gfc_ragged_create(ctypes.byref(h), -1, H, W, None, None, 0) == 1
    assert L.gfc_ragged_create(ctypes.byref(h), 2, H, W, None, None, 0) == 0
    n = ctypes.c_size_t()
    assert L.gfc_ragged_workspace_size(h, ctypes.byref(n)) == 3  # not built
    assert L.gfc_ragged_solve(h, None, None, None, None, 0, None) == 3
    L.gfc_ragged_destroy(h)


def test_plan_parameters_round_trip_and_low_bins():
    """Launch parameters are set and read back on the host; out-of-range values and unknown
    names are rejected; Kb is a read-only value of the plan; K defaults by the torus shape
    (the smallest of 4, 8, 16, 32 with N <= 16 K M) and may be raised up to 32."""
    want = {"col_c": 8, "col_rows": 32, "col_rows_b": 16, "low_bins": 4}
    p = gfc.Plan(801, 1200, params=want, tuned=False)
    got = p.params
    assert got.pop("row_split") == p.get_param("row_split_fwd")
    assert got == want
    assert p.get_param("low_bins_b") == 64
    # the split of each row pass is one compiled for the length; others are refused
    import sys
    sys.path.insert(0, os.path.dirname(gfc.__file__))
    import build_lib
    cands = build_lib.candidate_splits(2400)
    for ps in ("fwd", "edit", "inv", "bfwd", "binv"):
        n1 = p.get_param("row_split_" + ps)
        assert (n1, 2400 // n1) in cands, (ps, n1)
    assert gfc.lib().gfc_plan_set_param(p.handle, b"row_split", 7) == 1
    L = gfc.lib()
    for name, value in (("row_ppw", 1), ("col_c", 0), ("col_c", 3), ("col_rows", 24),
                        ("col_rows_b", 8), ("low_bins", 3), ("low_bins", 33),
                        ("low_bins_b", 8), ("row_strip", 4)):
        assert L.gfc_plan_set_param(p.handle, name.encode(), value) == 1, (name, value)
    assert L.gfc_plan_set_param(p.handle, b"low_bins", 13) == 0
    assert p.get_param("low_bins") == 13
    # a short row: Kb is capped by the half spectrum; K may not reach N / 2
    q = gfc.Plan(5, 6, 12, 16)
    assert q.get_param("low_bins") == 4 and q.get_param("low_bins_b") == 8
    assert L.gfc_plan_set_param(q.handle, b"low_bins", 8) == 1
    # default K by the torus shape: N <= 16 K M
    for (H, W, M, N), K in (((2, 1200, 6, 2400), 32), ((8, 1200, 16, 2400), 16),
                            ((16, 1200, 32, 2400), 8), ((32, 1200, 64, 2400), 4),
                            ((3, 1250, 8, 2400), 32), ((5000, 6, 10000, 16), 4)):
        assert gfc.Plan(H, W, M, N, tuned=False).get_param("low_bins") == K, (H, W, M, N)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """The product path has no fallback: without the HIP library every entry raises."""
    monkeypatch.setattr(gfc, "_lib", None)
    monkeypatch.setattr(gfc, "_LIB_PATH", str(tmp_path / "libgfc.so"))
    with pytest.raises(RuntimeError, match="missing"):
        gfc.lib()
    with pytest.raises(RuntimeError, match="missing"):
        gfc.Plan(64, 64)
    with pytest.raises(RuntimeError, match="missing"):
        gfc.Ragged([(64, 64, 0, 0)])
