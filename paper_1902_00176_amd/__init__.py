"""MI355X (gfx950) Green Function Convolution solver.

Thin ctypes binding over libgfc.so (the C ABI in include/gfc.h). This module only
marshals arguments: every step of the solve runs in the library's HIP kernels. PyTorch is
used for device memory and streams. If the library is missing or no GPU is present, the
solve calls raise; there is no CPU fallback.

    import paper_1902_00176_amd as gfc
    u = gfc.solve(gx, gy)                  # gx, gy: float32 CUDA tensors [..., H, W]
    u = gfc.GFCFunction.apply(gx, gy)      # differentiable (adjoint kernels in backward)
"""
from __future__ import annotations

import ctypes
import os
import re
import threading

import numpy as np

__all__ = ["GFCError", "Plan", "lib", "lib_path", "solve", "solve_backward", "GFCFunction",
           "supported_length", "default_grid", "header_functions"]

_HERE = os.path.dirname(os.path.abspath(__file__))
# GFC_LIBRARY names another build of the library (the autotuner's candidate library)
_LIB_PATH = os.environ.get("GFC_LIBRARY") or os.path.join(_HERE, "libgfc.so")
_HEADER = os.path.join(os.path.dirname(_HERE), "include", "gfc.h")
_lib = None
_lock = threading.Lock()

_STATUS = {0: "GFC_OK", 1: "GFC_E_ARG", 2: "GFC_E_SIZE", 3: "GFC_E_NOT_BUILT",
           4: "GFC_E_WORKSPACE", 5: "GFC_E_HIP", 6: "GFC_E_OOM"}


class GFCError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where} failed: {_STATUS.get(status, status)}")


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """Load libgfc.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                                   "python paper_1902_00176_amd/build_lib.py")
            L = ctypes.CDLL(_LIB_PATH)
            vp, i, u, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint, ctypes.c_size_t
            ip = ctypes.POINTER(ctypes.c_int)
            L.gfc_plan_create.argtypes = [ctypes.POINTER(vp), i, i, i, i, u]
            L.gfc_green_build.argtypes = [vp, vp]
            L.gfc_plan_get.argtypes = [vp, ip, ip, ip, ip, ip, ip]
            L.gfc_workspace_size.argtypes = [vp, i, ctypes.POINTER(sz)]
            L.gfc_solve_batch.argtypes = [vp, vp, vp, vp, i, vp, sz, vp]
            L.gfc_solve_backward.argtypes = [vp, vp, vp, vp, i, vp, sz, vp]
            L.gfc_solve_batch_color.argtypes = [vp, vp, vp, vp, vp, vp, i, vp, sz, vp]
            L.gfc_solve_edit.argtypes = [vp, vp, vp, vp, i, ctypes.c_float, vp, vp, vp, i, vp,
                                         sz, vp]
            L.gfc_solve_laplacian.argtypes = [vp, vp, vp, i, vp, sz, vp]
            L.gfc_solve_batch_noalloc.argtypes = [vp, vp, vp, vp, i, vp]
            L.gfc_solve_batch_noalloc.restype = ctypes.c_int
            L.gfc_plan3_create.argtypes = [ctypes.POINTER(vp), i, i, i, i, i, i, u]
            L.gfc_plan3_get.argtypes = [vp, ip, ip, ip, ip, ip, ip]
            L.gfc_green_build3.argtypes = [vp, vp]
            L.gfc_workspace3_size.argtypes = [vp, i, ctypes.POINTER(sz)]
            L.gfc_solve3_batch.argtypes = [vp, vp, vp, vp, vp, i, vp, sz, vp]
            L.gfc_plan3_destroy.argtypes = [vp]
            L.gfc_plan3_destroy.restype = None
            L.gfc_solve_batch_stage.argtypes = [vp, i, vp, vp, vp, i, vp, sz, vp]
            L.gfc_solve_backward_stage.argtypes = [vp, i, vp, vp, vp, i, vp, sz, vp]
            L.gfc_plan_set_param.argtypes = [vp, ctypes.c_char_p, i]
            L.gfc_plan_get_param.argtypes = [vp, ctypes.c_char_p, ip]
            L.gfc_green_export.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
            L.gfc_plan_destroy.argtypes = [vp]
            L.gfc_plan_destroy.restype = None
            L.gfc_supported_length.argtypes = [i]
            L.gfc_status_str.argtypes = [i]
            L.gfc_status_str.restype = ctypes.c_char_p
            for name in ("gfc_plan_create", "gfc_green_build", "gfc_plan_get",
                         "gfc_workspace_size", "gfc_solve_batch", "gfc_solve_backward",
                         "gfc_solve_batch_stage", "gfc_solve_backward_stage",
                         "gfc_plan_set_param", "gfc_plan_get_param",
                         "gfc_green_export", "gfc_supported_length"):
                getattr(L, name).restype = ctypes.c_int
            _bind_ragged(L)
            _lib = L
    return _lib


def _bind_ragged(L):
    vp, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    ip = ctypes.POINTER(ctypes.c_int)
    L.gfc_ragged_create.argtypes = [ctypes.POINTER(vp), i, ip, ip, ip, ip, ctypes.c_uint]
    L.gfc_ragged_build.argtypes = [vp, vp]
    L.gfc_ragged_image.argtypes = [vp, i, ip, ip, ip, ip]
    L.gfc_ragged_offsets.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.gfc_ragged_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    L.gfc_ragged_solve.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    L.gfc_ragged_solve_sequential.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    for name in ("gfc_ragged_create", "gfc_ragged_build", "gfc_ragged_image", "gfc_ragged_offsets",
                 "gfc_ragged_workspace_size", "gfc_ragged_solve", "gfc_ragged_solve_sequential"):
        getattr(L, name).restype = ctypes.c_int
    L.gfc_ragged_destroy.argtypes = [vp]
    L.gfc_ragged_destroy.restype = None


def header_functions() -> list[str]:
    """Names of the functions include/gfc.h declares."""
    with open(_HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gfc_[a-z_0-9]+)\s*\(", text)))


def _check(st: int, where: str):
    if st != 0:
        raise GFCError(st, where)


def supported_length(n: int) -> bool:
    return bool(lib().gfc_supported_length(int(n)))


def default_grid(H: int, W: int) -> tuple[int, int]:
    def sm(n):
        m = max(2, n)
        while True:
            r = m
            for p in (2, 3, 5):
                while r % p == 0:
                    r //= p
            if r == 1 and m % 2 == 0:
                return m
            m += 1
    return sm(max(2 * H, H + 2)), sm(max(2 * W, W + 2, 16))


def _stream_ptr(torch, device, stream):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _nbytes(t) -> int:
    return t.numel() * t.element_size()


def _overlaps(a, b) -> bool:
    """True when the memory of tensors a and b intersects."""
    if a is None or b is None or a.numel() == 0 or b.numel() == 0 or a.device != b.device:
        return False
    a0, b0 = a.data_ptr(), b.data_ptr()
    return a0 < b0 + _nbytes(b) and b0 < a0 + _nbytes(a)


def check_out(out, shape, dev, inputs=(), name="out"):
    """Validate a caller-supplied output tensor before its pointer reaches a kernel: float32,
    contiguous, the expected shape, on `dev`, sharing no memory with the inputs."""
    import torch
    if not isinstance(out, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if out.device != dev:
        raise ValueError(f"{name} is on {out.device}, expected {dev}")
    if out.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {out.dtype}")
    if tuple(out.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(out.shape)}, expected {tuple(shape)}")
    if not out.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    for t in inputs:
        if _overlaps(out, t):
            raise ValueError(f"{name} must not share memory with an input")
    return out


def check_workspace(ws, need: int, dev, others=()):
    """Validate a caller-supplied workspace: a contiguous tensor on `dev` of at least `need`
    bytes (any dtype), sharing no memory with the inputs and outputs of the call."""
    import torch
    if not isinstance(ws, torch.Tensor):
        raise TypeError("workspace must be a tensor")
    if ws.device != dev:
        raise ValueError(f"workspace is on {ws.device}, expected {dev}")
    if not ws.is_contiguous():
        raise ValueError("workspace must be contiguous")
    if _nbytes(ws) < need:
        raise ValueError(f"workspace too small: need {need} bytes, got {_nbytes(ws)}")
    for t in others:
        if _overlaps(ws, t):
            raise ValueError("workspace must not share memory with the inputs or outputs")
    return ws


PARAMS = ("col_c", "col_rows", "col_rows_b", "low_bins", "row_split")
_TUNING_PATH = os.path.join(_HERE, "tuning.json")
_tuning_db = None


def tuning_db() -> dict:
    """Launch parameters chosen by the autotuner (autotune.py), keyed "HxW@MxN"."""
    global _tuning_db
    if _tuning_db is None:
        import json
        path = os.environ.get("GFC_TUNING_DB", _TUNING_PATH)
        try:
            with open(path) as f:
                _tuning_db = json.load(f).get("plans", {})
        except (OSError, ValueError):
            _tuning_db = {}
    return _tuning_db


def tuning_key(H, W, M, N) -> str:
    return f"{H}x{W}@{M}x{N}"


class Plan:
    """A solver plan for H x W images on an M x N torus (M = N = 0: default torus).

    Launch parameters come from the autotuner's database when it holds this size;
    `params` overrides them (see gfc_plan_set_param); `tuned=False` keeps the defaults."""

    def __init__(self, H: int, W: int, M: int = 0, N: int = 0, params: dict | None = None,
                 tuned: bool = True):
        L = lib()
        h = ctypes.c_void_p()
        _check(L.gfc_plan_create(ctypes.byref(h), int(H), int(W), int(M), int(N), 0),
               "gfc_plan_create")
        self._h = h
        vals = [ctypes.c_int() for _ in range(6)]
        _check(L.gfc_plan_get(h, *[ctypes.byref(v) for v in vals]), "gfc_plan_get")
        self.H, self.W, self.M, self.N, self.oy, self.ox = [v.value for v in vals]
        self._built_on = None
        merged = dict(tuning_db().get(tuning_key(self.H, self.W, self.M, self.N), {})) if tuned else {}
        merged.update(params or {})
        for k, v in merged.items():
            if k in PARAMS:
                self.set_param(k, v)

    def set_param(self, name: str, value: int):
        _check(lib().gfc_plan_set_param(self._h, name.encode(), int(value)),
               f"gfc_plan_set_param({name}={value})")

    def get_param(self, name: str) -> int:
        v = ctypes.c_int()
        _check(lib().gfc_plan_get_param(self._h, name.encode(), ctypes.byref(v)),
               f"gfc_plan_get_param({name})")
        return v.value

    @property
    def params(self) -> dict:
        return {k: self.get_param(k) for k in PARAMS}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.gfc_plan_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def build(self, device=None, stream=None):
        import torch
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self._built_on is None:
            with torch.cuda.device(dev):
                _check(lib().gfc_green_build(self._h, _stream_ptr(torch, dev, stream)),
                       "gfc_green_build")
            self._built_on = dev
        elif self._built_on != dev:
            raise ValueError(f"plan built on {self._built_on}, used on {dev}")
        return self

    def workspace_size(self, B: int) -> int:
        n = ctypes.c_size_t()
        _check(lib().gfc_workspace_size(self._h, int(B), ctypes.byref(n)), "gfc_workspace_size")
        return n.value

    def green_spectrum(self) -> np.ndarray:
        out = np.empty((self.M, self.N // 2 + 1), dtype=np.float64)
        _check(lib().gfc_green_export(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "gfc_green_export")
        return out

    def _prep(self, *ts):
        import torch
        dev = ts[0].device
        if dev.type != "cuda":
            raise ValueError("GFC tensors must be on a CUDA (HIP) device")
        for t in ts:
            if t.dtype != torch.float32 or t.device != dev:
                raise TypeError("GFC tensors must be float32 on one device")
            if t.shape[-2:] != (self.H, self.W):
                raise ValueError(f"expected [..., {self.H}, {self.W}], got {tuple(t.shape)}")
        self.build(dev)
        return torch, dev

    def solve(self, gx, gy, out=None, workspace=None, stream=None):
        torch, dev = self._prep(gx, gy)
        if gx.shape != gy.shape:
            raise ValueError("gx and gy must have the same shape")
        gx = gx.contiguous()
        gy = gy.contiguous()
        B = gx.numel() // (self.H * self.W)
        u = check_out(out, gx.shape, dev, (gx, gy)) if out is not None else torch.empty_like(gx)
        ws = self._workspace(torch, dev, B, workspace, (gx, gy, u))
        with torch.cuda.device(dev):
            _check(lib().gfc_solve_batch(self._h, gx.data_ptr(), gy.data_ptr(), u.data_ptr(), B,
                                         ws.data_ptr() if ws is not None else None,
                                         _nbytes(ws) if ws is not None else 0,
                                         _stream_ptr(torch, dev, stream)), "gfc_solve_batch")
        return u

    def solve_color(self, gx, gy, I_mean, I_std, out=None, workspace=None, stream=None):
        """Solve, then the colour-preserving correction of eq. (25): each image is rescaled
        to the mean I_mean and population standard deviation I_std of its source image
        (float32 tensors with one value per image, on the same device)."""
        torch, dev = self._prep(gx, gy)
        if gx.shape != gy.shape:
            raise ValueError("gx and gy must have the same shape")
        gx = gx.contiguous()
        gy = gy.contiguous()
        B = gx.numel() // (self.H * self.W)
        I_mean = torch.as_tensor(I_mean, dtype=torch.float32, device=dev).reshape(-1).contiguous()
        I_std = torch.as_tensor(I_std, dtype=torch.float32, device=dev).reshape(-1).contiguous()
        if I_mean.numel() != B or I_std.numel() != B:
            raise ValueError(f"expected {B} means and standard deviations")
        u = (check_out(out, gx.shape, dev, (gx, gy, I_mean, I_std)) if out is not None
             else torch.empty_like(gx))
        ws = self._workspace(torch, dev, B, workspace, (gx, gy, I_mean, I_std, u))
        with torch.cuda.device(dev):
            _check(lib().gfc_solve_batch_color(
                self._h, gx.data_ptr(), gy.data_ptr(), I_mean.data_ptr(), I_std.data_ptr(),
                u.data_ptr(), B, ws.data_ptr() if ws is not None else None,
                _nbytes(ws) if ws is not None else 0, _stream_ptr(torch, dev, stream)),
                "gfc_solve_batch_color")
        return u

    def solve_edit(self, gx, gy, mode: str, param: float, C=None, I_mean=None, I_std=None,
                   out=None, workspace=None, stream=None):
        """Edit the gradient on the device, solve, and optionally correct colours (eq. (25)).
        mode "threshold": param = tau (keep |E| >= tau, Sec. 3.2.3); mode "gdm": param =
        alpha with edge map C (eq. (26))."""
        modes = {"threshold": EDIT_THRESHOLD, "gdm": EDIT_GDM}
        if mode not in modes:
            raise ValueError(f"unknown edit mode {mode!r}")
        ts = [gx, gy] + ([C] if C is not None else [])
        torch, dev = self._prep(*ts)
        if gx.shape != gy.shape or (C is not None and C.shape != gx.shape):
            raise ValueError("gx, gy and C must have the same shape")
        gx, gy = gx.contiguous(), gy.contiguous()
        C = C.contiguous() if C is not None else None
        B = gx.numel() // (self.H * self.W)
        stats = []
        for t in (I_mean, I_std):
            if t is not None:
                t = torch.as_tensor(t, dtype=torch.float32, device=dev).reshape(-1).contiguous()
                if t.numel() != B:
                    raise ValueError(f"expected {B} means and standard deviations")
            stats.append(t)
        ins = [t for t in (gx, gy, C, *stats) if t is not None]
        u = check_out(out, gx.shape, dev, ins) if out is not None else torch.empty_like(gx)
        ws = self._workspace(torch, dev, B, workspace, ins + [u])
        ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
        with torch.cuda.device(dev):
            _check(lib().gfc_solve_edit(
                self._h, gx.data_ptr(), gy.data_ptr(), ptr(C), modes[mode], float(param),
                ptr(stats[0]), ptr(stats[1]), u.data_ptr(), B, ptr(ws),
                _nbytes(ws) if ws is not None else 0, _stream_ptr(torch, dev, stream)),
                "gfc_solve_edit")
        return u

    def solve_laplacian(self, L, out=None, workspace=None, stream=None):
        """Solve from the Laplacian itself (Algorithm B): L [..., H+1, W+1] float32 on the
        support of div E, summing to 0. Returns u [..., H, W]."""
        import torch
        dev = L.device
        if dev.type != "cuda" or L.dtype != torch.float32:
            raise TypeError("L must be a float32 CUDA tensor")
        if tuple(L.shape[-2:]) != (self.H + 1, self.W + 1):
            raise ValueError(f"expected [..., {self.H + 1}, {self.W + 1}], got {tuple(L.shape)}")
        self.build(dev)
        L = L.contiguous()
        B = L.numel() // ((self.H + 1) * (self.W + 1))
        shape = L.shape[:-2] + (self.H, self.W)
        u = (check_out(out, shape, dev, (L,)) if out is not None
             else torch.empty(shape, dtype=torch.float32, device=dev))
        ws = self._workspace(torch, dev, B, workspace, (L, u))
        with torch.cuda.device(dev):
            _check(lib().gfc_solve_laplacian(self._h, L.data_ptr(), u.data_ptr(), B,
                                             ws.data_ptr() if ws is not None else None,
                                             _nbytes(ws) if ws is not None else 0,
                                             _stream_ptr(torch, dev, stream)),
                   "gfc_solve_laplacian")
        return u

    def backward(self, du, workspace=None, stream=None):
        torch, dev = self._prep(du)
        du = du.contiguous()
        B = du.numel() // (self.H * self.W)
        dgx = torch.empty_like(du)
        dgy = torch.empty_like(du)
        ws = self._workspace(torch, dev, B, workspace, (du, dgx, dgy))
        with torch.cuda.device(dev):
            _check(lib().gfc_solve_backward(self._h, du.data_ptr(), dgx.data_ptr(), dgy.data_ptr(), B,
                                            ws.data_ptr() if ws is not None else None,
                                            _nbytes(ws) if ws is not None else 0,
                                            _stream_ptr(torch, dev, stream)), "gfc_solve_backward")
        return dgx, dgy

    def _workspace(self, torch, dev, B, workspace, others=()):
        if B == 0:
            return None
        need = self.workspace_size(B)
        if workspace is not None:
            return check_workspace(workspace, need, dev, others)
        return torch.empty(need, dtype=torch.uint8, device=dev)


_plans: dict = {}


def get_plan(H: int, W: int, M: int = 0, N: int = 0) -> Plan:
    key = (int(H), int(W), int(M), int(N))
    with _lock:
        p = _plans.get(key)
    if p is None:
        p = Plan(*key)
        with _lock:
            _plans[key] = p
    return p


def solve(gx, gy, M: int = 0, N: int = 0, **kw):
    """u = GFC(gx, gy) for float32 CUDA tensors of shape [..., H, W]."""
    return get_plan(gx.shape[-2], gx.shape[-1], M or 0, N or 0).solve(gx, gy, **kw)


def solve_color(gx, gy, I_mean, I_std, M: int = 0, N: int = 0, **kw):
    """GFC(gx, gy) with the colour correction of eq. (25) to the source statistics."""
    return get_plan(gx.shape[-2], gx.shape[-1], M or 0, N or 0).solve_color(gx, gy, I_mean,
                                                                            I_std, **kw)


def solve_laplacian(L, M: int = 0, N: int = 0, **kw):
    """u from the Laplacian L [..., H+1, W+1] (Algorithm B's input)."""
    return get_plan(L.shape[-2] - 1, L.shape[-1] - 1, M or 0, N or 0).solve_laplacian(L, **kw)


class Plan3:
    """A solver plan for D x H x W volumes on a P x M x N torus (0: default extents).
    Three-dimensional GFC: the 7-point divergence, the Green's spectrum 1/lambda of the
    7-point stencil, u = v[block] - v[0,0,0]."""

    def __init__(self, D: int, H: int, W: int, P: int = 0, M: int = 0, N: int = 0):
        L = lib()
        h = ctypes.c_void_p()
        _check(L.gfc_plan3_create(ctypes.byref(h), int(D), int(H), int(W), int(P), int(M),
                                  int(N), 0), "gfc_plan3_create")
        self._h = h
        vals = [ctypes.c_int() for _ in range(6)]
        _check(L.gfc_plan3_get(h, *[ctypes.byref(v) for v in vals]), "gfc_plan3_get")
        self.D, self.H, self.W, self.P, self.M, self.N = [v.value for v in vals]
        self._built_on = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.gfc_plan3_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def build(self, device=None, stream=None):
        import torch
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self._built_on is None:
            with torch.cuda.device(dev):
                _check(lib().gfc_green_build3(self._h, _stream_ptr(torch, dev, stream)),
                       "gfc_green_build3")
            self._built_on = dev
        elif self._built_on != dev:
            raise ValueError(f"plan built on {self._built_on}, used on {dev}")
        return self

    def workspace_size(self, B: int) -> int:
        n = ctypes.c_size_t()
        _check(lib().gfc_workspace3_size(self._h, int(B), ctypes.byref(n)), "gfc_workspace3_size")
        return n.value

    def solve(self, gx, gy, gz, out=None, workspace=None, stream=None):
        import torch
        dev = gx.device
        shape = (self.D, self.H, self.W)
        for t in (gx, gy, gz):
            if t.device != dev or t.dtype != torch.float32 or dev.type != "cuda":
                raise TypeError("volume fields must be float32 CUDA tensors on one device")
            if tuple(t.shape[-3:]) != shape or t.shape != gx.shape:
                raise ValueError(f"expected [..., {self.D}, {self.H}, {self.W}], got {tuple(t.shape)}")
        self.build(dev)
        gx, gy, gz = gx.contiguous(), gy.contiguous(), gz.contiguous()
        B = gx.numel() // (self.D * self.H * self.W)
        u = check_out(out, gx.shape, dev, (gx, gy, gz)) if out is not None else torch.empty_like(gx)
        need = self.workspace_size(B)
        ws = (check_workspace(workspace, need, dev, (gx, gy, gz, u)) if workspace is not None
              else torch.empty(need, dtype=torch.uint8, device=dev))
        with torch.cuda.device(dev):
            _check(lib().gfc_solve3_batch(self._h, gx.data_ptr(), gy.data_ptr(), gz.data_ptr(),
                                          u.data_ptr(), B, ws.data_ptr(),
                                          ws.numel() * ws.element_size(),
                                          _stream_ptr(torch, dev, stream)), "gfc_solve3_batch")
        return u


def solve3(gx, gy, gz, P: int = 0, M: int = 0, N: int = 0, **kw):
    """u = GFC(gx, gy, gz) for float32 CUDA volumes [..., D, H, W]."""
    D, H, W = gx.shape[-3:]
    return Plan3(D, H, W, P, M, N).solve(gx, gy, gz, **kw)


EDIT_THRESHOLD = 1
EDIT_GDM = 2


def solve_edit(gx, gy, mode, param, C=None, I_mean=None, I_std=None, M: int = 0, N: int = 0,
               **kw):
    """Gradient-domain editing: device-side edit (threshold or GDM), solve, optional eq. (25)."""
    return get_plan(gx.shape[-2], gx.shape[-1], M or 0, N or 0).solve_edit(
        gx, gy, mode, param, C=C, I_mean=I_mean, I_std=I_std, **kw)


def solve_backward(du, M: int = 0, N: int = 0, **kw):
    """(dgx, dgy) = adjoint of the solve applied to du [..., H, W]."""
    return get_plan(du.shape[-2], du.shape[-1], M or 0, N or 0).backward(du, **kw)


RAGGED_NO_GRAPH = 1


class Ragged:
    """A ragged batch: images of different sizes solved together (gfc_ragged_*).

    sizes: a list of (H, W) or (H, W, M, N) (M = N = 0: the default torus of that image).
    Inputs and outputs are packed float32 device tensors: image i occupies
    [offsets[i], offsets[i+1]) row-major. pack() / unpack() convert from / to lists.
    """

    def __init__(self, sizes, flags: int = 0):
        sizes = [tuple(int(v) for v in s) + (0, 0)[:4 - len(s)] for s in sizes]
        self.B = len(sizes)
        arr = lambda k: (ctypes.c_int * max(1, self.B))(*[s[k] for s in sizes])
        h = ctypes.c_void_p()
        _check(lib().gfc_ragged_create(ctypes.byref(h), self.B, arr(0), arr(1), arr(2), arr(3),
                                       int(flags)), "gfc_ragged_create")
        self._h = h
        self._built_on = None
        self.sizes = []
        for k in range(self.B):
            v = [ctypes.c_int() for _ in range(4)]
            _check(lib().gfc_ragged_image(h, k, *[ctypes.byref(x) for x in v]), "gfc_ragged_image")
            self.sizes.append(tuple(x.value for x in v))
        off = (ctypes.c_int64 * (self.B + 1))()
        _check(lib().gfc_ragged_offsets(h, off), "gfc_ragged_offsets")
        self.offsets = np.array(off[:], dtype=np.int64)
        self._ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.gfc_ragged_destroy(h)
            self._h = None

    def build(self, device=None, stream=None):
        import torch
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self._built_on is None:
            with torch.cuda.device(dev):
                _check(lib().gfc_ragged_build(self._h, _stream_ptr(torch, dev, stream)),
                       "gfc_ragged_build")
            self._built_on = dev
        elif self._built_on != dev:
            raise ValueError(f"ragged batch built on {self._built_on}, used on {dev}")
        return self

    def workspace_size(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().gfc_ragged_workspace_size(self._h, ctypes.byref(n)), "gfc_ragged_workspace_size")
        return n.value

    def pack(self, arrays, device):
        """Concatenate a list of [H_i, W_i] arrays/tensors into one packed float32 tensor."""
        import torch
        parts = [torch.as_tensor(a, dtype=torch.float32).reshape(-1) for a in arrays]
        return torch.cat(parts).to(device) if parts else torch.empty(0, device=device)

    def unpack(self, packed):
        return [packed[self.offsets[k]:self.offsets[k + 1]].view(self.sizes[k][0], self.sizes[k][1])
                for k in range(self.B)]

    def _run(self, fn, name, gx, gy, out, workspace, stream):
        import torch
        dev = gx.device
        for t in (gx, gy):
            if t.dtype != torch.float32 or t.device != dev or t.dim() != 1 or not t.is_contiguous():
                raise TypeError("packed inputs must be contiguous 1-D float32 tensors on one device")
            if t.numel() != int(self.offsets[-1]):
                raise ValueError(f"packed inputs must hold {int(self.offsets[-1])} elements")
        self.build(dev)
        u = check_out(out, gx.shape, dev, (gx, gy)) if out is not None else torch.empty_like(gx)
        need = self.workspace_size()
        if workspace is None:
            if self._ws is None or _nbytes(self._ws) < need or self._ws.device != dev:
                self._ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
            workspace = self._ws
        else:
            check_workspace(workspace, need, dev, (gx, gy, u))
        with torch.cuda.device(dev):
            _check(fn(self._h, gx.data_ptr(), gy.data_ptr(), u.data_ptr(), workspace.data_ptr(),
                      _nbytes(workspace), _stream_ptr(torch, dev, stream)),
                   name)
        return u

    def solve(self, gx, gy, out=None, workspace=None, stream=None):
        """Packed forward solve of every image (one graph replay once captured)."""
        return self._run(lib().gfc_ragged_solve, "gfc_ragged_solve", gx, gy, out, workspace, stream)

    def solve_sequential(self, gx, gy, out=None, workspace=None, stream=None):
        """The same result by one single-image plain solve per image."""
        return self._run(lib().gfc_ragged_solve_sequential, "gfc_ragged_solve_sequential", gx, gy,
                         out, workspace, stream)


def ragged_solve(pairs, device=None):
    """Solve a list of (gx, gy) pairs of different sizes in one ragged launch; returns the
    list of u (views into one packed tensor)."""
    import torch
    dev = torch.device(device) if device is not None else pairs[0][0].device
    r = Ragged([tuple(gx.shape[-2:]) for gx, _ in pairs])
    gx = r.pack([p[0] for p in pairs], dev)
    gy = r.pack([p[1] for p in pairs], dev)
    return r.unpack(r.solve(gx, gy))


def _make_function():
    import torch

    class GFCFunction(torch.autograd.Function):
        """u = GFC(gx, gy) as a differentiable layer (the map is linear: nothing is saved)."""

        @staticmethod
        def forward(ctx, gx, gy, M: int = 0, N: int = 0):
            ctx.grid = (M, N)
            return solve(gx, gy, M, N)

        @staticmethod
        def backward(ctx, du):
            dgx, dgy = solve_backward(du, *ctx.grid)
            return dgx, dgy, None, None

    return GFCFunction


class _LazyFunction:
    _f = None

    def __getattr__(self, name):
        if _LazyFunction._f is None:
            _LazyFunction._f = _make_function()
        return getattr(_LazyFunction._f, name)


GFCFunction = _LazyFunction()
