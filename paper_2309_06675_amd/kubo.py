"""Thin Python binding of the C ABI in include/kubo.h (argument marshalling only).

Every step of the computation runs in the HIP library ``libkubo.so``; this
module converts arguments, owns the workspace tensor and passes PyTorch's
current stream.  If the library is missing the import fails loudly: there is
no CPU fallback.

Low-level names mirror the C entry points (``kubo_plan``, ``kubo_ahc``,
``kubo_ahc_backward``, ``kubo_plan_device_status``, ``kubo_plan_destroy``,
``kubo_status_string``, ``kubo_plan_info``).  On top of them:

* :class:`Plan` -- a plan plus its workspace (a uint8 CUDA tensor),
* :func:`ahc` -- a differentiable ``torch.autograd.Function`` front end.
"""

from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkubo.so")

KUBO_OK = 0
KUBO_E_INVALID = 1
KUBO_E_UNSUPPORTED = 2
KUBO_E_WORKSPACE = 3
KUBO_E_HIP = 4
KUBO_E_NOCONV = 5
KUBO_E_NONFINITE = 6

KUBO_F_GRAPH = 0x1
KUBO_F_TIMING = 0x2
KUBO_F_FORWARD_ONLY = 0x4
KUBO_F_TENSOR = 0x8
TENSOR_COMPONENTS = ("xy", "yz", "zx", "spin_xy")
KUBO_F_DEBUG_SWEEPCAP = 0x100

EXPORTED = ("kubo_plan", "kubo_ahc", "kubo_ahc_backward", "kubo_plan_device_status",
            "kubo_plan_destroy", "kubo_status_string", "kubo_plan_info", "kubo_plan_kernel_time",
            "kubo_ahc_noalloc", "kubo_ahc_tensor", "kubo_ahc_gf")

KUBO_NOALLOC_MAX_BYTES = 64 << 20
KUBO_GF_MAX_NODES = 65536
KUBO_DEVICE_NOCONV = 0x1
KUBO_DEVICE_NONFINITE = 0x2


class KuboError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {kubo_status_string(status)}")


class kubo_model_desc(ctypes.Structure):
    _fields_ = [("n_orb", ctypes.c_int32), ("n_R", ctypes.c_int32),
                ("R", ctypes.POINTER(ctypes.c_int32)), ("grid", ctypes.c_int32 * 3),
                ("k_begin", ctypes.c_int64), ("k_count", ctypes.c_int64)]


class kubo_tile(ctypes.Structure):
    _fields_ = [("n_orb", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("k_block", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libkubo.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2309_06675_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.kubo_plan.restype = ctypes.c_int
        L.kubo_plan.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(kubo_model_desc), ctypes.c_int32,
                                ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(kubo_tile),
                                ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.kubo_ahc.restype = ctypes.c_int
        L.kubo_ahc.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double, vp, vp,
                               ctypes.c_size_t, vp]
        L.kubo_ahc_tensor.restype = ctypes.c_int
        L.kubo_ahc_tensor.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double, vp, vp, vp,
                                      ctypes.c_size_t, vp]
        L.kubo_ahc_backward.restype = ctypes.c_int
        L.kubo_ahc_backward.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double, vp, vp, vp,
                                        ctypes.c_size_t, vp]
        L.kubo_plan_device_status.restype = ctypes.c_int
        L.kubo_plan_device_status.argtypes = [vp, vp, vp]
        L.kubo_plan_destroy.restype = None
        L.kubo_plan_destroy.argtypes = [vp]
        L.kubo_status_string.restype = ctypes.c_char_p
        L.kubo_status_string.argtypes = [ctypes.c_int]
        L.kubo_plan_kernel_time.restype = ctypes.c_int
        L.kubo_plan_kernel_time.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
        L.kubo_ahc_gf.restype = ctypes.c_int
        L.kubo_ahc_gf.argtypes = [vp, vp, vp, ctypes.c_double, vp, vp, ctypes.c_int32, vp, vp,
                                  ctypes.c_size_t, vp]
        L.kubo_ahc_noalloc.restype = ctypes.c_int
        L.kubo_ahc_noalloc.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double, vp, vp, vp]
        L.kubo_plan_info.restype = ctypes.c_int
        L.kubo_plan_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int32)]
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# same-name wrappers of the C entry points
# ---------------------------------------------------------------------------


def kubo_status_string(status: int) -> str:
    return lib().kubo_status_string(int(status)).decode()


def kubo_plan(models: Sequence[kubo_model_desc], n_fermi: int, flags: int = 0,
              tiles: Optional[Sequence[kubo_tile]] = None):
    """Returns (status, plan handle or None, workspace bytes)."""
    arr = (kubo_model_desc * len(models))(*models)
    tl = None
    nt = 0
    if tiles:
        tl = (kubo_tile * len(tiles))(*tiles)
        nt = len(tiles)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t(0)
    st = lib().kubo_plan(ctypes.byref(h), arr, len(models), int(n_fermi), int(flags), tl, nt,
                         ctypes.byref(ws))
    return st, (h if st == KUBO_OK else None), ws.value


def kubo_ahc(plan, t_ptr: int, ef_ptr: int, eta: float, kT: float, sigma_ptr: int, ws_ptr: int,
             ws_bytes: int, stream: int) -> int:
    return lib().kubo_ahc(plan, t_ptr, ef_ptr, float(eta), float(kT), sigma_ptr, ws_ptr,
                          int(ws_bytes), stream)


def kubo_ahc_tensor(plan, t_ptr: int, ef_ptr: int, eta: float, kT: float, spin_ptr: int,
                    sigma_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> int:
    return lib().kubo_ahc_tensor(plan, t_ptr, ef_ptr, float(eta), float(kT), spin_ptr, sigma_ptr,
                                 ws_ptr, int(ws_bytes), stream)


def kubo_ahc_gf(plan, t_ptr: int, ef_ptr: int, gamma: float, omega_ptr: int, weight_ptr: int,
                n_omega: int, sigma_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> int:
    return lib().kubo_ahc_gf(plan, t_ptr, ef_ptr, float(gamma), omega_ptr, weight_ptr,
                             int(n_omega), sigma_ptr, ws_ptr, int(ws_bytes), stream)


def kubo_ahc_backward(plan, t_ptr: int, ef_ptr: int, eta: float, kT: float, sbar_ptr: int,
                      grad_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> int:
    return lib().kubo_ahc_backward(plan, t_ptr, ef_ptr, float(eta), float(kT), sbar_ptr, grad_ptr,
                                   ws_ptr, int(ws_bytes), stream)


def kubo_ahc_noalloc(plan, t_ptr: int, ef_ptr: int, eta: float, kT: float, sigma_ptr: int,
                     status_ptr: int, stream: int) -> int:
    return lib().kubo_ahc_noalloc(plan, t_ptr, ef_ptr, float(eta), float(kT), sigma_ptr,
                                  status_ptr, stream)


def kubo_plan_device_status(plan, ws_ptr: int, stream: int) -> int:
    return lib().kubo_plan_device_status(plan, ws_ptr, stream)


def kubo_plan_destroy(plan) -> None:
    lib().kubo_plan_destroy(plan)


def kubo_plan_info(plan):
    tk = ctypes.c_int64()
    nm = ctypes.c_int32()
    st = lib().kubo_plan_info(plan, ctypes.byref(tk), ctypes.byref(nm))
    return st, tk.value, nm.value


def kubo_plan_kernel_time(plan, which: int, reset: bool = False):
    """(status, total_ms, launches, k_points) of timing slot `which` (0 forward, 1 backward,
    2 tensor, 3 Green's-function form, 4 the large-n reduction kernel)."""
    ms = ctypes.c_double()
    nl = ctypes.c_int64()
    kp = ctypes.c_int64()
    st = lib().kubo_plan_kernel_time(plan, int(which), ctypes.byref(ms), ctypes.byref(nl),
                                     ctypes.byref(kp), 1 if reset else 0)
    return st, ms.value, nl.value, kp.value


# ---------------------------------------------------------------------------
# Plan object
# ---------------------------------------------------------------------------


def make_desc(n_orb: int, R: np.ndarray, grid: Sequence[int], k_begin: int = 0,
              k_count: int = -1):
    """A kubo_model_desc plus the array that keeps its R pointer alive."""
    R = np.ascontiguousarray(R, dtype=np.int32)
    d = kubo_model_desc()
    d.n_orb = int(n_orb)
    d.n_R = int(R.shape[0])
    d.R = R.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.grid = (ctypes.c_int32 * 3)(*[int(g) for g in grid])
    d.k_begin = int(k_begin)
    d.k_count = int(k_count)
    return d, R


class Plan:
    """A kubo plan for one or more models, with its own device workspace."""

    def __init__(self, models: Iterable, grid=None, n_fermi: int = 1, flags: int = 0,
                 tiles="auto", slabs: Optional[Sequence[tuple]] = None, device: str = "cuda"):
        """models: objects with .n and .R (e.g. synth.TBModel); grid: one grid or one per model;
        slabs: optional (k_begin, k_count) per model; tiles: (n_orb, threads, k_block) tuples,
        None for the built-in defaults, or "auto" for the autotuner's cache (if any)."""
        models = list(models)
        if isinstance(tiles, str) and tiles == "auto":
            from . import autotune

            tiles = autotune.lookup([m.n for m in models]) or None
        grids = [grid] * len(models) if (grid is None or np.ndim(grid[0]) == 0) else list(grid)
        keep = []
        descs = []
        for i, m in enumerate(models):
            kb, kc = (0, -1) if slabs is None else slabs[i]
            d, R = make_desc(m.n, m.R, grids[i], kb, kc)
            keep.append(R)
            descs.append(d)
        tl = None
        if tiles:
            tl = []
            for (n, th, kbk) in tiles:
                t = kubo_tile()
                t.n_orb, t.threads, t.k_block, t.reserved = int(n), int(th), int(kbk), 0
                tl.append(t)
        st, h, wsb = kubo_plan(descs, n_fermi, flags, tl)
        if st != KUBO_OK:
            raise KuboError(st, "kubo_plan")
        self.handle = h
        self.ws_bytes = wsb
        self.n_models = len(models)
        self.n_fermi = int(n_fermi)
        self.sizes = [(m.n, m.n_R) for m in models]
        self.t_elems = sum(n * n * nr for n, nr in self.sizes)
        self.device = device
        self._ws = None
        self._ws_stream = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            kubo_plan_destroy(h)
            self.handle = None

    @property
    def total_k(self) -> int:
        return kubo_plan_info(self.handle)[1]

    def workspace(self):
        """The plan's device workspace, allocated on first use on the current stream.
        Use on another stream is recorded with the caching allocator, so the memory
        is not handed out again before the work queued there has finished."""
        import torch

        if self._ws is None:
            self._ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=self.device)
            self._ws_stream = torch.cuda.current_stream(self._ws.device)
        else:
            cur = torch.cuda.current_stream(self._ws.device)
            if cur != self._ws_stream:
                self._ws.record_stream(cur)
        return self._ws

    def _check_t(self, t):
        import torch

        if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("t must be a contiguous complex128 CUDA tensor")
        if t.numel() != self.t_elems:
            raise ValueError(f"t has {t.numel()} elements, the plan expects {self.t_elems}")

    def _check_f(self, x, name):
        import torch

        if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
        if x.numel() != self.n_models * self.n_fermi:
            raise ValueError(f"{name} must have n_models * n_fermi elements")

    def forward(self, t, e_fermi, eta: float, kT: float, out=None):
        """sigma [n_models, n_fermi] (float64, on the device), enqueued on the current stream."""
        import torch

        self._check_t(t)
        self._check_f(e_fermi, "e_fermi")
        if out is None:
            out = torch.empty(self.n_models, self.n_fermi, dtype=torch.float64, device=t.device)
        ws = self.workspace()
        stream = torch.cuda.current_stream(t.device).cuda_stream
        st = kubo_ahc(self.handle, t.data_ptr(), e_fermi.data_ptr(), eta, kT, out.data_ptr(),
                      ws.data_ptr(), self.ws_bytes, stream)
        if st != KUBO_OK:
            raise KuboError(st, "kubo_ahc")
        return out

    def tensor(self, t, e_fermi, eta: float, kT: float, spin=None, out=None):
        """[n_models, 4, n_fermi] float64: sigma_xy, sigma_yz, sigma_zx and the spin Hall
        conductivity (spin: float64 CUDA tensor with one s_z value per orbital of every
        model, or None), enqueued on the current stream.  Needs a KUBO_F_TENSOR plan."""
        import torch

        self._check_t(t)
        self._check_f(e_fermi, "e_fermi")
        sp = 0
        if spin is not None:
            if spin.dtype != torch.float64 or not spin.is_cuda or not spin.is_contiguous():
                raise ValueError("spin must be a contiguous float64 CUDA tensor")
            if spin.numel() != sum(n for n, _ in self.sizes):
                raise ValueError("spin needs one value per orbital of every model")
            sp = spin.data_ptr()
        if out is None:
            out = torch.empty(self.n_models, 4, self.n_fermi, dtype=torch.float64,
                              device=t.device)
        ws = self.workspace()
        stream = torch.cuda.current_stream(t.device).cuda_stream
        st = kubo_ahc_tensor(self.handle, t.data_ptr(), e_fermi.data_ptr(), eta, kT, sp,
                             out.data_ptr(), ws.data_ptr(), self.ws_bytes, stream)
        if st != KUBO_OK:
            raise KuboError(st, "kubo_ahc_tensor")
        return out

    def gf(self, t, e_fermi, gamma: float, omega, weight, out=None):
        """[n_models, n_fermi] float64: the Green's-function form of sigma_xy with scattering
        rate gamma, the w-integral over (0, inf) given by the nodes `omega` and weights
        `weight` (contiguous float64 CUDA tensors of one length); models with n <= 32."""
        import torch

        self._check_t(t)
        self._check_f(e_fermi, "e_fermi")
        for x, name in ((omega, "omega"), (weight, "weight")):
            if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
        if omega.numel() != weight.numel():
            raise ValueError("omega and weight need the same length")
        if out is None:
            out = torch.empty(self.n_models, self.n_fermi, dtype=torch.float64, device=t.device)
        ws = self.workspace()
        stream = torch.cuda.current_stream(t.device).cuda_stream
        st = kubo_ahc_gf(self.handle, t.data_ptr(), e_fermi.data_ptr(), gamma, omega.data_ptr(),
                         weight.data_ptr(), omega.numel(), out.data_ptr(), ws.data_ptr(),
                         self.ws_bytes, stream)
        if st != KUBO_OK:
            raise KuboError(st, "kubo_ahc_gf")
        return out

    def backward(self, t, e_fermi, eta: float, kT: float, sigma_bar, out=None):
        """dL/dRe t + i dL/dIm t for L = sum sigma_bar * sigma (complex128, like t)."""
        import torch

        self._check_t(t)
        self._check_f(e_fermi, "e_fermi")
        self._check_f(sigma_bar, "sigma_bar")
        if out is None:
            out = torch.empty_like(t)
        ws = self.workspace()
        stream = torch.cuda.current_stream(t.device).cuda_stream
        st = kubo_ahc_backward(self.handle, t.data_ptr(), e_fermi.data_ptr(), eta, kT,
                               sigma_bar.data_ptr(), out.data_ptr(), ws.data_ptr(), self.ws_bytes,
                               stream)
        if st != KUBO_OK:
            raise KuboError(st, "kubo_ahc_backward")
        return out

    def kernel_time(self, which: int = 0, reset: bool = False):
        """(total_ms, launches, k_points) recorded under KUBO_F_TIMING (which: 0 forward,
        1 backward, 2 tensor, 3 Green's-function form, 4 the large-n reduction kernel)."""
        st, ms, nl, kp = kubo_plan_kernel_time(self.handle, which, reset)
        if st != KUBO_OK:
            raise KuboError(st, "kubo_plan_kernel_time")
        return ms, nl, kp

    def device_status(self) -> int:
        import torch

        stream = torch.cuda.current_stream().cuda_stream
        return kubo_plan_device_status(self.handle, self.workspace().data_ptr(), stream)


# ---------------------------------------------------------------------------
# autograd front end
# ---------------------------------------------------------------------------


def _autograd_fn():
    import torch

    class KuboAHC(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t, plan, e_fermi, eta, kT):
            ctx.plan, ctx.eta, ctx.kT = plan, eta, kT
            ctx.save_for_backward(t, e_fermi)
            return plan.forward(t.contiguous(), e_fermi.contiguous(), eta, kT)

        @staticmethod
        def backward(ctx, gsig):
            t, e_fermi = ctx.saved_tensors
            g = ctx.plan.backward(t.contiguous(), e_fermi.contiguous(), ctx.eta, ctx.kT,
                                  gsig.contiguous().to(torch.float64))
            return g, None, None, None, None

    return KuboAHC


_FN = None


def ahc(t, plan: Plan, e_fermi, eta: float, kT: float):
    """sigma_xy [n_models, n_fermi], differentiable in t (complex128, models concatenated)."""
    global _FN
    if _FN is None:
        _FN = _autograd_fn()
    return _FN.apply(t, plan, e_fermi, eta, kT)


def to_device_t(models: List, device="cuda"):
    """Concatenate the models' t arrays into one complex128 device tensor."""
    import torch

    flat = np.concatenate([np.ascontiguousarray(m.t, np.complex128).reshape(-1) for m in models])
    return torch.from_numpy(flat).to(device)
