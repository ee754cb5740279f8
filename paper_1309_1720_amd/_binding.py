"""ctypes binding of librd.so (include/rd.h).

Argument marshalling only: tensors are passed as device pointers, the
workspace is a byte tensor from torch's caching allocator, work goes on
torch's current HIP stream.  Every step of the computation runs in the HIP
library; there is no CPU fallback -- a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# RD_LIBRARY selects another build of the same library (the host-sanitised
# one of build.build_asan, for CPU-only ABI checks).
LIB_PATH = os.environ.get("RD_LIBRARY") or os.path.join(_HERE, "librd.so")
ABI_VERSION = 2

MODELS = {"diffusion": 0, "barkley": 1, "fk": 2, "bocf": 3, "fhn": 4}
SCHEMES = {"euler": 1, "heun": 2, "rk4": 4, "rush_larsen": 5, "implicit_euler": 6}
BCS = {"noflux": 0, "periodic": 1}
STENCILS = {"lap5": 5, "lap9": 9, "lap9_aniso": 10, "lap7": 7, "lap19": 19, "lap27": 27}
STENCILS_3D = ("lap7", "lap19", "lap27")
OPS = {"step": 0, "jvp": 1, "vjp": 2, "batched": 3, "batched_jvp": 4}
N_FIELDS = {"diffusion": 1, "barkley": 2, "fk": 3, "bocf": 4, "fhn": 2}

STATUS = {0: "RD_OK", -1: "RD_EINVAL", -2: "RD_EUNSUPPORTED", -3: "RD_EWORKSPACE", -4: "RD_EHIP",
          -5: "RD_ENONFINITE"}


class RDError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS.get(code, code)}: {message}")
        self.code = code


class _CProblem(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("model", C.c_int32), ("scheme", C.c_int32),
        ("stencil", C.c_int32), ("bc", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
        ("dx", C.c_double), ("dt", C.c_double), ("nsteps", C.c_int64),
        ("D_par", C.c_double), ("D_perp", C.c_double), ("theta0", C.c_double),
        ("theta1", C.c_double), ("step_k", C.c_double),
        ("params", C.POINTER(C.c_double)), ("nparams", C.c_int32),
        ("checkpoint_every", C.c_int32), ("nz", C.c_int32),
    ]


_PTR = C.c_void_p
_DPP = C.POINTER(C.c_void_p)
_lib = None


def lib() -> C.CDLL:
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run "
                               "`python -m paper_1309_1720_amd.build`")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(_CProblem)
        sig = {
            "rd_abi_version": ([], C.c_int),
            "rd_n_fields": ([C.c_int32], C.c_int),
            "rd_n_params": ([C.c_int32], C.c_int),
            "rd_checkpoint_count": ([P, C.POINTER(C.c_int64)], C.c_int),
            "rd_workspace_bytes": ([P, C.c_int32, C.POINTER(C.c_size_t)], C.c_int),
            "rd_step": ([P, _DPP, _PTR, _PTR, C.c_size_t, _PTR], C.c_int),
            "rd_step_noalloc": ([P, _DPP, _PTR, _PTR], C.c_int),
            "rd_jvp": ([P, _DPP, _DPP, _PTR, C.c_size_t, _PTR], C.c_int),
            "rd_vjp": ([P, _PTR, _DPP, _PTR, C.c_size_t, _PTR], C.c_int),
            "rd_step_batched_workspace_bytes": ([P, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)], C.c_int),
            "rd_step_batched": ([P, C.c_int32, C.POINTER(_DPP), C.POINTER(_DPP), _PTR, C.c_size_t, _PTR], C.c_int),
            "rd_set_tile_rows": ([C.c_int32], C.c_int),
            "rd_set_autotune": ([C.c_int32], C.c_int),
            "rd_set_fused_adjoint": ([C.c_int32], C.c_int),
            "rd_set_check_finite": ([C.c_int32], C.c_int),
            "rd_get_tile_rows": ([P, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
            "rd_set_kernel_variant": ([C.c_int32], C.c_int),
            "rd_get_plan": ([P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
            "rd_set_steps_per_launch": ([C.c_int32], C.c_int),
            "rd_vec_gram_workspace_bytes": ([C.c_int32, C.POINTER(C.c_size_t)], C.c_int),
            "rd_vec_gram": ([C.POINTER(_PTR), C.c_int32, _PTR, C.c_int64, _PTR, _PTR, C.c_size_t, _PTR], C.c_int),
            "rd_vec_lincomb": ([_PTR, C.c_double, C.POINTER(_PTR), C.POINTER(C.c_double), C.c_int32, C.c_int64,
                                _PTR], C.c_int),
            "rd_get_steps_per_launch": ([P, C.POINTER(C.c_int32)], C.c_int),
            "rd_last_error": ([], C.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        if L.rd_abi_version() != ABI_VERSION:
            raise RuntimeError(f"librd.so ABI {L.rd_abi_version()} != binding ABI {ABI_VERSION}")
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise RDError(rc, lib().rd_last_error().decode())
    return rc


@dataclass
class Problem:
    """One integration problem; mirrors ``rd_problem`` of include/rd.h."""
    model: str
    scheme: str
    stencil: str
    nx: int
    ny: int
    dx: float
    dt: float
    nsteps: int = 1
    D_par: float = 1.0
    D_perp: float | None = None
    theta0: float = 0.0
    theta1: float = 0.0
    step_k: float = 28.4
    params: tuple = field(default_factory=tuple)
    checkpoint_every: int = 0
    bc: str = "noflux"
    nz: int = 1

    @property
    def nfields(self) -> int:
        return N_FIELDS[self.model]

    @property
    def shape(self) -> tuple:
        """Shape of one field tensor: (nz, ny, nx) for the 3-D stencils, else (ny, nx)."""
        return (self.nz, self.ny, self.nx) if self.stencil in STENCILS_3D else (self.ny, self.nx)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    @classmethod
    def from_workload(cls, w: dict, params, **overrides) -> "Problem":
        keys = ("model", "scheme", "stencil", "nx", "ny", "dx", "dt", "nsteps", "D_par",
                "D_perp", "theta0", "theta1", "step_k", "checkpoint_every", "bc", "nz")
        kw = {k: w[k] for k in keys if k in w}
        kw["params"] = tuple(float(x) for x in params)
        kw.update(overrides)
        return cls(**kw)

    def to_c(self):
        """(_CProblem, params buffer) -- keep the buffer alive during the call."""
        n = len(self.params)
        buf = (C.c_double * max(n, 1))(*[float(x) for x in self.params])
        cp = _CProblem(
            abi_version=ABI_VERSION, model=MODELS[self.model], scheme=SCHEMES[self.scheme],
            stencil=STENCILS[self.stencil], bc=BCS[self.bc], nx=int(self.nx), ny=int(self.ny),
            dx=float(self.dx), dt=float(self.dt), nsteps=int(self.nsteps),
            D_par=float(self.D_par),
            D_perp=float(self.D_par if self.D_perp is None else self.D_perp),
            theta0=float(self.theta0), theta1=float(self.theta1), step_k=float(self.step_k),
            params=C.cast(buf, C.POINTER(C.c_double)), nparams=n,
            checkpoint_every=int(self.checkpoint_every), nz=int(self.nz))
        return cp, buf


def _ptrs(tensors, prob: Problem, what: str):
    if len(tensors) != prob.nfields:
        raise ValueError(f"{what}: {prob.model} has {prob.nfields} fields, got {len(tensors)}")
    for t in tensors:
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ValueError(f"{what}: expected HIP device tensors")
        if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != prob.shape:
            raise ValueError(f"{what}: expected contiguous float64 tensors of shape "
                             f"{prob.shape}, got {t.dtype} {tuple(t.shape)}")
    arr = (C.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])
    return arr


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


# Eager calls: one workspace buffer per (device, stream), grown on demand and
# reused by later eager calls on that stream (stream order keeps consecutive
# calls apart).  Calls made while the stream is being captured into a HIP
# graph never touch that cache: each gets a buffer of its own, which the graph
# replays write into, kept alive here until release_workspaces().  So growing
# the eager buffer never frees memory a graph holds, and eager calls never
# share a buffer with a graph replayed on another stream.
_WORKSPACES: dict = {}
_CAPTURED: list = []


def _workspace(nbytes: int, device):
    if nbytes == 0:
        return None, 0
    dev = torch.device(device)
    if torch.cuda.is_current_stream_capturing():
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        _CAPTURED.append(ws)
        return ws, ws.data_ptr()
    key = (dev.index if dev.index is not None else torch.cuda.current_device(), _stream(dev))
    ws = _WORKSPACES.get(key)
    if ws is None or ws.numel() < nbytes:
        _WORKSPACES.pop(key, None)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        _WORKSPACES[key] = ws
    return ws, ws.data_ptr()


def release_workspaces() -> None:
    """Drop the cached workspace buffers (returned to torch's allocator),
    including those of captured calls: replaying a graph captured before this
    call is then no longer allowed."""
    _WORKSPACES.clear()
    _CAPTURED.clear()


def n_fields(model: str) -> int:
    return _check(lib().rd_n_fields(MODELS[model]))


def n_params(model: str) -> int:
    return _check(lib().rd_n_params(MODELS[model]))


def workspace_bytes(prob, op: str = "step") -> int:
    """rd_workspace_bytes: ``prob`` is one Problem for "step", "jvp", "vjp",
    and the list of a batch's problems for "batched" and "batched_jvp"."""
    if op in ("batched", "batched_jvp"):
        probs = list(prob)
        cps, bufs = zip(*[p.to_c() for p in probs])
        arr = (_CProblem * len(probs))(*cps)
        out = C.c_size_t(len(probs))  # nbatch on entry
        _check(lib().rd_workspace_bytes(arr, OPS[op], C.byref(out)))
        del bufs
        return out.value
    cp, _buf = prob.to_c()
    out = C.c_size_t(0)
    _check(lib().rd_workspace_bytes(C.byref(cp), OPS[op], C.byref(out)))
    return out.value


def checkpoint_count(prob: Problem) -> int:
    cp, _buf = prob.to_c()
    out = C.c_int64(0)
    _check(lib().rd_checkpoint_count(C.byref(cp), C.byref(out)))
    return out.value


def set_tile_rows(rows: int) -> None:
    """Rows per wavefront band for later calls (<= 0: automatic)."""
    _check(lib().rd_set_tile_rows(int(rows)))


def get_tile_rows(prob: Problem, op: str = "step") -> int:
    """Band height the library uses for ``op`` on ``prob`` (see rd_get_tile_rows)."""
    cp, _buf = prob.to_c()
    out = C.c_int32(0)
    _check(lib().rd_get_tile_rows(C.byref(cp), OPS[op], C.byref(out)))
    return out.value


VARIANTS = {"sweep": 0, "pipe": 1}


def set_kernel_variant(variant) -> None:
    """Fix the fused-step kernel ("sweep", "pipe") or None for the autotuner."""
    _check(lib().rd_set_kernel_variant(-1 if variant is None else VARIANTS[variant]))


def get_plan(prob: Problem, op: str = "step"):
    """(kernel variant name, rows per band) used for ``op`` on ``prob``."""
    cp, _buf = prob.to_c()
    v, r = C.c_int32(0), C.c_int32(0)
    _check(lib().rd_get_plan(C.byref(cp), OPS[op], C.byref(v), C.byref(r)))
    return {0: "sweep", 1: "pipe"}[v.value], r.value


def set_steps_per_launch(steps) -> None:
    """Fix the steps one rd_step launch advances (1, 2, 4, 8; capped by the
    model's maximum) or None for the autotuner."""
    _check(lib().rd_set_steps_per_launch(-1 if steps is None else int(steps)))


def get_steps_per_launch(prob: Problem) -> int:
    """Steps per launch rd_step uses for ``prob``."""
    cp, _buf = prob.to_c()
    k = C.c_int32(0)
    _check(lib().rd_get_steps_per_launch(C.byref(cp), C.byref(k)))
    return k.value


def _vec_check(t, n, what):
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == n):
        raise ValueError(f"{what}: need a contiguous float64 device tensor of {n} elements")


def vec_gram(xs, w: torch.Tensor) -> torch.Tensor:
    """Device tensor of <x_k, w> for the flat float64 device tensors ``xs``."""
    n = w.numel()
    _vec_check(w, n, "w")
    for x in xs:
        _vec_check(x, n, "x")
    m = len(xs)
    out = torch.empty(m, dtype=torch.float64, device=w.device)
    need = C.c_size_t(0)
    _check(lib().rd_vec_gram_workspace_bytes(m, C.byref(need)))
    ws, wsp = _workspace(need.value, w.device)
    xp = (_PTR * m)(*[x.data_ptr() for x in xs])
    _check(lib().rd_vec_gram(xp, m, w.data_ptr(), n, out.data_ptr(), wsp, need.value, _stream(w.device)))
    return out


def vec_lincomb(y: torch.Tensor, beta: float, xs=(), coef=()) -> torch.Tensor:
    """y <- beta y + sum_k coef[k] xs[k] in place (flat float64 device tensors)."""
    n = y.numel()
    _vec_check(y, n, "y")
    for x in xs:
        _vec_check(x, n, "x")
    m = len(xs)
    if len(coef) != m:
        raise ValueError("one coefficient per vector")
    xp = (_PTR * max(m, 1))(*[x.data_ptr() for x in xs])
    cp = (C.c_double * max(m, 1))(*[float(c) for c in coef])
    _check(lib().rd_vec_lincomb(y.data_ptr(), float(beta), xp, cp, m, n, _stream(y.device)))
    return y


def set_autotune(enable: bool) -> None:
    """Enable or disable the band-height autotuner (see rd_set_autotune)."""
    _check(lib().rd_set_autotune(1 if enable else 0))


def set_fused_adjoint(enable: bool) -> None:
    """Whether rd_vjp recomputes stage inputs inside its adjoint kernel where
    the model allows (see rd_set_fused_adjoint); results are bit-identical."""
    _check(lib().rd_set_fused_adjoint(1 if enable else 0))


def set_check_finite(enable: bool) -> None:
    """Enable or disable the NaN/infinity check of every call's result (see
    rd_set_check_finite); the cached workspaces are dropped because the
    required sizes change."""
    _check(lib().rd_set_check_finite(1 if enable else 0))
    release_workspaces()


def step(prob: Problem, fields, checkpoints: torch.Tensor | None = None):
    """Advance ``fields`` (list of float64 device tensors of shape ``prob.shape``) in place by
    ``prob.nsteps`` steps; optionally store checkpoints (see rd_step)."""
    L = lib()
    f = _ptrs(fields, prob, "fields")
    dev = fields[0].device
    cp, _buf = prob.to_c()
    ckpt = 0
    if checkpoints is not None:
        need = checkpoint_count(prob) * prob.nfields * prob.cells
        if (not checkpoints.is_cuda or checkpoints.dtype != torch.float64
                or not checkpoints.is_contiguous() or checkpoints.numel() < need):
            raise ValueError(f"checkpoints: need a contiguous float64 device tensor of >= {need} elements")
        ckpt = checkpoints.data_ptr()
    ws, wsp = _workspace(workspace_bytes(prob, "step"), dev)
    _check(L.rd_step(C.byref(cp), f, ckpt, wsp, ws.numel() if ws is not None else 0, _stream(dev)))
    return fields


def step_noalloc(prob: Problem, fields, checkpoints: torch.Tensor | None = None):
    """rd_step_noalloc: rd_step with the library's own per-GPU scratch (no
    workspace, nothing allocated); raises RDError(RD_EWORKSPACE) for grids
    beyond its size."""
    L = lib()
    f = _ptrs(fields, prob, "fields")
    dev = fields[0].device
    cp, _buf = prob.to_c()
    ckpt = 0
    if checkpoints is not None:
        need = checkpoint_count(prob) * prob.nfields * prob.cells
        if (not checkpoints.is_cuda or checkpoints.dtype != torch.float64
                or not checkpoints.is_contiguous() or checkpoints.numel() < need):
            raise ValueError(f"checkpoints: need a contiguous float64 device tensor of >= {need} elements")
        ckpt = checkpoints.data_ptr()
    _check(L.rd_step_noalloc(C.byref(cp), f, ckpt, _stream(dev)))
    return fields


def jvp(prob: Problem, fields, tangents):
    """Advance state and tangent together in place (rd_jvp)."""
    L = lib()
    f = _ptrs(fields, prob, "fields")
    t = _ptrs(tangents, prob, "tangents")
    dev = fields[0].device
    cp, _buf = prob.to_c()
    ws, wsp = _workspace(workspace_bytes(prob, "jvp"), dev)
    _check(L.rd_jvp(C.byref(cp), f, t, wsp, ws.numel() if ws is not None else 0, _stream(dev)))
    return fields, tangents


def vjp(prob: Problem, checkpoints: torch.Tensor, cotangents):
    """lambda(T) -> lambda(0) in place from rd_step's checkpoints (rd_vjp)."""
    L = lib()
    c = _ptrs(cotangents, prob, "cotangents")
    dev = cotangents[0].device
    cp, _buf = prob.to_c()
    if not checkpoints.is_cuda or checkpoints.dtype != torch.float64 or not checkpoints.is_contiguous():
        raise ValueError("checkpoints: expected a contiguous float64 device tensor")
    need = checkpoint_count(prob) * prob.nfields * prob.cells
    if checkpoints.numel() < need:
        raise ValueError(f"checkpoints: need >= {need} elements, got {checkpoints.numel()}")
    ws, wsp = _workspace(workspace_bytes(prob, "vjp"), dev)
    _check(L.rd_vjp(C.byref(cp), checkpoints.data_ptr(), c, wsp,
                    ws.numel() if ws is not None else 0, _stream(dev)))
    return cotangents


def step_batched(probs, fields_list, tangents_list=None):
    """Advance several problems together (rd_step_batched)."""
    L = lib()
    n = len(probs)
    if len(fields_list) != n or (tangents_list is not None and len(tangents_list) != n):
        raise ValueError("one field list (and tangent list) per problem")
    cps, bufs = zip(*[p.to_c() for p in probs])
    arr = (_CProblem * n)(*cps)
    fptrs = [_ptrs(fl, p, "fields") for fl, p in zip(fields_list, probs)]
    fpp = (_DPP * n)(*[C.cast(a, _DPP) for a in fptrs])
    tpp = None
    if tangents_list is not None:
        tptrs = [_ptrs(tl, p, "tangents") for tl, p in zip(tangents_list, probs)]
        tpp = (_DPP * n)(*[C.cast(a, _DPP) for a in tptrs])
    dev = fields_list[0][0].device
    need = C.c_size_t(n)  # nbatch on entry
    _check(L.rd_workspace_bytes(arr, OPS["batched" if tangents_list is None else "batched_jvp"], C.byref(need)))
    ws, wsp = _workspace(need.value, dev)
    _check(L.rd_step_batched(arr, n, fpp, tpp, wsp, need.value, _stream(dev)))
    del bufs
    return fields_list
