"""ctypes binding of libjko.so (argument marshalling only).

Every computation happens in the HIP library; this module checks dtypes,
devices and contiguity, allocates the caller-owned workspace with torch, and
passes raw device pointers and the current HIP stream.  There is no CPU
fallback: if the library is not built, or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libjko.so")

# status codes (include/jko.h)
JKO_OK = 0
JKO_ERR_INVALID = -1
JKO_ERR_WORKSPACE = -2
JKO_ERR_HIP = -3
JKO_ERR_NONFINITE = -4
JKO_ERR_INFEASIBLE = -5

PRECISIONS = {"fp32": 0, "split_bf16": 1}
ENERGY_KINDS = {"zero": 0, "congestion": 1, "porous": 2, "entropy": 3, "binary_congestion": 4, "gen_entropy": 5,
                "attraction": 6}
OP_GIBBS, OP_STEP, OP_FLOW, OP_BACKWARD, OP_ATTRACTION_STEP, OP_ATTRACTION_FLOW = 0, 1, 2, 3, 4, 5
FLAG_NO_RESIDENT = 1   # jko_flags: keep one launch per Gibbs application
FLAG_AXIS_PASSES = 2   # jko_flags: 3D applications as three axis passes
FLAG_ABSORB_ON_A = 4   # jko_flags: the absorption switch watches max|log a| alone


class JKOError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"jko status {status}: {message}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int32 * 3)]


class EnergyC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("w", ctypes.c_void_p), ("kappa", ctypes.c_void_p),
                ("kappa_scalar", ctypes.c_float), ("coef", ctypes.c_void_p),
                ("coef_scalar", ctypes.c_float), ("m", ctypes.c_float),
                ("density_scale", ctypes.c_float), ("newton_steps", ctypes.c_int32),
                ("m_field", ctypes.c_void_p), ("target", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("tau", ctypes.c_double), ("tol_l1", ctypes.c_double),
                ("max_iters", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("absorb_threshold", ctypes.c_double)]


class HeatDomain(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int32), ("n1", ctypes.c_int32), ("mask", ctypes.c_void_p), ("L", ctypes.c_int32),
                ("per_product", ctypes.c_int32)]


# Version of the C ABI this binding marshals for (jko_version()).
ABI_VERSION = 2

# Doubles in jko_step's device statistics record (JKO_STATS_DEV_DOUBLES).
STATS_DEV_DOUBLES = 8


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("absorptions", ctypes.c_int32),
                ("stop_reason", ctypes.c_int32), ("status", ctypes.c_int32),
                ("marginal_l1", ctypes.c_double), ("mass", ctypes.c_double),
                ("max_abs_log_a", ctypes.c_double), ("max_abs_log_b", ctypes.c_double)]

    def as_dict(self) -> dict:
        return dict(iters=self.iters, absorptions=self.absorptions,
                    stop="tol" if self.stop_reason == 0 else "cap", status=self.status,
                    marginal_l1=self.marginal_l1, mass=self.mass,
                    max_abs_log_a=self.max_abs_log_a, max_abs_log_b=self.max_abs_log_b)


_lib = None


def load(path: str = LIB_PATH):
    """Load libjko.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1502_06216_amd.build`")
    lib = ctypes.CDLL(path)
    vp, sz, i32, f64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double
    G, E, P, S = ctypes.POINTER(Grid), ctypes.POINTER(EnergyC), ctypes.POINTER(Params), ctypes.POINTER(Stats)
    lib.jko_workspace_bytes.argtypes = [G, P, i32, i32]
    lib.jko_workspace_bytes.restype = sz
    lib.jko_gibbs_apply.argtypes = [G, f64, i32, vp, vp, vp, sz, vp]
    lib.jko_gibbs_apply.restype = i32
    lib.jko_step.argtypes = [G, E, P, vp, vp, S, vp, vp, sz, vp]
    lib.jko_step.restype = i32
    lib.jko_step_static.argtypes = [G, E, P, vp, vp, S, vp]
    lib.jko_step_static.restype = i32
    lib.jko_flow.argtypes = [G, E, P, i32, vp, vp, vp, S, vp, sz, vp]
    lib.jko_flow.restype = i32
    lib.jko_backward.argtypes = [G, E, P, i32, ctypes.POINTER(i32), vp, vp, vp, vp, vp, sz, vp]
    lib.jko_backward.restype = i32
    lib.jko_time_iteration.argtypes = [G, E, P, vp, i32, ctypes.POINTER(f64), ctypes.POINTER(i32), vp, sz, vp]
    lib.jko_time_iteration.restype = i32
    H = ctypes.POINTER(HeatDomain)
    lib.jko_heat_workspace_bytes.argtypes = [H]
    lib.jko_heat_workspace_bytes.restype = sz
    lib.jko_heat_build.argtypes = [H, f64, vp, sz, vp]
    lib.jko_heat_build.restype = i32
    lib.jko_heat_apply.argtypes = [H, vp, vp, vp, sz, vp]
    lib.jko_heat_apply.restype = i32
    lib.jko_heat_flow.argtypes = [H, E, P, i32, vp, vp, S, vp, sz, vp]
    lib.jko_heat_flow.restype = i32
    lib.jko_status_string.argtypes = [i32]
    lib.jko_status_string.restype = ctypes.c_char_p
    lib.jko_last_error.argtypes = []
    lib.jko_last_error.restype = ctypes.c_char_p
    lib.jko_version.argtypes = []
    lib.jko_version.restype = i32
    if lib.jko_version() != ABI_VERSION:
        raise RuntimeError(f"{path} has ABI version {lib.jko_version()}, this binding expects {ABI_VERSION}: "
                           "rebuild it with `python -m paper_1502_06216_amd.build`")
    _lib = lib
    return lib


def _check(status: int):
    if status != JKO_OK:
        lib = load()
        msg = lib.jko_last_error().decode() or lib.jko_status_string(status).decode()
        raise JKOError(status, msg)


def make_grid(shape: Sequence[int]) -> Grid:
    g = Grid()
    g.ndim = len(shape)
    for k in range(3):
        g.n[k] = int(shape[k]) if k < len(shape) else 1
    return g


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _field(t: Optional[torch.Tensor], shape, name: str) -> Optional[torch.Tensor]:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise TypeError(f"{name} must be a contiguous float32 tensor of shape {tuple(shape)}")
    return t


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


@dataclass
class EnergySpec:
    """Energy f of the JKO step (Section 4 of the paper); fields are device
    float32 tensors of the grid's shape or None for the scalar defaults.
    kind: "zero", "congestion", "binary_congestion" (the non-convex {0, kappa}
    constraint of Section 4.5; finite kappa, no backward), "porous", "entropy",
    "gen_entropy" (the generalised entropies of Section 4.4 with per-cell
    weights coef and exponents m_field >= 1), "attraction" (Wasserstein
    attraction towards the density target, with capacity kappa, Section 5.2;
    1D/2D grids, plain domain, no backward)."""
    kind: str = "zero"
    w: Optional[torch.Tensor] = None
    kappa: Optional[torch.Tensor] = None
    kappa_scalar: float = math.inf
    coef: Optional[torch.Tensor] = None
    coef_scalar: float = 1.0
    m: float = 2.0
    density_scale: float = 1.0
    newton_steps: int = 8
    m_field: Optional[torch.Tensor] = None
    target: Optional[torch.Tensor] = None

    def to_c(self, shape) -> EnergyC:
        e = EnergyC()
        e.kind = ENERGY_KINDS[self.kind]
        e.w = _ptr(_field(self.w, shape, "w"))
        e.kappa = _ptr(_field(self.kappa, shape, "kappa"))
        e.kappa_scalar = float(self.kappa_scalar)
        e.coef = _ptr(_field(self.coef, shape, "coef"))
        e.coef_scalar = float(self.coef_scalar)
        e.m = float(self.m)
        e.density_scale = float(self.density_scale)
        e.newton_steps = int(self.newton_steps)
        e.m_field = _ptr(_field(self.m_field, shape, "m_field"))
        e.target = _ptr(_field(self.target, shape, "target"))
        return e


def make_params(gamma, tau, max_iters=300, tol=0.0, check_every=10, precision="fp32",
                absorb_threshold=math.inf, resident=True, planes=True, absorb_on_a=False) -> Params:
    p = Params()
    p.gamma = float(gamma)
    p.tau = float(tau)
    p.tol_l1 = float(tol)
    p.max_iters = int(max_iters)
    p.check_every = int(check_every)
    p.precision = PRECISIONS[precision]
    p.flags = ((0 if resident else FLAG_NO_RESIDENT) | (0 if planes else FLAG_AXIS_PASSES)
               | (FLAG_ABSORB_ON_A if absorb_on_a else 0))
    p.absorb_threshold = float(absorb_threshold)
    return p


def workspace_bytes(shape, op: int, n: int = 0, params: Optional[Params] = None) -> int:
    lib = load()
    g = make_grid(shape)
    return int(lib.jko_workspace_bytes(ctypes.byref(g), ctypes.byref(params) if params else None, op, n))


def gibbs_apply(x: torch.Tensor, gamma: float, precision: str = "fp32",
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = xi x for a float32 field on the GPU (xi = exp(-|x_i - x_j|^2/gamma))."""
    lib = load()
    shape = tuple(x.shape)
    _field(x, shape, "x")
    y = torch.empty_like(x) if out is None else _field(out, shape, "out")
    g = make_grid(shape)
    nb = lib.jko_workspace_bytes(ctypes.byref(g), None, OP_GIBBS, 0)
    ws = _workspace(nb, x.device)
    _check(lib.jko_gibbs_apply(ctypes.byref(g), float(gamma), PRECISIONS[precision], _ptr(x), _ptr(y),
                               _ptr(ws), ws.numel(), _stream(x.device)))
    return y


def step(p: torch.Tensor, energy: EnergySpec, gamma: float, tau: float, max_iters: int = 300,
         tol: float = 0.0, check_every: int = 10, precision: str = "fp32",
         absorb_threshold: float = math.inf, out: Optional[torch.Tensor] = None,
         with_stats: bool = True, resident: bool = True, planes: bool = True, absorb_on_a: bool = False,
         stats_dev: Optional[torch.Tensor] = None):
    """One JKO step p -> argmin_p' W_gamma(p', p) + tau f(p').  Returns
    (p_next, stats dict or None).  resident=False keeps one launch per Gibbs
    application (per pass) where a resident kernel (the 2D tile kernel or the
    pass kernel) would run the step; planes=False runs 3D applications as
    three axis passes instead of a plane pass and an axis-0 pass, and 2D
    applications as per-axis passes (resident: the pass kernel) instead of
    the fused tile kernel; absorb_on_a=True makes the absorption switch watch
    max|log a| alone.  stats_dev (a float64 tensor of STATS_DEV_DOUBLES elements on the
    same device) receives the statistics on the device, ordered on the current
    stream after p_next, with no read-back; stats_from_device() reads it."""
    lib = load()
    shape = tuple(p.shape)
    _field(p, shape, "p")
    if stats_dev is not None and (not isinstance(stats_dev, torch.Tensor) or stats_dev.device != p.device
                                  or stats_dev.dtype != torch.float64 or not stats_dev.is_contiguous()
                                  or stats_dev.numel() < STATS_DEV_DOUBLES):
        raise TypeError(f"stats_dev must be a contiguous float64 tensor of at least {STATS_DEV_DOUBLES} "
                        f"elements on {p.device}")
    pout = torch.empty_like(p) if out is None else _field(out, shape, "out")
    g = make_grid(shape)
    prm = make_params(gamma, tau, max_iters, tol, check_every, precision, absorb_threshold, resident, planes,
                      absorb_on_a)
    e = energy.to_c(shape)
    op = OP_ATTRACTION_STEP if energy.kind == "attraction" else OP_STEP
    nb = lib.jko_workspace_bytes(ctypes.byref(g), ctypes.byref(prm), op, 0)
    ws = _workspace(nb, p.device)
    st = Stats()
    _check(lib.jko_step(ctypes.byref(g), ctypes.byref(e), ctypes.byref(prm), _ptr(p), _ptr(pout),
                        ctypes.byref(st) if with_stats else None, _ptr(stats_dev), _ptr(ws), ws.numel(),
                        _stream(p.device)))
    return pout, (st.as_dict() if with_stats else None)


def stats_from_device(rec: torch.Tensor) -> dict:
    """The statistics dict of a device record written by step(stats_dev=...)
    (reads it back, after the work queued before on the current stream)."""
    v = rec[:STATS_DEV_DOUBLES].tolist()
    return dict(iters=int(v[0]), absorptions=int(v[1]), stop="tol" if int(v[2]) == 0 else "cap",
                status=int(v[3]), marginal_l1=v[4], mass=v[5], max_abs_log_a=v[6], max_abs_log_b=v[7])


def step_static(p: torch.Tensor, energy: EnergySpec, gamma: float, tau: float, max_iters: int = 300,
                tol: float = 0.0, check_every: int = 10, precision: str = "fp32",
                absorb_threshold: float = math.inf, out: Optional[torch.Tensor] = None,
                with_stats: bool = True, resident: bool = True, planes: bool = True, absorb_on_a: bool = False):
    """step() on the library's static device workspace (jko_step_static): no
    workspace tensor is allocated.  `out` (optional) lets the caller supply
    the output buffer too, so that the call allocates nothing."""
    lib = load()
    shape = tuple(p.shape)
    _field(p, shape, "p")
    pout = torch.empty_like(p) if out is None else _field(out, shape, "out")
    g = make_grid(shape)
    prm = make_params(gamma, tau, max_iters, tol, check_every, precision, absorb_threshold, resident, planes,
                      absorb_on_a)
    e = energy.to_c(shape)
    st = Stats()
    _check(lib.jko_step_static(ctypes.byref(g), ctypes.byref(e), ctypes.byref(prm), _ptr(p), _ptr(pout),
                               ctypes.byref(st) if with_stats else None, _stream(p.device)))
    return pout, (st.as_dict() if with_stats else None)


def flow(p0: torch.Tensor, energy: EnergySpec, gamma: float, tau: float, n_steps: int,
         max_iters: int = 300, tol: float = 0.0, check_every: int = 10, precision: str = "fp32",
         absorb_threshold: float = math.inf, checkpoints: bool = False, with_stats: bool = True,
         out: Optional[torch.Tensor] = None, resident: bool = True, planes: bool = True,
         absorb_on_a: bool = False):
    """n_steps JKO steps from p0.  Returns (p_T, stats list or None,
    checkpoints tensor (n_steps, *shape) or None)."""
    lib = load()
    shape = tuple(p0.shape)
    _field(p0, shape, "p0")
    pT = torch.empty_like(p0) if out is None else _field(out, shape, "out")
    ck = torch.empty((n_steps,) + shape, dtype=torch.float32, device=p0.device) if checkpoints else None
    g = make_grid(shape)
    prm = make_params(gamma, tau, max_iters, tol, check_every, precision, absorb_threshold, resident, planes,
                      absorb_on_a)
    e = energy.to_c(shape)
    op = OP_ATTRACTION_FLOW if energy.kind == "attraction" else OP_FLOW
    nb = lib.jko_workspace_bytes(ctypes.byref(g), ctypes.byref(prm), op, n_steps)
    ws = _workspace(nb, p0.device)
    sts = (Stats * n_steps)() if with_stats else None
    _check(lib.jko_flow(ctypes.byref(g), ctypes.byref(e), ctypes.byref(prm), int(n_steps), _ptr(p0), _ptr(pT),
                        _ptr(ck), sts, _ptr(ws), ws.numel(), _stream(p0.device)))
    return pT, ([s.as_dict() for s in sts] if with_stats else None), ck


def backward(checkpoints: torch.Tensor, iters_per_step: Sequence[int], dL_dpT: torch.Tensor,
             energy: EnergySpec, gamma: float, tau: float, precision: str = "fp32",
             want_w: bool = True, want_p0: bool = True, resident: bool = True, planes: bool = True):
    """Gradients (dL/dw or None, dL/dp0 or None) of L(p_T) through the flow
    recorded in `checkpoints` at the given iteration counts."""
    lib = load()
    n_steps = int(checkpoints.shape[0])
    shape = tuple(checkpoints.shape[1:])
    if not checkpoints.is_contiguous() or checkpoints.dtype != torch.float32:
        raise TypeError("checkpoints must be contiguous float32")
    _field(dL_dpT, shape, "dL_dpT")
    iters = (ctypes.c_int32 * n_steps)(*[int(k) for k in iters_per_step])
    g = make_grid(shape)
    prm = make_params(gamma, tau, max(iters_per_step), 0.0, 1, precision, resident=resident, planes=planes)
    e = energy.to_c(shape)
    nb = lib.jko_workspace_bytes(ctypes.byref(g), ctypes.byref(prm), OP_BACKWARD, max(iters_per_step))
    ws = _workspace(nb, dL_dpT.device)
    gw = torch.empty_like(dL_dpT) if want_w else None
    gp = torch.empty_like(dL_dpT) if want_p0 else None
    _check(lib.jko_backward(ctypes.byref(g), ctypes.byref(e), ctypes.byref(prm), n_steps, iters,
                            _ptr(checkpoints), _ptr(dL_dpT), _ptr(gw), _ptr(gp), _ptr(ws), ws.numel(),
                            _stream(dL_dpT.device)))
    return gw, gp


def time_iteration(p: torch.Tensor, energy: EnergySpec, gamma: float, tau: float,
                   precision: str = "fp32", reps: int = 50, iters: int = 1, resident: bool = True,
                   planes: bool = True):
    """Mean duration (ms) of each kernel launch, in launch order, timed with
    HIP events on the current stream (measurement aid): the launches of one
    iteration, or the one resident launch running `iters` iterations."""
    lib = load()
    shape = tuple(p.shape)
    _field(p, shape, "p")
    g = make_grid(shape)
    prm = make_params(gamma, tau, iters, 0.0, 1, precision, resident=resident, planes=planes)
    e = energy.to_c(shape)
    nb = lib.jko_workspace_bytes(ctypes.byref(g), ctypes.byref(prm), OP_STEP, 0)
    ws = _workspace(nb, p.device)
    out = (ctypes.c_double * (2 * len(shape)))()
    cnt = ctypes.c_int32(0)
    _check(lib.jko_time_iteration(ctypes.byref(g), ctypes.byref(e), ctypes.byref(prm), _ptr(p), int(reps), out,
                                  ctypes.byref(cnt), _ptr(ws), ws.numel(), _stream(p.device)))
    return list(out)[:cnt.value]


class JKOFlowFn(torch.autograd.Function):
    """p_T = JKO flow of p0 for the congestion energy with potential w, at
    fixed iteration counts; backward calls the library's adjoint, which
    recomputes each step from its checkpoint."""

    @staticmethod
    def forward(ctx, p0, w, kappa, gamma, tau, n_steps, iters, precision):
        en = EnergySpec(kind="congestion", w=w.detach(), kappa=kappa)
        pT, stats, ck = flow(p0.detach(), en, gamma, tau, n_steps, max_iters=iters, tol=0.0,
                             precision=precision, checkpoints=True, with_stats=False)
        ctx.save_for_backward(ck, w.detach(), kappa)
        ctx.cfg = (gamma, tau, n_steps, iters, precision)
        return pT

    @staticmethod
    def backward(ctx, grad_out):
        ck, w, kappa = ctx.saved_tensors
        gamma, tau, n_steps, iters, precision = ctx.cfg
        en = EnergySpec(kind="congestion", w=w, kappa=kappa)
        gw, gp = backward(ck, [iters] * n_steps, grad_out.contiguous(), en, gamma, tau, precision,
                          want_w=ctx.needs_input_grad[1], want_p0=ctx.needs_input_grad[0])
        return gp, gw, None, None, None, None, None, None


class HeatOperator:
    """The heat-kernel Gibbs operator xi~ = (Id - (gamma/L) Delta_M)^{-L} of
    Section 4.1 on the free cells of a 2D grid (mask: CUDA bool/uint8 tensor
    of the grid's shape, True = free; None = no obstacle).  Up to 65536 cells
    construction builds xi~ once on the GPU into a workspace this object owns
    (N^2 * 2 bytes and more); above (or with per_product=True) every product
    is L solves on the grid instead and nothing is stored.  apply() and
    flow() then use it.  The mask is kept (the library reads it on every
    call)."""

    def __init__(self, shape, gamma: float, L: int = 10, mask: Optional[torch.Tensor] = None, device=None,
                 per_product: bool = False):
        lib = load()
        shape = tuple(int(n) for n in shape)
        if len(shape) == 1:
            shape = (1, shape[0])
        if len(shape) != 2:
            raise ValueError("the heat kernel takes 1D or 2D grids")
        self.shape = shape
        self.gamma = float(gamma)
        self.L = int(L)
        if mask is not None:
            if not isinstance(mask, torch.Tensor) or mask.device.type != "cuda":
                raise TypeError("mask must be a CUDA (HIP) tensor")
            if mask.numel() != shape[0] * shape[1]:
                raise TypeError(f"mask must have {shape[0] * shape[1]} cells")
            device = mask.device
            self.mask = mask.reshape(shape).to(torch.uint8).contiguous()
        else:
            self.mask = None
            device = torch.device("cuda") if device is None else torch.device(device)
        self.device = device
        self.dom = HeatDomain(shape[0], shape[1], _ptr(self.mask), self.L, 1 if per_product else 0)
        nb = lib.jko_heat_workspace_bytes(ctypes.byref(self.dom))
        if nb == 0:
            raise JKOError(JKO_ERR_INVALID, f"invalid heat domain {shape}, L={L}")
        self.ws = _workspace(nb, device)
        _check(lib.jko_heat_build(ctypes.byref(self.dom), self.gamma, _ptr(self.ws), self.ws.numel(),
                                  _stream(device)))

    def _grid_field(self, t, name):
        if t is None:
            return None
        if t.numel() != self.shape[0] * self.shape[1]:
            raise TypeError(f"{name} must have {self.shape[0] * self.shape[1]} cells")
        return _field(t, tuple(t.shape), name)

    def apply(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """y = xi~ x for a float32 CUDA field of the grid's cells."""
        lib = load()
        self._grid_field(x, "x")
        y = torch.empty_like(x) if out is None else self._grid_field(out, "out")
        _check(lib.jko_heat_apply(ctypes.byref(self.dom), _ptr(x), _ptr(y), _ptr(self.ws), self.ws.numel(),
                                  _stream(x.device)))
        return y

    def flow(self, p0: torch.Tensor, energy: EnergySpec, tau: float, n_steps: int, max_iters: int = 300,
             tol: float = 0.0, check_every: int = 10, with_stats: bool = True, out: Optional[torch.Tensor] = None):
        """n_steps JKO steps from p0 with xi~ as the Gibbs kernel.  Returns
        (p_T, stats list or None)."""
        lib = load()
        self._grid_field(p0, "p0")
        pT = torch.empty_like(p0) if out is None else self._grid_field(out, "out")
        prm = make_params(self.gamma, tau, max_iters, tol, check_every)
        e = energy.to_c(tuple(p0.shape))
        sts = (Stats * n_steps)() if with_stats else None
        _check(lib.jko_heat_flow(ctypes.byref(self.dom), ctypes.byref(e), ctypes.byref(prm), int(n_steps), _ptr(p0),
                                 _ptr(pT), sts, _ptr(self.ws), self.ws.numel(), _stream(p0.device)))
        return pT, ([st.as_dict() for st in sts] if with_stats else None)

    def step(self, p: torch.Tensor, energy: EnergySpec, tau: float, **kw):
        pT, sts = self.flow(p, energy, tau, 1, **kw)
        return pT, (sts[0] if sts else None)
