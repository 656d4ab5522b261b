"""MI355X butterfly evaluator for 2-D discrete Fourier integral operators.

    u(x) = sum_{k in Omega} exp(2 pi i Phi(x,k)) f(k),  x in X          (eq:dfio)

evaluated by the butterfly algorithm of Candes, Demanet & Ying (Sec. 4):
polar P-tree x dyadic X-tree, tensor Chebyshev expansions per box pair,
HIP kernels for gfx950 behind the C ABI of ``include/fio.h``.

This module is argument marshalling only: every step of the pass runs in
the HIP library ``libfio.so``.  PyTorch provides device memory and streams.
If the library is missing the calls raise; there is no CPU fallback.

    >>> plan = Plan(1024, 9)                       # eq:ex1 phase, FP32 weights
    >>> u = plan.apply(f)                          # f: (N, N) or (R, N, N) complex64 on cuda
    >>> g = plan.adjoint(u)                        # B^H u
    >>> u = fio_apply(f, plan)                     # autograd: backward is the adjoint
    >>> u = fio_apply(f, plan, a)                  # a = (a1, a2): gradients for the phase too
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

__all__ = [
    "Phase", "Plan", "Plan3", "Batch", "FIOApply", "FIOApply3", "FIOApplyPhase", "fio_apply", "direct_rows",
    "select_q",
    "load_library", "library_path",
    "FOURIER", "ELLIPSE", "C128", "C64", "EXPORTED_SYMBOLS",
]

FOURIER = 0
ELLIPSE = 1
SPHERES = 1  # three-dimensional phase kind of eq:ex3 (Plan3)
C128 = 0
C64 = 1
CONTRACT_FP = 0
CONTRACT_BF16 = 1
CONTRACT_MFMA = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfio.so")

# every symbol include/fio.h declares
EXPORTED_SYMBOLS = (
    "fio_plan", "fio_plan_ex", "fio_set_phase", "fio_plan_get_info", "fio_plan_autotune", "fio_plan_set_shape", "fio_apply",
    "fio_apply_adjoint", "fio_debug_stage", "fio_destroy", "fio_last_error",
    "fio_profile_enable", "fio_profile_read", "fio_apply_dphase", "fio_apply_amplitude",
    "fio_apply_amplitude_adjoint", "fio_apply_amplitude_noalloc", "fio_batch_create", "fio_batch_apply", "fio_batch_apply_adjoint",
    "fio_batch_destroy", "fio_direct_rows", "fio_select_q", "fio3_plan", "fio3_apply", "fio3_apply_adjoint",
    "fio3_destroy",
)

# kernel kinds of fio_profile_read (FIO_K_* in include/fio.h)
KERNEL_KINDS = ("init", "plevel", "switch", "xlevel", "term",
                "term_adj", "xlevel_adj", "switch_adj", "plevel_adj", "init_adj",
                "tangent", "tables")


def library_path() -> str:
    return _LIB_PATH


@dataclass(frozen=True)
class Phase:
    """Phase descriptor (``fio_phase_t``).  ELLIPSE with the defaults is eq:ex1."""

    kind: int = ELLIPSE
    a1: float = 1.0
    a2: float = 1.0
    eta1: float = 0.0
    eta2: float = 0.0


class _CPhase(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("a1", ctypes.c_double), ("a2", ctypes.c_double),
                ("eta1", ctypes.c_double), ("eta2", ctypes.c_double)]


class _COpts(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int), ("lm", ctypes.c_int), ("dtype", ctypes.c_int),
                ("nrhs_max", ctypes.c_int), ("contract", ctypes.c_int)]


class _CInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("q", ctypes.c_int), ("L", ctypes.c_int), ("s", ctypes.c_int),
                ("lm", ctypes.c_int), ("dtype", ctypes.c_int), ("contract", ctypes.c_int),
                ("n_pairs", ctypes.c_int64),
                ("weights_per_level", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("max_box_sources", ctypes.c_int), ("nrhs_max", ctypes.c_int), ("chunk", ctypes.c_int),
                ("switch_items", ctypes.c_int)]


class _CTune(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int), ("switch_items", ctypes.c_int), ("candidates", ctypes.c_int),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]


_lib = None


def load_library():
    """Load ``libfio.so`` (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"HIP library {_LIB_PATH} is not built; run "
                           "`python -m paper_0809_0719_amd.build` (or __graft_entry__.build())")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i = ctypes.c_void_p, ctypes.c_int
    lib.fio_plan.argtypes = [i, i, ctypes.POINTER(_CPhase), ctypes.POINTER(vp)]
    lib.fio_plan_ex.argtypes = [i, i, ctypes.POINTER(_CPhase), ctypes.POINTER(_COpts), ctypes.POINTER(vp)]
    lib.fio_set_phase.argtypes = [vp, ctypes.POINTER(_CPhase)]
    lib.fio_plan_get_info.argtypes = [vp, ctypes.POINTER(_CInfo)]
    lib.fio_plan_autotune.argtypes = [vp, ctypes.c_int, ctypes.POINTER(_CTune)]
    lib.fio_plan_set_shape.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.fio_apply.argtypes = [vp, vp, vp, i, i, vp]
    lib.fio_apply_adjoint.argtypes = [vp, vp, vp, i, i, vp]
    lib.fio_apply_dphase.argtypes = [vp, vp, vp, vp, vp, i, vp]
    lib.fio_apply_amplitude.argtypes = [vp, vp, vp, vp, i, vp, vp]
    lib.fio_apply_amplitude_adjoint.argtypes = [vp, vp, vp, vp, i, vp, vp]
    lib.fio_apply_amplitude_noalloc.argtypes = [vp, vp, vp, vp, i, vp, vp]
    lib.fio_debug_stage.argtypes = [vp, vp, i, vp, vp]
    lib.fio_batch_create.argtypes = [ctypes.POINTER(vp), i, i, ctypes.POINTER(vp)]
    lib.fio_batch_apply.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    lib.fio_batch_apply_adjoint.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    lib.fio_batch_destroy.argtypes = [vp]
    lib.fio_direct_rows.argtypes = [vp, vp, vp, i, vp, vp]
    lib.fio3_plan.argtypes = [i, i, i, i, i, i, ctypes.POINTER(vp)]
    lib.fio3_apply.argtypes = [vp, vp, vp, vp]
    lib.fio3_apply_adjoint.argtypes = [vp, vp, vp, vp]
    lib.fio3_destroy.argtypes = [vp]
    lib.fio_select_q.argtypes = [i, ctypes.POINTER(_CPhase), ctypes.POINTER(_COpts), ctypes.c_double, i, i, i,
                                 ctypes.c_uint64, ctypes.POINTER(i), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)]
    lib.fio_destroy.argtypes = [vp]
    lib.fio_profile_enable.argtypes = [vp, i]
    lib.fio_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), i]
    lib.fio_last_error.restype = ctypes.c_char_p
    for name in EXPORTED_SYMBOLS:
        if name != "fio_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != 0:
        msg = load_library().fio_last_error().decode(errors="replace")
        raise RuntimeError(f"{what} failed ({rc}): {msg}")


def _cphase(ph: Phase) -> _CPhase:
    return _CPhase(int(ph.kind), float(ph.a1), float(ph.a2), float(ph.eta1), float(ph.eta2))


class Plan:
    """A butterfly plan (``fio_plan_ex``) on the current HIP device.

    N: grid side (power of two, 8..8192); q: Chebyshev points per dimension
    (3..16); phase: :class:`Phase`; s, lm: start offset and switch level
    (defaults min(3, L/2) and L/2); dtype: torch.complex64 (FP32 weights,
    FP64 phases) or torch.complex128 (FP64 throughout); nrhs_max: right-hand
    sides processed together, sharing every kernel value of the levels and
    the switch (the plan holds 2 x nrhs_max x N^2 q^2 complex weights);
    contract: "fp" (contractions in the weight precision on the vector ALUs)
    or "bf16" (BF16 operands, FP32 accumulation on the matrix cores;
    complex64 plans, q <= 12) or "mfma" (FP32 matrix-core p-levels and
    adjoint x-levels for chunks of 32 or more right-hand sides, the rest as
    "fp"; complex64 plans, q <= 9).
    """

    def __init__(self, N: int, q: int, phase: Phase = Phase(), s: int | None = None,
                 lm: int | None = None, dtype: torch.dtype = torch.complex64, nrhs_max: int = 1,
                 contract: str = "fp"):
        lib = load_library()
        if dtype not in (torch.complex64, torch.complex128):
            raise ValueError("dtype must be torch.complex64 or torch.complex128")
        self.dtype = dtype
        self.device = torch.device("cuda", torch.cuda.current_device())
        codes = {"fp": CONTRACT_FP, "bf16": CONTRACT_BF16, "mfma": CONTRACT_MFMA}
        if contract not in codes:
            raise ValueError('contract must be "fp", "bf16" or "mfma"')
        opts = _COpts(-1 if s is None else int(s), -1 if lm is None else int(lm),
                      C64 if dtype == torch.complex64 else C128, int(nrhs_max), codes[contract])
        h = ctypes.c_void_p()
        _check(lib.fio_plan_ex(int(N), int(q), ctypes.byref(_cphase(phase)), ctypes.byref(opts),
                               ctypes.byref(h)), "fio_plan_ex")
        self._h = h
        self.phase = phase
        info = _CInfo()
        _check(lib.fio_plan_get_info(h, ctypes.byref(info)), "fio_plan_get_info")
        self.N, self.q, self.L, self.s, self.lm = info.N, info.q, info.L, info.s, info.lm
        self.workspace_bytes = int(info.workspace_bytes)
        self.max_box_sources = int(info.max_box_sources)
        self.nrhs_max = int(info.nrhs_max)
        self.contract = contract
        self.n_stages = self.L - 2 * self.s + 2

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().fio_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- parameters ---------------------------------------------------------
    def set_phase(self, phase: Phase):
        _check(load_library().fio_set_phase(self._h, ctypes.byref(_cphase(phase))), "fio_set_phase")
        self.phase = phase

    def shape(self) -> dict:
        """The launch shape applies use: right-hand sides per pass and pair
        items per workgroup of the matrix-core switches."""
        info = _CInfo()
        _check(load_library().fio_plan_get_info(self._h, ctypes.byref(info)), "fio_plan_get_info")
        return {"chunk": int(info.chunk), "switch_items": int(info.switch_items)}

    def set_shape(self, chunk: int, switch_items: int):
        """Set the launch shape directly (``fio_plan_set_shape``)."""
        _check(load_library().fio_plan_set_shape(self._h, int(chunk), int(switch_items)), "fio_plan_set_shape")

    def autotune(self, nrhs: int) -> dict:
        """Time the launch shapes for calls of nrhs right-hand sides and keep
        the fastest (``fio_plan_autotune``; synchronises the device)."""
        t = _CTune()
        _check(load_library().fio_plan_autotune(self._h, int(nrhs), ctypes.byref(t)), "fio_plan_autotune")
        return {"chunk": int(t.chunk), "switch_items": int(t.switch_items), "candidates": int(t.candidates),
                "best_ms": float(t.best_ms), "default_ms": float(t.default_ms)}

    # -- helpers ------------------------------------------------------------
    def _prep(self, x: torch.Tensor, name: str):
        if not isinstance(x, torch.Tensor) or not x.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if x.dtype != self.dtype:
            raise TypeError(f"{name} must be {self.dtype} (got {x.dtype})")
        if x.shape[-2:] != (self.N, self.N):
            raise ValueError(f"{name} must have trailing shape ({self.N}, {self.N}), got {tuple(x.shape)}")
        if x.device != self.device:
            raise ValueError(f"{name} is on {x.device}, plan on {self.device}")
        x = x.contiguous()
        nrhs = x.numel() // (self.N * self.N)
        return x, nrhs

    def _out(self, out: torch.Tensor | None, like: torch.Tensor, name: str) -> torch.Tensor:
        """The output tensor: a new one shaped like the input, or the caller's
        ``out``, which the kernels overwrite through its data pointer -- so it
        must have the input's shape and dtype, sit on the plan's device, be
        contiguous and share no memory with the input."""
        if out is None:
            return torch.empty_like(like)
        if not isinstance(out, torch.Tensor) or not out.is_cuda or out.device != self.device:
            raise ValueError(f"{name} must be a tensor on {self.device}")
        if out.dtype != like.dtype or out.shape != like.shape:
            raise ValueError(f"{name} must be {like.dtype} of shape {tuple(like.shape)} "
                             f"(got {out.dtype} {tuple(out.shape)})")
        if not out.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        a0, a1 = out.data_ptr(), out.data_ptr() + out.numel() * out.element_size()
        b0, b1 = like.data_ptr(), like.data_ptr() + like.numel() * like.element_size()
        if a0 < b1 and b0 < a1:
            raise ValueError(f"{name} must not overlap the input")
        return out

    @property
    def _dtype_code(self) -> int:
        return C64 if self.dtype == torch.complex64 else C128

    # -- the butterfly ------------------------------------------------------
    def apply(self, f: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """u = B f for f of shape (..., N, N) with f[..., k1+N/2, k2+N/2]."""
        f, nrhs = self._prep(f, "f")
        u = self._out(out, f, "out")
        if nrhs == 0:
            return u
        st = torch.cuda.current_stream(self.device).cuda_stream
        _check(load_library().fio_apply(self._h, f.data_ptr(), u.data_ptr(), nrhs, self._dtype_code, st),
               "fio_apply")
        return u

    def adjoint(self, u: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """f = B^H u for u of shape (..., N, N) with u[..., i1, i2] = u(i1/N, i2/N)."""
        u, nrhs = self._prep(u, "u")
        f = self._out(out, u, "out")
        if nrhs == 0:
            return f
        st = torch.cuda.current_stream(self.device).cuda_stream
        _check(load_library().fio_apply_adjoint(self._h, u.data_ptr(), f.data_ptr(), nrhs, self._dtype_code, st),
               "fio_apply_adjoint")
        return f

    def apply_dphase(self, f: torch.Tensor, primal: bool = True):
        """(u, du/da1, du/da2) for f of shape (..., N, N): the butterfly and its
        exact derivatives with respect to the velocity scalings of the phase
        (u is None when ``primal`` is False).  Requires q <= 12."""
        f, nrhs = self._prep(f, "f")
        u = torch.empty_like(f) if primal else None
        d1 = torch.empty_like(f)
        d2 = torch.empty_like(f)
        if nrhs == 0:
            return u, d1, d2
        st = torch.cuda.current_stream(self.device).cuda_stream
        _check(load_library().fio_apply_dphase(self._h, f.data_ptr(), None if u is None else u.data_ptr(),
                                               d1.data_ptr(), d2.data_ptr(), nrhs, st), "fio_apply_dphase")
        return u, d1, d2

    def _prep_factors(self, g: torch.Tensor, h: torch.Tensor):
        g, rg = self._prep(g, "g")
        h, rh = self._prep(h, "h")
        if rg != rh or rg < 1:
            raise ValueError(f"g and h must hold the same number (>= 1) of factors, got {rg} and {rh}")
        return g, h, rg

    def apply_amplitude(self, f: torch.Tensor, g: torch.Tensor, h: torch.Tensor,
                        out: torch.Tensor | None = None) -> torch.Tensor:
        """u = sum_t g_t . B(h_t . f): the FIO with amplitude a(x,k) = sum_t g_t(x) h_t(k)
        (g: (rank, N, N) on the x grid, h: (rank, N, N) on the frequency grid, f: (N, N))."""
        f, nrhs = self._prep(f, "f")
        if nrhs != 1:
            raise ValueError("apply_amplitude takes one right-hand side")
        g, h, rank = self._prep_factors(g, h)
        u = self._out(out, f, "out")
        st = torch.cuda.current_stream(self.device).cuda_stream
        _check(load_library().fio_apply_amplitude(self._h, f.data_ptr(), g.data_ptr(), h.data_ptr(), rank,
                                                  u.data_ptr(), st), "fio_apply_amplitude")
        return u

    def adjoint_amplitude(self, u: torch.Tensor, g: torch.Tensor, h: torch.Tensor,
                          out: torch.Tensor | None = None) -> torch.Tensor:
        """f = sum_t conj(h_t) . B^H(conj(g_t) . u): the adjoint of apply_amplitude."""
        u, nrhs = self._prep(u, "u")
        if nrhs != 1:
            raise ValueError("adjoint_amplitude takes one right-hand side")
        g, h, rank = self._prep_factors(g, h)
        f = self._out(out, u, "out")
        st = torch.cuda.current_stream(self.device).cuda_stream
        _check(load_library().fio_apply_amplitude_adjoint(self._h, u.data_ptr(), g.data_ptr(), h.data_ptr(),
                                                          rank, f.data_ptr(), st), "fio_apply_amplitude_adjoint")
        return f

    def debug_stage(self, f: torch.Tensor, stage: int) -> torch.Tensor:
        """Weights after forward stage ``stage`` (layout in include/fio.h)."""
        f, nrhs = self._prep(f, "f")
        if nrhs != 1:
            raise ValueError("debug_stage takes one right-hand side")
        w = torch.empty(self.N * self.N * self.q * self.q, dtype=self.dtype, device=self.device)
        st = torch.cuda.current_stream(self.device).cuda_stream
        _check(load_library().fio_debug_stage(self._h, f.data_ptr(), int(stage), w.data_ptr(), st),
               "fio_debug_stage")
        return w

    # -- per-kernel timing ----------------------------------------------------
    def profile(self, enable: bool = True):
        """Bracket every kernel launch with HIP events on its stream."""
        _check(load_library().fio_profile_enable(self._h, int(bool(enable))), "fio_profile_enable")

    def profile_read(self) -> dict:
        """{kind: (total ms, launches)} since the last read (waits for the events)."""
        n = len(KERNEL_KINDS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(load_library().fio_profile_read(self._h, ms, cnt, n), "fio_profile_read")
        return {k: (ms[i], int(cnt[i])) for i, k in enumerate(KERNEL_KINDS) if cnt[i]}

    def stage_level(self, stage: int) -> int:
        """Tree level l of T_X of the weights after ``stage``."""
        if stage <= self.lm - self.s:
            return self.s + stage
        return self.lm + (stage - (self.lm - self.s) - 1)


class FIOApply(torch.autograd.Function):
    """u = B f with backward grad_f = B^H grad_u (B is C-linear, so the
    conjugate-Wirtinger vector-Jacobian product is the adjoint)."""

    @staticmethod
    def forward(ctx, f: torch.Tensor, plan: Plan):
        ctx.plan = plan
        return plan.apply(f)

    @staticmethod
    def backward(ctx, grad_u: torch.Tensor):
        return ctx.plan.adjoint(grad_u.contiguous()), None


class FIOApplyPhase(torch.autograd.Function):
    """u = B(a) f with the velocity scalings a = (a1, a2) of the ellipse phase
    as a second differentiable input.  Backward: grad_f = B^H grad_u, and
    grad_a_j = Re <grad_u, du/da_j> with du/da_j from the forward-mode
    tangent pass (two parameters, so one tangent pass per right-hand side)."""

    @staticmethod
    def forward(ctx, f: torch.Tensor, a: torch.Tensor, plan: Plan):
        a1, a2 = (float(v) for v in a.detach().to("cpu", torch.float64))
        ph = plan.phase
        phase = Phase(ph.kind, a1, a2, ph.eta1, ph.eta2)
        plan.set_phase(phase)
        ctx.plan, ctx.phase, ctx.a_meta = plan, phase, (a.device, a.dtype)
        ctx.save_for_backward(f)
        return plan.apply(f)

    @staticmethod
    def backward(ctx, grad_u: torch.Tensor):
        plan = ctx.plan
        (f,) = ctx.saved_tensors
        plan.set_phase(ctx.phase)
        grad_u = grad_u.contiguous()
        grad_f = grad_a = None
        if ctx.needs_input_grad[0]:
            grad_f = plan.adjoint(grad_u)
        if ctx.needs_input_grad[1]:
            _, d1, d2 = plan.apply_dphase(f, primal=False)
            g = torch.stack([torch.sum((grad_u.conj() * d).real.double()) for d in (d1, d2)])
            grad_a = g.to(device=ctx.a_meta[0], dtype=ctx.a_meta[1])
        return grad_f, grad_a, None


def fio_apply(f: torch.Tensor, plan: Plan, a: torch.Tensor | None = None) -> torch.Tensor:
    """u = B f with autograd.  With ``a`` (a real tensor (a1, a2)), the plan's
    ellipse velocity scalings are set to ``a`` and ``a`` gets gradients too."""
    if a is None:
        return FIOApply.apply(f, plan)
    return FIOApplyPhase.apply(f, a, plan)


class Batch:
    """Several plans applied as one unit (``fio_batch_create``): each plan's
    apply runs on one of ``nstreams`` internal streams, forked from and
    joined back into the current stream, so problems of different sizes run
    side by side; a stream capture of :meth:`apply` records the whole batch
    as one graph.  The batch keeps references to its plans."""

    def __init__(self, plans, nstreams: int = 4):
        self.plans = list(plans)
        if len({id(p) for p in self.plans}) != len(self.plans):
            raise ValueError("a plan appears twice in the batch")
        handles = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(load_library().fio_batch_create(handles, len(self.plans), int(nstreams), ctypes.byref(h)),
               "fio_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().fio_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _run(self, fn, xs, outs, name):
        if len(xs) != len(self.plans):
            raise ValueError(f"need {len(self.plans)} inputs, got {len(xs)}")
        xs = [p._prep(x, name)[0] for p, x in zip(self.plans, xs)]
        for p, x in zip(self.plans, xs):
            if x.numel() != p.N * p.N:
                raise ValueError(f"{name}: one right-hand side per plan")
        if outs is not None and len(outs) != len(xs):
            raise ValueError(f"need {len(xs)} outputs, got {len(outs)}")
        outs = [p._out(None if outs is None else outs[i], x, f"{name} output {i}")
                for i, (p, x) in enumerate(zip(self.plans, xs))]
        n = len(xs)
        a = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        b = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        st = torch.cuda.current_stream(self.plans[0].device).cuda_stream
        _check(fn(self._h, a, b, st), name)
        return outs

    def apply(self, fs, outs=None):
        """[B_i f_i] for the plans B_i (one (N_i, N_i) input each)."""
        return self._run(load_library().fio_batch_apply, fs, outs, "fio_batch_apply")

    def adjoint(self, us, outs=None):
        """[B_i^H u_i]."""
        return self._run(load_library().fio_batch_apply_adjoint, us, outs, "fio_batch_apply_adjoint")


def direct_rows(plan: Plan, f: torch.Tensor, rows: torch.Tensor) -> torch.Tensor:
    """u(x_r) = sum_k exp(2 pi i Phi(x_r, k)) f(k) for the flat target indices
    ``rows`` (int64, on the plan's device), FP64 inside (``fio_direct_rows``)."""
    f, nrhs = plan._prep(f, "f")
    if nrhs != 1:
        raise ValueError("direct_rows takes one right-hand side")
    rows = rows.to(device=plan.device, dtype=torch.int64).contiguous()
    out = torch.empty(rows.numel(), dtype=plan.dtype, device=plan.device)
    if rows.numel() == 0:
        return out
    st = torch.cuda.current_stream(plan.device).cuda_stream
    _check(load_library().fio_direct_rows(plan._h, f.data_ptr(), rows.data_ptr(), rows.numel(), out.data_ptr(), st),
           "fio_direct_rows")
    return out


def select_q(N: int, phase: Phase = Phase(), tol: float = 1e-4, qmin: int = 3, qmax: int = 16,
             nrows: int = 64, seed: int = 0, s: int | None = None, lm: int | None = None,
             dtype: torch.dtype = torch.complex64):
    """The smallest q in [qmin, qmax] whose estimated error eq:err is <= tol
    (``fio_select_q``).  Returns (q, estimate, {q: estimate for every q tried});
    when no q reaches tol, q is qmax and its estimate exceeds tol."""
    opts = _COpts(-1 if s is None else int(s), -1 if lm is None else int(lm),
                  C64 if dtype == torch.complex64 else C128, 1, CONTRACT_FP)
    q = ctypes.c_int()
    err = ctypes.c_double()
    n = max(qmax - qmin + 1, 1)
    errs = (ctypes.c_double * n)()
    _check(load_library().fio_select_q(int(N), ctypes.byref(_cphase(phase)), ctypes.byref(opts), float(tol),
                                       int(qmin), int(qmax), int(nrows), int(seed) & (2**64 - 1), ctypes.byref(q),
                                       ctypes.byref(err), errs), "fio_select_q")
    tried = {qmin + i: errs[i] for i in range(n) if errs[i] == errs[i]}
    return q.value, err.value, tried


class Plan3:
    """Three-dimensional butterfly plan (``fio3_plan``): N^3 targets and
    frequencies, q^3 Chebyshev grids, octrees.  kind: FOURIER (x . k) or
    SPHERES (eq:ex3); s, lm as for :class:`Plan`; dtype complex64 or
    complex128.  Forward and adjoint applies of one right-hand side (N, N, N)."""

    def __init__(self, N: int, q: int, kind: int = SPHERES, s: int | None = None, lm: int | None = None,
                 dtype: torch.dtype = torch.complex64):
        lib = load_library()
        if dtype not in (torch.complex64, torch.complex128):
            raise ValueError("dtype must be torch.complex64 or torch.complex128")
        self.N, self.q, self.kind, self.dtype = int(N), int(q), int(kind), dtype
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        _check(lib.fio3_plan(self.N, self.q, self.kind, -1 if s is None else int(s), -1 if lm is None else int(lm),
                             C64 if dtype == torch.complex64 else C128, ctypes.byref(h)), "fio3_plan")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().fio3_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, f: torch.Tensor) -> torch.Tensor:
        """u = B f for f of shape (N, N, N), f[k1+N/2, k2+N/2, k3+N/2]."""
        if not isinstance(f, torch.Tensor) or not f.is_cuda or f.dtype != self.dtype:
            raise TypeError(f"f must be a {self.dtype} CUDA (HIP) tensor")
        if tuple(f.shape) != (self.N,) * 3:
            raise ValueError(f"f must have shape ({self.N}, {self.N}, {self.N})")
        f = f.contiguous()
        u = torch.empty_like(f)
        st = torch.cuda.current_stream(self.device).cuda_stream
        _check(load_library().fio3_apply(self._h, f.data_ptr(), u.data_ptr(), st), "fio3_apply")
        return u

    def adjoint(self, u: torch.Tensor) -> torch.Tensor:
        """f = B^H u for u of shape (N, N, N), u[i1, i2, i3] = u(i/N)."""
        if not isinstance(u, torch.Tensor) or not u.is_cuda or u.dtype != self.dtype:
            raise TypeError(f"u must be a {self.dtype} CUDA (HIP) tensor")
        if tuple(u.shape) != (self.N,) * 3:
            raise ValueError(f"u must have shape ({self.N}, {self.N}, {self.N})")
        u = u.contiguous()
        f = torch.empty_like(u)
        st = torch.cuda.current_stream(self.device).cuda_stream
        _check(load_library().fio3_apply_adjoint(self._h, u.data_ptr(), f.data_ptr(), st), "fio3_apply_adjoint")
        return f


class FIOApply3(torch.autograd.Function):
    """u = B f for a :class:`Plan3`, with backward grad_f = B^H grad_u."""

    @staticmethod
    def forward(ctx, f: torch.Tensor, plan: Plan3):
        ctx.plan = plan
        return plan.apply(f)

    @staticmethod
    def backward(ctx, grad_u: torch.Tensor):
        return ctx.plan.adjoint(grad_u.contiguous()), None
