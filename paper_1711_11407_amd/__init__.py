"""MI355X-native FPS-SFT: the D-dimensional sparse Fourier transform of
Wang, Patel and Petropulu (arXiv 1711.11407), hot path in gfx950 HIP kernels.

Python surface over the C ABI (include/fpssft.h). PyTorch provides device
memory and streams only; every step of the transform runs in the HIP
kernels of libfpssft.so.

    plan = Plan([CubeSpec((256, 256), seed=3)])
    res = plan.execute(0, x)             # x: complex64 cuda tensor
    h = res.host()                       # synchronises
    h["k"], h["freqs"], h["amps"]        # the recovered set

Differentiable amplitudes (frequencies fixed, not differentiated):

    amps = sft_amplitudes(plan, 0, x)    # torch.autograd.Function
    (amps.abs() ** 2).sum().backward()   # x.grad via the adjoint kernel
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional, Sequence

import numpy as np

from . import _binding as B
from ._binding import FpsSftError  # noqa: F401

STATUS_OK, STATUS_INCOMPLETE, STATUS_CAPACITY = B.OK, B.INCOMPLETE, B.CAPACITY


@dataclasses.dataclass
class CubeSpec:
    """Problem description of one cube (fpssft_desc)."""

    dims: Sequence[int]
    seed: int = 0
    max_iters: int = 0          # 0: floor(N / ((D+1) L)), at least 1
    max_k: int = 4096
    zero_thresh: float = 1e-3
    mag_rel_tol: float = 1e-3
    grid_tol: float = 1e-2
    schedule: Optional[np.ndarray] = None   # int32 [T][2][D] (alpha, tau)
    axis_schedule: bool = False  # generated slopes e_{t mod D} (FPSSFT_FLAG_AXIS_SCHEDULE)
    amp_average: bool = False    # amplitude averaged over the D+1 lines (FPSSFT_FLAG_AMP_AVERAGE)
    literal_peel: bool = False   # time-domain construction-subtraction (FPSSFT_FLAG_LITERAL_PEEL)
    deterministic: bool = False  # FPSSFT_FLAG_DETERMINISTIC (every plan is bit-reproducible)

    @property
    def flags(self) -> int:
        return ((B.FLAG_AXIS_SCHEDULE if self.axis_schedule else 0)
                | (B.FLAG_AMP_AVERAGE if self.amp_average else 0)
                | (B.FLAG_LITERAL_PEEL if self.literal_peel else 0)
                | (B.FLAG_DETERMINISTIC if self.deterministic else 0))

    def to_c(self):
        d = B.Desc()
        dims = [int(v) for v in self.dims]
        if not 1 <= len(dims) <= B.MAX_D:
            raise ValueError("1 <= D <= 4")
        d.ndim = len(dims)
        for k in range(B.MAX_D):
            d.dims[k] = dims[k] if k < len(dims) else 1
        d.max_iters = int(self.max_iters)
        d.max_k = int(self.max_k)
        d.seed = int(self.seed) & ((1 << 64) - 1)
        d.zero_thresh = float(self.zero_thresh)
        d.mag_rel_tol = float(self.mag_rel_tol)
        d.grid_tol = float(self.grid_tol)
        d.flags = self.flags
        keep = None
        if self.schedule is not None:
            keep = np.ascontiguousarray(self.schedule, dtype=np.int32)
            d.schedule = keep.ctypes.data_as(C.POINTER(C.c_int32))
        return d, keep


def validate(spec: CubeSpec):
    """(L, T_max) of a description, or raises FpsSftError."""
    d, _keep = spec.to_c()
    L, T = C.c_int32(), C.c_int32()
    B.check(B.lib().fpssft_validate(C.byref(d), C.byref(L), C.byref(T)), "validate")
    return L.value, T.value


def schedule_generate(spec: CubeSpec, T: int) -> np.ndarray:
    """The SplitMix64 line schedule of a description: int32 [T][2][D]."""
    d, _keep = spec.to_c()
    out = np.zeros((T, 2, d.ndim), dtype=np.int32)
    B.check(B.lib().fpssft_schedule_generate(C.byref(d), T, out.ctypes.data_as(C.POINTER(C.c_int32))),
            "schedule_generate")
    return out


def _torch():
    import torch
    return torch


def _stream_ptr(stream) -> C.c_void_p:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


@dataclasses.dataclass
class Result:
    """Device outputs of one cube (fpssft_out): the recovered set (distinct
    frequencies, amplitudes summed over their detections; entries k..k+kd-1
    are merged frequencies whose sum vanished, left out of the set) and the
    detection trace in canonical (iteration, bin) order."""

    freqs: "object"     # int32 [max_k, D]
    amps: "object"      # complex64 [max_k]
    rec_iter: "object"  # int32 [max_k]: detection -> iteration
    rec_bin: "object"   # int32 [max_k]: detection -> bin
    rec_sin: "object"   # int32 [max_k]: detection -> index in freqs/amps
    info: "object"      # int32 [8]: k, iterations, status, n, kd, 0, 0, 0

    def c_out(self) -> B.Out:
        o = B.Out()
        o.freqs = self.freqs.data_ptr()
        o.amps = self.amps.data_ptr()
        o.rec_iter = self.rec_iter.data_ptr()
        o.rec_bin = self.rec_bin.data_ptr()
        o.rec_sin = self.rec_sin.data_ptr()
        o.info = self.info.data_ptr()
        return o

    def host(self) -> dict:
        """Synchronise and copy the set (k entries), the merged frequencies
        left out of it (kd) and the n detections to numpy."""
        info = self.info.cpu().numpy()
        k, n, kd = int(info[0]), int(info[3]), int(info[4])
        freqs = self.freqs[:k + kd].cpu().numpy()
        amps = self.amps[:k + kd].cpu().numpy()
        return dict(k=k, iters=int(info[1]), status=int(info[2]), n=n, kd=kd,
                    freqs=freqs[:k], amps=amps[:k], dropped_freqs=freqs[k:], dropped_amps=amps[k:],
                    rec_iter=self.rec_iter[:n].cpu().numpy(), rec_bin=self.rec_bin[:n].cpu().numpy(),
                    rec_sin=self.rec_sin[:n].cpu().numpy())


class Plan:
    """A plan for a batch of cubes on the current CUDA (HIP) device."""

    def __init__(self, specs: Sequence[CubeSpec], tuning: Optional[dict] = None):
        self.specs = list(specs)
        descs = (B.Desc * len(self.specs))()
        keep = []
        for i, s in enumerate(self.specs):
            d, k = s.to_c()
            descs[i] = d
            keep.append(k)
        tn = None
        shapes = None
        if tuning:
            tn = B.Tuning()
            tn.block_threads = int(tuning.get("block_threads", 0))
            tn.max_radix = int(tuning.get("max_radix", 0))
            tn.chunk_iters = int(tuning.get("chunk_iters", -1))
            tn.lines_wg = int(tuning.get("lines_wg", 0))
            tn.lines_threads = int(tuning.get("lines_threads", 0))
            tn.direct_launch = int(tuning.get("direct_launch", 0))
            # an explicit lines_wg without lines_samples means lines_wg
            tn.lines_samples = int(tuning.get("lines_samples", -1 if "lines_wg" in tuning else 0))
            tn.group_by_length = int(tuning.get("group_by_length", 0))
            sh = tuning.get("shapes") or []
            # per-(D, L) launch shapes: {"ndim", "line_length", "block_threads",
            # "lines_samples"} (missing fields: plan-wide)
            shapes = (B.ShapeTuning * max(1, len(sh)))()
            for i, e in enumerate(sh):
                shapes[i].ndim = int(e["ndim"])
                shapes[i].line_length = int(e["line_length"])
                shapes[i].block_threads = int(e.get("block_threads", 0))
                shapes[i].lines_samples = int(e.get("lines_samples", 0))
            tn.nshapes = len(sh)
            tn.shapes = C.cast(shapes, C.POINTER(B.ShapeTuning))
        h = C.c_void_p()
        B.check(B.lib().fpssft_plan_create(descs, len(self.specs), C.byref(tn) if tn else None, C.byref(h)),
                "plan_create")
        self._h = h
        # kept with the plan: at interpreter exit the module's globals may be
        # gone before the plan is collected
        self._destroy = B.lib().fpssft_plan_destroy
        self.tuning = tuning
        self.info = []
        for c in range(len(self.specs)):
            L, T, off = C.c_int32(), C.c_int32(), C.c_int64()
            B.check(B.lib().fpssft_plan_cube_info(h, c, C.byref(L), C.byref(T), C.byref(off)), "cube_info")
            self.info.append((L.value, T.value, off.value))

    def __del__(self):
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self._h = None

    def close(self):
        self.__del__()

    # -- host queries ------------------------------------------------------
    def __len__(self):
        return len(self.specs)

    def line_length(self, cube: int) -> int:
        return self.info[cube][0]

    def max_iters(self, cube: int) -> int:
        return self.info[cube][1]

    def schedule(self, cube: int) -> np.ndarray:
        L, T, _ = self.info[cube]
        D = len(self.specs[cube].dims)
        out = np.zeros((T, 2, D), dtype=np.int32)
        B.check(B.lib().fpssft_plan_get_schedule(self._h, cube, out.ctypes.data_as(C.POINTER(C.c_int32))),
                "get_schedule")
        return out

    def spectra_elems(self) -> int:
        return int(B.lib().fpssft_plan_spectra_elems(self._h))

    # -- device calls ------------------------------------------------------
    def alloc_result(self, cube: int, device=None) -> Result:
        torch = _torch()
        s = self.specs[cube]
        dev = device or torch.device("cuda", torch.cuda.current_device())
        D = len(s.dims)
        return Result(freqs=torch.zeros((s.max_k, D), dtype=torch.int32, device=dev),
                      amps=torch.zeros(s.max_k, dtype=torch.complex64, device=dev),
                      rec_iter=torch.zeros(s.max_k, dtype=torch.int32, device=dev),
                      rec_bin=torch.zeros(s.max_k, dtype=torch.int32, device=dev),
                      rec_sin=torch.zeros(s.max_k, dtype=torch.int32, device=dev),
                      info=torch.zeros(B.INFO_LEN, dtype=torch.int32, device=dev))

    def _check_x(self, cube: int, x):
        torch = _torch()
        s = self.specs[cube]
        if not (x.is_cuda and x.dtype == torch.complex64 and x.is_contiguous()):
            raise ValueError("x must be a contiguous complex64 CUDA tensor")
        if tuple(x.shape) != tuple(int(v) for v in s.dims):
            raise ValueError(f"x has shape {tuple(x.shape)}, the plan expects {tuple(s.dims)}")

    def execute(self, cube: int, x, out: Optional[Result] = None, stream=None) -> Result:
        """Plain per-cube path (fpssft_execute)."""
        self._check_x(cube, x)
        out = out or self.alloc_result(cube, x.device)
        o = out.c_out()
        B.check(B.lib().fpssft_execute(self._h, cube, C.c_void_p(x.data_ptr()), C.byref(o),
                                       _stream_ptr(stream)), "execute")
        return out

    def execute_noalloc(self, cube: int, x, out: Result, stream=None) -> Result:
        """fpssft_execute_noalloc: the plain path with its scratch in the
        library's static device array (no device allocation in the call;
        the caller provides the outputs)."""
        self._check_x(cube, x)
        o = out.c_out()
        B.check(B.lib().fpssft_execute_noalloc(self._h, cube, C.c_void_p(x.data_ptr()), C.byref(o),
                                               _stream_ptr(stream)), "execute_noalloc")
        return out

    def execute_batched(self, xs, outs: Optional[Sequence[Result]] = None, stream=None):
        """All cubes in one persistent launch per kernel instantiation, replayed
        from a HIP graph or launched directly (fpssft_execute_batched)."""
        if len(xs) != len(self):
            raise ValueError("one input per cube")
        for c, x in enumerate(xs):
            self._check_x(c, x)
        outs = outs or [self.alloc_result(c, xs[c].device) for c in range(len(self))]
        ptrs = (C.c_void_p * len(self))(*[x.data_ptr() for x in xs])
        os_ = (B.Out * len(self))(*[o.c_out() for o in outs])
        B.check(B.lib().fpssft_execute_batched(self._h, ptrs, os_, _stream_ptr(stream)), "execute_batched")
        return outs

    def bind(self, xs, outs: Optional[Sequence[Result]] = None) -> "Bound":
        """Check the inputs once and keep the marshalled C arguments, so that
        repeated calls on the same tensors cost one C call each."""
        return Bound(self, xs, outs)

    def lines_fft(self, cube: int, x, t0: int, count: int, out=None, stream=None):
        """Line gather + 1/L-normalised DFT of iterations t0..t0+count-1:
        complex64 [count, D+1, L]."""
        torch = _torch()
        self._check_x(cube, x)
        L = self.line_length(cube)
        D = len(self.specs[cube].dims)
        if out is None:
            out = torch.empty((count, D + 1, L), dtype=torch.complex64, device=x.device)
        B.check(B.lib().fpssft_lines_fft(self._h, cube, C.c_void_p(x.data_ptr()), t0, count,
                                         C.c_void_p(out.data_ptr()), _stream_ptr(stream)), "lines_fft")
        return out

    def lines_fft_all(self, xs, out=None, stream=None):
        """Every cube's lines over its whole budget, packed (see info)."""
        torch = _torch()
        for c, x in enumerate(xs):
            self._check_x(c, x)
        if out is None:
            out = torch.empty(self.spectra_elems(), dtype=torch.complex64, device=xs[0].device)
        ptrs = (C.c_void_p * len(self))(*[x.data_ptr() for x in xs])
        B.check(B.lib().fpssft_lines_fft_all(self._h, ptrs, C.c_void_p(out.data_ptr()), _stream_ptr(stream)),
                "lines_fft_all")
        return out

    def amp_backward(self, cube: int, fwd: Result, grad_amps, grad_x=None, stream=None):
        """grad_x = M^H grad_amps for the amplitudes of a forward run."""
        torch = _torch()
        s = self.specs[cube]
        ga = grad_amps.to(torch.complex64).contiguous()
        if ga.numel() < s.max_k:
            ga = torch.nn.functional.pad(ga, (0, s.max_k - ga.numel()))
        if grad_x is None:
            grad_x = torch.empty(tuple(int(v) for v in s.dims), dtype=torch.complex64, device=ga.device)
        o = fwd.c_out()
        B.check(B.lib().fpssft_amp_backward(self._h, cube, C.byref(o), C.c_void_p(ga.data_ptr()),
                                            C.c_void_p(grad_x.data_ptr()), _stream_ptr(stream)), "amp_backward")
        return grad_x

    def amp_backward_batched(self, fwds: Sequence[Result], grad_amps, grad_xs=None, stream=None):
        torch = _torch()
        gas = []
        for c, g in enumerate(grad_amps):
            g = g.to(torch.complex64).contiguous()
            mk = self.specs[c].max_k
            if g.numel() < mk:
                g = torch.nn.functional.pad(g, (0, mk - g.numel()))
            gas.append(g)
        if grad_xs is None:
            grad_xs = [torch.empty(tuple(int(v) for v in s.dims), dtype=torch.complex64, device=gas[0].device)
                       for s in self.specs]
        os_ = (B.Out * len(self))(*[f.c_out() for f in fwds])
        gp = (C.c_void_p * len(self))(*[g.data_ptr() for g in gas])
        xp = (C.c_void_p * len(self))(*[g.data_ptr() for g in grad_xs])
        B.check(B.lib().fpssft_amp_backward_batched(self._h, os_, gp, xp, _stream_ptr(stream)),
                "amp_backward_batched")
        return grad_xs


class Bound:
    """A plan bound to fixed input and output tensors (see Plan.bind). The
    caller keeps the tensors alive and unchanged in shape while it is used."""

    def __init__(self, plan: Plan, xs, outs=None):
        if len(xs) != len(plan):
            raise ValueError("one input per cube")
        for c, x in enumerate(xs):
            plan._check_x(c, x)
        self.plan = plan
        self.xs = list(xs)
        self.outs = list(outs) if outs else [plan.alloc_result(c, xs[c].device) for c in range(len(plan))]
        self._xp = (C.c_void_p * len(plan))(*[x.data_ptr() for x in self.xs])
        self._op = (B.Out * len(plan))(*[o.c_out() for o in self.outs])
        self._x1 = [C.c_void_p(x.data_ptr()) for x in self.xs]
        self._o1 = [C.byref(self._op[c]) for c in range(len(plan))]
        self._fn_b = B.lib().fpssft_execute_batched
        self._fn_p = B.lib().fpssft_execute
        self._fn_l = B.lib().fpssft_lines_fft_all
        self.spectra = None

    def run_batched(self, stream=None):
        B.check(self._fn_b(self.plan._h, self._xp, self._op, _stream_ptr(stream)), "execute_batched")
        return self.outs

    def run_lines_all(self, stream=None):
        """fpssft_lines_fft_all into a packed spectra buffer owned here."""
        if self.spectra is None:
            torch = _torch()
            self.spectra = torch.empty(self.plan.spectra_elems(), dtype=torch.complex64,
                                       device=self.xs[0].device)
            self._sp = C.c_void_p(self.spectra.data_ptr())
        B.check(self._fn_l(self.plan._h, self._xp, self._sp, _stream_ptr(stream)), "lines_fft_all")
        return self.spectra

    def run_plain(self, cube: int, stream=None):
        B.check(self._fn_p(self.plan._h, cube, self._x1[cube], self._o1[cube], _stream_ptr(stream)), "execute")
        return self.outs[cube]

    def run_plain_all(self, stream=None):
        s = _stream_ptr(stream)
        h = self.plan._h
        fn = self._fn_p
        for c in range(len(self.xs)):
            st = fn(h, c, self._x1[c], self._o1[c], s)
            if st < 0:
                B.check(st, "execute")
        return self.outs

    def bind_backward(self, grad_amps, grad_xs=None):
        """Fix the amplitude cotangents (complex64 CUDA tensors of max_k
        entries, one per cube) and the gradient cubes for run_backward."""
        torch = _torch()
        if len(grad_amps) != len(self.plan):
            raise ValueError("one cotangent per cube")
        for c, g in enumerate(grad_amps):
            if not (g.is_cuda and g.dtype == torch.complex64 and g.is_contiguous()
                    and g.numel() == self.plan.specs[c].max_k):
                raise ValueError("grad_amps[c] must be a contiguous complex64 CUDA tensor of max_k entries")
        if grad_xs is None:
            grad_xs = [torch.empty_like(x) for x in self.xs]
        self.grad_amps, self.grad_xs = list(grad_amps), list(grad_xs)
        self._gp = (C.c_void_p * len(self.plan))(*[g.data_ptr() for g in self.grad_amps])
        self._gxp = (C.c_void_p * len(self.plan))(*[g.data_ptr() for g in self.grad_xs])
        self._fn_bw = B.lib().fpssft_amp_backward_batched
        return self.grad_xs

    def run_backward(self, stream=None):
        """fpssft_amp_backward_batched on the bound outputs, cotangents and
        gradient cubes (bind_backward first)."""
        B.check(self._fn_bw(self.plan._h, self._op, self._gp, self._gxp, _stream_ptr(stream)),
                "amp_backward_batched")
        return self.grad_xs


# ---------------------------------------------------------------------------
# Differentiable amplitudes
# ---------------------------------------------------------------------------

def _make_fn():
    torch = _torch()

    class AmpFn(torch.autograd.Function):
        """amps = FPS-SFT amplitudes of x; frequencies and the decision trace
        are returned as non-differentiable outputs and held fixed in the
        backward (the adjoint kernel)."""

        @staticmethod
        def forward(ctx, x, plan, cube):
            res = plan.execute(cube, x.detach())
            ctx.plan, ctx.cube, ctx.res = plan, cube, res
            ctx.mark_non_differentiable(res.freqs, res.info)
            return res.amps, res.freqs, res.info

        @staticmethod
        def backward(ctx, grad_amps, _gf, _gi):
            if grad_amps is None:
                return None, None, None
            gx = ctx.plan.amp_backward(ctx.cube, ctx.res, grad_amps)
            return gx, None, None

    class AmpBatchedFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, plan, *xs):
            res = plan.execute_batched([x.detach() for x in xs])
            ctx.plan, ctx.res = plan, res
            outs = []
            for r in res:
                ctx.mark_non_differentiable(r.freqs, r.info)
                outs += [r.amps, r.freqs, r.info]
            return tuple(outs)

        @staticmethod
        def backward(ctx, *grads):
            torch_ = _torch()
            gas = []
            for c, r in enumerate(ctx.res):
                g = grads[3 * c]
                gas.append(g if g is not None else torch_.zeros_like(r.amps))
            gxs = ctx.plan.amp_backward_batched(ctx.res, gas)
            return (None, *gxs)

    return AmpFn, AmpBatchedFn


_FNS = None


def _fns():
    global _FNS
    if _FNS is None:
        _FNS = _make_fn()
    return _FNS


def sft_amplitudes(plan: Plan, cube: int, x):
    """(amps [max_k] differentiable, freqs [max_k, D], info [8]) of one cube:
    the recovered set is amps[:k], freqs[:k] with k = info[0]."""
    return _fns()[0].apply(x, plan, cube)


def sft_amplitudes_batched(plan: Plan, xs):
    """Per cube (amps, freqs, info) of a batched forward; amps differentiable."""
    outs = _fns()[1].apply(plan, *xs)
    return [tuple(outs[3 * c:3 * c + 3]) for c in range(len(xs))]
