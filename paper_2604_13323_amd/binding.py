"""ctypes binding of libmcproj (the HIP library); argument marshalling only.

Configuration batches are torch tensors of shape [d, N] (structure of arrays: row c
holds coordinate c of every configuration), float32 or float64, on the current HIP
device. Every call is enqueued on torch's current stream. All arithmetic happens in
the library's kernels; this module never computes on the data.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcproj.so")

MC_F32, MC_F64 = 0, 1
CONVERGED, MAX_ITER, SINGULAR, DIVERGED, NONFINITE = range(5)
FREE, COLLIDES, UNCHECKED = 0, 1, 2
VARIANTS = {"auto": 0, "plain": 1, "fused": 2}
(EXT_OK, EXT_ZERO, EXT_NO_PARTICLE, EXT_COLLISION, EXT_TOO_FAR, EXT_INTERP_FAILED, EXT_INTERP_COLLISION,
 EXT_GAP) = range(8)


class McError(RuntimeError):
    pass


class Opts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("lambda_", ctypes.c_double), ("max_step", ctypes.c_double),
                ("fp64_cond_threshold", ctypes.c_double), ("check_collision", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("waves_per_block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("lanes_per_config", ctypes.c_int32), ("step_form", ctypes.c_int32)]


class LaunchShape(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("lanes_per_config", ctypes.c_int32), ("check_lanes", ctypes.c_int32)]

    def as_dict(self):
        return dict(waves_per_block=self.waves_per_block, blocks_per_cu=self.blocks_per_cu,
                    lanes_per_config=self.lanes_per_config, check_lanes=self.check_lanes)


class ExtendOpts(ctypes.Structure):
    _fields_ = [("r", ctypes.c_double), ("delta", ctypes.c_double), ("n", ctypes.c_int32)]


_lib = None

EXPORTS = ["mc_default_opts", "mc_problem_create", "mc_problem_destroy", "mc_problem_dof", "mc_problem_rows",
           "mc_problem_family", "mc_last_error", "project_batch", "check_batch", "project_vjp",
           "interpolate_geodesics", "path_length_grad", "mc_eval_residual_jacobian", "mc_fallback_count", "extend_batch",
           "mc_eval_condition", "mc_queue_counts", "mc_autotune_candidates", "mc_autotune_project", "mc_tuned_shape",
           "mc_set_kernel_timing", "mc_last_kernel_ms", "project_batch_noalloc", "project_vjp_exact",
           "mc_set_check_lanes"]


def lib():
    """Load libmcproj.so. Raises when it has not been built: there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise McError(f"HIP library {LIB_PATH} is missing: build it first (python -m paper_2604_13323_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.mc_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.mc_default_opts.restype = None
    L.mc_problem_create.argtypes = [P, ctypes.c_size_t, ctypes.POINTER(P)]
    L.mc_problem_destroy.argtypes = [P]
    L.mc_problem_destroy.restype = None
    for f in ("mc_problem_dof", "mc_problem_rows", "mc_problem_family"):
        getattr(L, f).argtypes = [P]
        getattr(L, f).restype = I32
    L.mc_last_error.argtypes = []
    L.mc_last_error.restype = ctypes.c_char_p
    L.project_batch.argtypes = [P, I64, P, I64, P, I64, P, P, P, P, P, P, I32, P, ctypes.POINTER(Opts), P]
    L.project_batch_noalloc.argtypes = L.project_batch.argtypes
    L.check_batch.argtypes = [P, I64, P, I64, ctypes.c_int, P, P, P]
    L.project_vjp.argtypes = [P, I64, P, I64, P, P, P, ctypes.POINTER(Opts), P]
    L.project_vjp_exact.argtypes = [P, I64, P, I64, P, P, P, P, ctypes.POINTER(Opts), P]
    L.interpolate_geodesics.argtypes = [P, I32, P, P, I64, I64, P, I64, ctypes.c_int, P]
    L.path_length_grad.argtypes = [P, I64, P, I64, P, I32, P, P, ctypes.c_int, P]
    L.mc_eval_residual_jacobian.argtypes = [P, I64, P, I64, ctypes.c_int, P, P, P]
    L.mc_fallback_count.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]
    L.extend_batch.argtypes = [P, I64, P, P, I64, P, ctypes.POINTER(ExtendOpts), ctypes.POINTER(Opts), P, I64, P, P,
                               P, P]
    L.mc_eval_condition.argtypes = [P, I64, P, I64, ctypes.c_int, ctypes.c_double, P, P]
    L.mc_queue_counts.argtypes = [P, ctypes.POINTER(ctypes.c_uint32)]
    L.mc_autotune_candidates.argtypes = [ctypes.POINTER(LaunchShape)]
    L.mc_autotune_candidates.restype = I32
    L.mc_autotune_project.argtypes = [P, I64, P, I64, ctypes.POINTER(Opts), I32, P, ctypes.POINTER(LaunchShape),
                                      ctypes.POINTER(ctypes.c_float)]
    L.mc_tuned_shape.argtypes = [P, ctypes.c_int, I32, ctypes.POINTER(LaunchShape)]
    L.mc_set_kernel_timing.argtypes = [P, I32]
    L.mc_set_check_lanes.argtypes = [P, I32]
    L.mc_last_kernel_ms.argtypes = [P, I32, ctypes.POINTER(ctypes.c_float)]
    for f in EXPORTS:
        if f not in ("mc_default_opts", "mc_problem_destroy", "mc_problem_dof", "mc_problem_rows",
                     "mc_problem_family", "mc_last_error", "mc_autotune_candidates"):
            getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != 0:
        raise McError(f"{what} failed ({rc}): {lib().mc_last_error().decode()}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return MC_F32
    if t.dtype == torch.float64:
        return MC_F64
    raise McError(f"unsupported dtype {t.dtype}")


def _soa(q: torch.Tensor, d: int, name: str):
    if q.dim() != 2 or q.shape[0] != d:
        raise McError(f"{name}: expected shape [{d}, N], got {tuple(q.shape)}")
    if not q.is_cuda:
        raise McError(f"{name}: expected a device tensor")
    if q.stride(1) != 1 and q.shape[1] > 1:
        raise McError(f"{name}: rows must be contiguous")
    return q.shape[1], max(q.stride(0), q.shape[1])  # a single column's strides are arbitrary


MODES = {"stacked": 0, "cyclic": 1}
STEP_FORMS = {"inner": 0, "outer": 1}


def make_opts(dtype=MC_F32, tol=1e-6, max_iter=50, alpha=1.0, lam=0.0, max_step=0.0, cond=1e6, check=True,
              variant="auto", waves_per_block=0, blocks_per_cu=0, mode="stacked", lanes_per_config=0,
              step_form="inner") -> Opts:
    o = Opts()
    lib().mc_default_opts(ctypes.byref(o))
    o.dtype = dtype
    o.tol = tol
    o.max_iter = max_iter
    o.alpha = alpha
    o.lambda_ = lam
    o.max_step = max_step
    o.fp64_cond_threshold = cond
    o.check_collision = 1 if check else 0
    o.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    o.waves_per_block = waves_per_block
    o.blocks_per_cu = blocks_per_cu
    o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    o.lanes_per_config = lanes_per_config
    o.step_form = STEP_FORMS[step_form] if isinstance(step_form, str) else int(step_form)
    return o


@dataclass
class ExtendResult:
    q: torch.Tensor          # [d, E] q_proj of the selected particle (where particle >= 0)
    result: torch.Tensor     # int8 [E], EXT_*
    particle: torch.Tensor   # int32 [E], selected particle or -1
    n_points: torch.Tensor   # int32 [E], points of the validated chain (EXT_OK)


@dataclass
class ProjectResult:
    q: torch.Tensor
    status: torch.Tensor
    iters: torch.Tensor
    resid: torch.Tensor
    verdict: torch.Tensor | None
    geo_ok: torch.Tensor | None


class Problem:
    """A scene on the current HIP device (wraps mc_problem)."""

    def __init__(self, blob: bytes):
        self._blob = ctypes.create_string_buffer(bytes(blob), len(blob))
        h = ctypes.c_void_p()
        _check(lib().mc_problem_create(self._blob, len(blob), ctypes.byref(h)), "mc_problem_create")
        self._h = h
        self.d = int(lib().mc_problem_dof(h))
        self.m = int(lib().mc_problem_rows(h))
        self.family = int(lib().mc_problem_family(h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            try:
                torch.cuda.synchronize()
            except Exception:
                pass
            _lib.mc_problem_destroy(h)
            self._h = None

    # -- projection -------------------------------------------------------
    def project(self, q: torch.Tensor, tol=1e-6, max_iter=50, alpha=1.0, lam=0.0, max_step=0.0, cond=1e6,
                check=True, variant="auto", geo_offsets=None, geo_ok=False, waves_per_block=0, blocks_per_cu=0,
                out: ProjectResult | None = None, geo_offsets_host=None, mode="stacked",
                lanes_per_config=0, noalloc=False, step_form="inner") -> ProjectResult:
        """Project the columns of q ([d, n], float32 or float64). geo_offsets (CSR, int32) may be a host array
        or a device tensor; the plain variant also needs them on the host (geo_offsets_host, or a host
        geo_offsets). Under stream capture pass device offsets, `out`, and call once eagerly beforehand with a
        batch at least as large (that sizes the library's work queues). noalloc=True calls project_batch_noalloc (the
        library's fixed scratch array instead of the problem's grown queues: nothing is allocated)."""
        n, ld = _soa(q, self.d, "project")
        dt = _dtype_code(q)
        dev = q.device
        if out is None:
            out = ProjectResult(q=torch.empty((self.d, n), dtype=q.dtype, device=dev),
                                status=torch.empty(n, dtype=torch.int8, device=dev),
                                iters=torch.empty(n, dtype=torch.int8, device=dev),
                                resid=torch.empty(n, dtype=q.dtype, device=dev),
                                verdict=torch.empty(n, dtype=torch.uint8, device=dev),
                                geo_ok=None)
        offs_dev, offs_host, n_geo = None, None, 0
        if geo_offsets_host is not None:
            offs_host = np.ascontiguousarray(np.asarray(geo_offsets_host, dtype=np.int32))
            n_geo = len(offs_host) - 1
        if geo_offsets is not None:
            if isinstance(geo_offsets, torch.Tensor) and geo_offsets.is_cuda:
                offs_dev = geo_offsets
                n_geo = geo_offsets.numel() - 1
            else:
                offs_np = np.ascontiguousarray(np.asarray(geo_offsets, dtype=np.int32))
                n_geo = len(offs_np) - 1
                if offs_host is None:
                    offs_host = offs_np
                offs_dev = torch.from_numpy(offs_np).to(dev)
            out._offs = offs_dev  # keep alive while the stream runs
            if geo_ok and out.geo_ok is None:
                out.geo_ok = torch.empty(n_geo, dtype=torch.uint8, device=dev)
        o = make_opts(dt, tol, max_iter, alpha, lam, max_step, cond, check, variant, waves_per_block, blocks_per_cu,
                      mode, lanes_per_config, step_form)
        fn = lib().project_batch_noalloc if noalloc else lib().project_batch
        rc = fn(self._h, n, _ptr(q), ld, _ptr(out.q), out.q.stride(0), _ptr(out.status),
                                 _ptr(out.iters), _ptr(out.resid), _ptr(out.verdict), _ptr(offs_dev),
                                 None if offs_host is None else offs_host.ctypes.data_as(ctypes.c_void_p),
                                 n_geo, _ptr(out.geo_ok) if geo_ok else None, ctypes.byref(o), _stream())
        _check(rc, "project_batch_noalloc" if noalloc else "project_batch")
        return out

    def extend(self, q_start: torch.Tensor, q_target: torch.Tensor, eps: torch.Tensor, r: float, delta: float,
               tol=1e-6, max_iter=50, max_step=0.0, cond=1e6, mode="stacked", waves_per_block=0,
               blocks_per_cu=0) -> ExtendResult:
        """ConstrainedExtend for E extensions: q_start, q_target [d, E] (same dtype and strides), eps [E, n] the
        particle offsets along the extension direction (the N(0, sigma^2) draws)."""
        E, ld = _soa(q_start, self.d, "extend")
        if q_target.shape != q_start.shape or q_target.stride() != q_start.stride() or q_target.dtype != q_start.dtype:
            raise McError("extend: q_target must match q_start in shape, strides and dtype")
        if eps.dim() != 2 or eps.shape[0] != E or not eps.is_contiguous() or eps.dtype != q_start.dtype:
            raise McError("extend: eps must be a contiguous [E, n] tensor of q_start's dtype")
        n = eps.shape[1]
        dev = q_start.device
        out = ExtendResult(q=torch.empty((self.d, E), dtype=q_start.dtype, device=dev),
                           result=torch.empty(E, dtype=torch.int8, device=dev),
                           particle=torch.empty(E, dtype=torch.int32, device=dev),
                           n_points=torch.empty(E, dtype=torch.int32, device=dev))
        xo = ExtendOpts(r=float(r), delta=float(delta), n=int(n))
        o = make_opts(_dtype_code(q_start), tol, max_iter, max_step=max_step, cond=cond, mode=mode,
                      waves_per_block=waves_per_block, blocks_per_cu=blocks_per_cu)
        _check(lib().extend_batch(self._h, E, _ptr(q_start), _ptr(q_target), ld, _ptr(eps), ctypes.byref(xo),
                                  ctypes.byref(o), _ptr(out.q), out.q.stride(0), _ptr(out.result), _ptr(out.particle),
                                  _ptr(out.n_points), _stream()), "extend_batch")
        return out

    def check(self, q: torch.Tensor, min_signed_dist=False):
        n, ld = _soa(q, self.d, "check")
        v = torch.empty(n, dtype=torch.uint8, device=q.device)
        sd = torch.empty(n, dtype=q.dtype, device=q.device) if min_signed_dist else None
        _check(lib().check_batch(self._h, n, _ptr(q), ld, _dtype_code(q), _ptr(v), _ptr(sd), _stream()), "check_batch")
        return (v, sd) if min_signed_dist else v

    def vjp(self, q_proj: torch.Tensor, status: torch.Tensor, g_out: torch.Tensor, cond=1e6):
        """g_in [d, n] of q_proj's dtype; q_proj, g_out and g_in share one leading dimension (g_in is
        allocated with q_proj's strides, so a column slice of a wider array is handled in place)."""
        n, ld = _soa(q_proj, self.d, "vjp")
        if g_out.shape != q_proj.shape or g_out.stride() != q_proj.stride() or g_out.dtype != q_proj.dtype:
            g_out = g_out.to(q_proj.dtype).contiguous()
            q_proj = q_proj.contiguous()
            ld = q_proj.stride(0)
        g_in = torch.empty_strided(q_proj.shape, q_proj.stride(), dtype=q_proj.dtype, device=q_proj.device)
        o = make_opts(_dtype_code(q_proj), cond=cond)
        _check(lib().project_vjp(self._h, n, _ptr(q_proj), ld, _ptr(status), _ptr(g_out), _ptr(g_in),
                                 ctypes.byref(o), _stream()), "project_vjp")
        return g_in

    def vjp_exact(self, q_in: torch.Tensor, status: torch.Tensor, iters: torch.Tensor, g_out: torch.Tensor,
                  alpha=1.0, lam=0.0):
        """Exact VJP of the projection map at the forward call's inputs q_in (with its status and iters):
        g_in [d, n] with q_in's strides."""
        n, ld = _soa(q_in, self.d, "vjp_exact")
        if g_out.shape != q_in.shape or g_out.stride() != q_in.stride() or g_out.dtype != q_in.dtype:
            g_out = g_out.to(q_in.dtype).contiguous()
            q_in = q_in.contiguous()
            ld = q_in.stride(0)
        g_in = torch.empty_strided(q_in.shape, q_in.stride(), dtype=q_in.dtype, device=q_in.device)
        o = make_opts(_dtype_code(q_in), alpha=alpha, lam=lam)
        _check(lib().project_vjp_exact(self._h, n, _ptr(q_in), ld, _ptr(status), _ptr(iters), _ptr(g_out), _ptr(g_in),
                                       ctypes.byref(o), _stream()), "project_vjp_exact")
        return g_in

    def interpolate(self, endpoints: torch.Tensor, geo_offsets: torch.Tensor, total: int):
        """endpoints [d, 2 n_geo] (columns 2g, 2g+1 = the two ends); geo_offsets int32 device [n_geo + 1];
        total = geo_offsets[n_geo] (known to the caller, so nothing is read back from the device)."""
        n_geo = geo_offsets.numel() - 1
        out = torch.empty((self.d, total), dtype=endpoints.dtype, device=endpoints.device)
        _check(lib().interpolate_geodesics(self._h, n_geo, _ptr(geo_offsets), _ptr(endpoints), endpoints.stride(0),
                                           int(total), _ptr(out), out.stride(0), _dtype_code(endpoints), _stream()),
               "interpolate_geodesics")
        return out

    def path_length_grad(self, q: torch.Tensor, geo_offsets: torch.Tensor, with_loss=True):
        """Gradient [d, n] with q's strides (the library writes it with q's leading dimension)."""
        n, ld = _soa(q, self.d, "path_length_grad")
        g = torch.empty_strided(q.shape, q.stride(), dtype=q.dtype, device=q.device)
        loss = torch.empty(1, dtype=q.dtype, device=q.device) if with_loss else None
        _check(lib().path_length_grad(self._h, n, _ptr(q), ld, _ptr(geo_offsets), geo_offsets.numel() - 1, _ptr(g),
                                      _ptr(loss), _dtype_code(q), _stream()), "path_length_grad")
        return g, loss

    def eval_fj(self, q: torch.Tensor):
        n, ld = _soa(q, self.d, "eval_fj")
        F = torch.empty((self.m, n), dtype=q.dtype, device=q.device)
        J = torch.empty((self.m * self.d, n), dtype=q.dtype, device=q.device)
        if ld != n:
            q = q.contiguous()
        _check(lib().mc_eval_residual_jacobian(self._h, n, _ptr(q), n, _dtype_code(q), _ptr(F), _ptr(J), _stream()),
               "mc_eval_residual_jacobian")
        return F, J

    def condition(self, q: torch.Tensor, lam=0.0):
        """The kernels' condition estimate (max L_ii / min L_ii)^2 of J J^T + lam I at every column of q
        (+inf where the factorisation fails), in q's precision mode."""
        n, ld = _soa(q, self.d, "condition")
        k = torch.empty(n, dtype=q.dtype, device=q.device)
        _check(lib().mc_eval_condition(self._h, n, _ptr(q), ld, _dtype_code(q), float(lam), _ptr(k), _stream()),
               "mc_eval_condition")
        return k

    def queue_counts(self):
        """[taken beyond the static share, FP64 projections, FP64 VJPs, exact collision checks] of the last calls."""
        c = (ctypes.c_uint32 * 4)()
        _check(lib().mc_queue_counts(self._h, c), "mc_queue_counts")
        return [int(x) for x in c]

    def autotune(self, q: torch.Tensor, reps=5, tol=1e-6, max_iter=50, cond=1e6, check=True, mode="stacked", **kw):
        """The library's launch-shape autotuner on batch q; returns (best shape, [(shape, ms)])."""
        n, ld = _soa(q, self.d, "autotune")
        o = make_opts(_dtype_code(q), tol, max_iter, cond=cond, check=check, mode=mode, **kw)
        nc = lib().mc_autotune_candidates(None)
        shapes = (LaunchShape * nc)()
        lib().mc_autotune_candidates(shapes)
        ms = (ctypes.c_float * nc)()
        best = LaunchShape()
        _check(lib().mc_autotune_project(self._h, n, _ptr(q), ld, ctypes.byref(o), int(reps), _stream(),
                                         ctypes.byref(best), ms), "mc_autotune_project")
        return best.as_dict(), [(shapes[c].as_dict(), float(ms[c])) for c in range(nc)]

    def tuned_shape(self, dtype=torch.float32, mode="stacked"):
        """The shape the autotuner stored for (dtype, mode), or None."""
        out = LaunchShape()
        rc = lib().mc_tuned_shape(self._h, MC_F64 if dtype == torch.float64 else MC_F32, MODES[mode], ctypes.byref(out))
        return out.as_dict() if rc == 0 else None

    def set_check_lanes(self, lanes=0):
        """Lanes per configuration of the exact collision check (0: by queue length; 1, 2, 4, 8, 16, 64)."""
        _check(lib().mc_set_check_lanes(self._h, int(lanes)), "mc_set_check_lanes")

    def kernel_timing(self, on=True):
        """Bracket the main projection and VJP launches with HIP events (see last_kernel_ms)."""
        _check(lib().mc_set_kernel_timing(self._h, 1 if on else 0), "mc_set_kernel_timing")

    def last_kernel_ms(self, which="projection") -> float:
        """Duration of the main kernel launch of the last timed project (or vjp) call; waits for it."""
        ms = ctypes.c_float()
        _check(lib().mc_last_kernel_ms(self._h, {"projection": 0, "vjp": 1}[which], ctypes.byref(ms)),
               "mc_last_kernel_ms")
        return float(ms.value)

    def fallback_count(self, reset=False) -> int:
        c = ctypes.c_uint64()
        _check(lib().mc_fallback_count(self._h, 1 if reset else 0, ctypes.byref(c)), "mc_fallback_count")
        return int(c.value)


class ProjectFn(torch.autograd.Function):
    """q_proj = P(q_in); backward gives (I - J^+ J) g at q_proj (implicit differentiation at
    convergence; only q_proj and status are saved, the backward kernel recomputes the kinematics
    and the Jacobian), or with exact=True the exact derivative of the map at q_in (q_in, status and
    iters saved; the backward kernel replays the steps)."""

    @staticmethod
    def forward(ctx, q_in: torch.Tensor, problem: Problem, kwargs: dict):
        kwargs = dict(kwargs)
        exact = kwargs.pop("exact", False)
        r = problem.project(q_in.detach(), **kwargs)
        ctx.problem = problem
        ctx.cond = kwargs.get("cond", 1e6)
        ctx.exact = exact
        ctx.step = (kwargs.get("alpha", 1.0), kwargs.get("lam", 0.0))
        if exact:
            ctx.save_for_backward(q_in.detach(), r.status, r.iters)
        else:
            ctx.save_for_backward(r.q, r.status)
        ctx.mark_non_differentiable(r.status)
        return r.q, r.status

    @staticmethod
    def backward(ctx, g_q, g_status):
        if ctx.exact:
            q_in, status, iters = ctx.saved_tensors
            g_in = ctx.problem.vjp_exact(q_in, status, iters, g_q.contiguous(), alpha=ctx.step[0], lam=ctx.step[1])
        else:
            q, status = ctx.saved_tensors
            g_in = ctx.problem.vjp(q, status, g_q.contiguous(), cond=ctx.cond)
        return g_in, None, None


def project(q_in: torch.Tensor, problem: Problem, **kwargs):
    """Differentiable projection: returns (q_proj, status)."""
    return ProjectFn.apply(q_in, problem, kwargs)


class PathLengthFn(torch.autograd.Function):
    """Path length summed over geodesics (CSR offsets); gradient from the library kernel."""

    @staticmethod
    def forward(ctx, q: torch.Tensor, problem: Problem, geo_offsets: torch.Tensor):
        g, loss = problem.path_length_grad(q.detach(), geo_offsets)
        ctx.save_for_backward(g)
        return loss[0]

    @staticmethod
    def backward(ctx, gl):
        (g,) = ctx.saved_tensors
        return g * gl, None, None
