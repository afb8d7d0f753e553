"""FP64 CPU oracle for the batched manifold projection (test infrastructure only).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg may
import this package. The HIP library never loads it, and it shares no code with
the HIP path. The arithmetic lives in ``oracle.cpp`` (plain scalar C++17,
OpenMP over configurations); this module is argument marshalling.

All configuration arrays here are row-major ``[n, d]`` float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

CONVERGED, MAX_ITER, SINGULAR, DIVERGED, NONFINITE = range(5)


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.oracle_scene_info.argtypes = [P, ctypes.c_size_t, P]
        L.oracle_link_frames.argtypes = [P, ctypes.c_size_t, P, P]
        L.oracle_frame_poses.argtypes = [P, ctypes.c_size_t, P, P]
        L.oracle_so3_log.argtypes = [P, P]
        L.oracle_so3_log.restype = None
        L.oracle_residual.argtypes = [P, ctypes.c_size_t, ctypes.c_int64, P, P, ctypes.c_int]
        L.oracle_jacobian.argtypes = [P, ctypes.c_size_t, ctypes.c_int64, P, P, ctypes.c_int]
        L.oracle_project.argtypes = [P, ctypes.c_size_t, ctypes.c_int64, P, P, P, P, P, ctypes.c_double,
                                     ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, P,
                                     ctypes.c_int]
        L.oracle_check.argtypes = [P, ctypes.c_size_t, ctypes.c_int64, P, P, P, ctypes.c_int]
        L.oracle_vjp.argtypes = [P, ctypes.c_size_t, ctypes.c_int64, P, P, P, P, P, ctypes.c_int]
        L.oracle_path_length.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_int32, P, P]
        L.oracle_kappa_est.argtypes = [P, ctypes.c_size_t, ctypes.c_int64, P, ctypes.c_double, P, P, ctypes.c_int]
        L.oracle_vjp_exact.argtypes = [P, ctypes.c_size_t, ctypes.c_int64, P, P, P, ctypes.c_double, ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_double, P, ctypes.c_int]
        L.oracle_max_threads.argtypes = []
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Problem:
    """A parsed scene blob (kept as bytes; the C++ side re-parses it per call)."""

    def __init__(self, blob: bytes):
        self.blob = bytes(blob)
        self._buf = ctypes.create_string_buffer(self.blob, len(self.blob))
        info = np.zeros(8, np.int32)
        rc = lib().oracle_scene_info(self._buf, len(self.blob), _p(info))
        if rc != 0:
            raise ValueError("oracle: invalid scene blob")
        (self.family, self.d, self.m, self.n_joints, self.n_frames, self.n_blocks,
         self.n_spheres, self.n_obstacles) = [int(x) for x in info]

    def _args(self):
        return self._buf, len(self.blob)

    def link_frames(self, q):
        q = np.ascontiguousarray(q, np.float64).reshape(self.d)
        out = np.zeros((self.n_joints, 12))
        assert lib().oracle_link_frames(*self._args(), _p(q), _p(out)) == 0
        return out

    def frame_poses(self, q):
        q = np.ascontiguousarray(q, np.float64).reshape(self.d)
        out = np.zeros((self.n_frames, 12))
        assert lib().oracle_frame_poses(*self._args(), _p(q), _p(out)) == 0
        return out

    def residual(self, q, threads: int = 0):
        q = np.ascontiguousarray(q, np.float64).reshape(-1, self.d)
        F = np.zeros((q.shape[0], self.m))
        assert lib().oracle_residual(*self._args(), q.shape[0], _p(q), _p(F), threads) == 0
        return F

    def jacobian(self, q, threads: int = 0):
        q = np.ascontiguousarray(q, np.float64).reshape(-1, self.d)
        J = np.zeros((q.shape[0], self.m, self.d))
        assert lib().oracle_jacobian(*self._args(), q.shape[0], _p(q), _p(J), threads) == 0
        return J

    def project(self, q, tol=1e-6, max_iter=50, alpha=1.0, lam=0.0, max_step=0.0, threads: int = 0,
                path_info: bool = False, mode: str = "stacked"):
        """Returns (q_out, status, iters, resid) and, with path_info, an [n, 4] path record: the
        smallest sigma_min(J) along each path, its longest step (the longest iteration displacement
        in cyclic mode), the largest rotation angle of a pose error at any residual evaluation, and
        the smallest multiplicative distance max(||F|| / tol, tol / ||F||) of a convergence test to
        the tolerance. mode: "stacked" (one system per step) or "cyclic" (one step per constraint
        block, in order)."""
        q = np.ascontiguousarray(q, np.float64).reshape(-1, self.d)
        n = q.shape[0]
        qo = np.zeros_like(q)
        st = np.zeros(n, np.int8)
        it = np.zeros(n, np.int32)
        rs = np.zeros(n, np.float64)
        pi = np.zeros((n, 4)) if path_info else None
        rc = lib().oracle_project(*self._args(), n, _p(q), _p(qo), _p(st), _p(it), _p(rs), float(tol),
                                  int(max_iter), float(alpha), float(lam), float(max_step), threads,
                                  None if pi is None else _p(pi), {"stacked": 0, "cyclic": 1}[mode])
        if rc != 0:
            raise ValueError("oracle_project failed (%d)" % rc)
        return (qo, st, it, rs, pi) if path_info else (qo, st, it, rs)

    def check(self, q, threads: int = 0):
        q = np.ascontiguousarray(q, np.float64).reshape(-1, self.d)
        v = np.zeros(q.shape[0], np.uint8)
        sd = np.zeros(q.shape[0], np.float64)
        assert lib().oracle_check(*self._args(), q.shape[0], _p(q), _p(v), _p(sd), threads) == 0
        return v, sd

    def vjp(self, q, g, status=None, threads: int = 0):
        q = np.ascontiguousarray(q, np.float64).reshape(-1, self.d)
        g = np.ascontiguousarray(g, np.float64).reshape(-1, self.d)
        n = q.shape[0]
        gi = np.zeros_like(q)
        kap = np.zeros(n)
        st = None if status is None else np.ascontiguousarray(status, np.int8)
        assert lib().oracle_vjp(*self._args(), n, _p(q), None if st is None else _p(st), _p(g), _p(gi),
                                _p(kap), threads) == 0
        return gi, kap

    def vjp_exact(self, q0, g, tol=1e-13, max_iter=100, alpha=1.0, lam=0.0, threads: int = 0):
        """(g_in, status): g_in = (dP/dq0)^T g, the derivative of the projection map at the (possibly
        off-manifold) inputs q0, by forward-mode dual numbers through every Newton step run to tol."""
        q0 = np.ascontiguousarray(q0, np.float64).reshape(-1, self.d)
        g = np.ascontiguousarray(g, np.float64).reshape(-1, self.d)
        gi = np.zeros_like(q0)
        st = np.zeros(len(q0), np.int8)
        rc = lib().oracle_vjp_exact(*self._args(), len(q0), _p(q0), _p(g), _p(gi), float(tol), int(max_iter),
                                    float(alpha), float(lam), _p(st), threads)
        if rc == 3:
            raise NotImplementedError("oracle: no dual-number derivative for scenes with bounded or polygon rows")
        assert rc == 0
        return gi, st

    def kappa_est(self, q, lam=0.0, threads: int = 0):
        """(kappa_est, kappa2) per configuration: (max L_ii / min L_ii)^2 of the FP64 Cholesky factor
        of J J^T + lam I (+inf when a pivot is not positive), and (sigma_max / sigma_min)^2 of J."""
        q = np.ascontiguousarray(q, np.float64).reshape(-1, self.d)
        ke = np.zeros(q.shape[0])
        k2 = np.zeros(q.shape[0])
        assert lib().oracle_kappa_est(*self._args(), q.shape[0], _p(q), float(lam), _p(ke), _p(k2), threads) == 0
        return ke, k2


def so3_log(R):
    R = np.ascontiguousarray(R, np.float64).reshape(9)
    w = np.zeros(3)
    lib().oracle_so3_log(_p(R), _p(w))
    return w


def path_length(q, geo_offsets):
    q = np.ascontiguousarray(q, np.float64)
    n, d = q.shape
    offs = np.ascontiguousarray(geo_offsets, np.int32)
    g = np.zeros_like(q)
    L = np.zeros(1)
    assert lib().oracle_path_length(n, d, _p(q), _p(offs), len(offs) - 1, _p(g), _p(L)) == 0
    return float(L[0]), g


def interpolate_interior(endpoints, geo_offsets):
    """Interior points t_k = k/(n+1), k = 1..n, on the chord between two endpoints of every geodesic
    (the interpolation step of Alg. 2); endpoints [n_geo, 2, d]."""
    e = np.asarray(endpoints, np.float64)
    offs = np.asarray(geo_offsets)
    out = []
    for g in range(len(offs) - 1):
        n = int(offs[g + 1] - offs[g])
        t = np.arange(1, n + 1) / (n + 1)
        out.append(e[g, 0][None, :] + t[:, None] * (e[g, 1] - e[g, 0])[None, :])
    return np.concatenate(out, 0) if out else np.zeros((0, e.shape[-1]))


def max_threads() -> int:
    return int(lib().oracle_max_threads())
