"""CPU oracle for the loop-of-stencil-reduce pattern -- test infrastructure only.

Thin ctypes wrapper over ``liblsr_oracle.so`` (built from ``lsr_oracle.c`` by
``oracle/build.py``). Only the tests, the smoke check and the benchmark's CPU
baseline leg use it; the GPU library neither imports nor links it.

Parity unpinned by the paper: the restoration functional phi(t) = sqrt(beta+t^2),
beta, the detection bound w_max and the adaptive-median edge rules. They are
pinned by closed forms (affine and constant fixed points, the quadratic form's
neighbour mean) and brute force on small images, not by any number the paper
prints.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsr_oracle.so")

RED_MAX_ABS_DELTA, RED_L2_DELTA, RED_SUM, RED_MEAN_ABS_DELTA = 1, 2, 3, 4
COND_BELOW, COND_STABLE_FOR, COND_NEVER = 1, 2, 3
BC_RING, BC_TORUS, BC_BOTTOM = 0, 1, 2


class _Res(C.Structure):
    _fields_ = [("n", C.c_int64), ("r", C.c_double), ("count", C.c_uint64),
                ("converged", C.c_int32), ("run", C.c_int32), ("checks", C.c_int64),
                ("numeric_error", C.c_int32), ("pad", C.c_int32)]


@dataclass
class OracleResult:
    n: int
    r: float
    count: int
    converged: bool
    run: int
    checks: int
    numeric_error: bool
    trace: np.ndarray


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle.build import build
            build()
        lib = C.CDLL(LIB_PATH)
        P = C.c_void_p
        lib.orc_jacobi_run.argtypes = [C.c_int, P, P, C.c_int64, C.c_int64, C.c_double, C.c_double,
                                       C.c_int, C.c_int, C.c_double, C.c_int, C.c_int64, P,
                                       C.c_int64, C.POINTER(_Res)]
        lib.orc_life_run.argtypes = [P, C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int,
                                     C.c_int64, P, C.c_int64, C.POINTER(_Res)]
        lib.orc_amf_detect.argtypes = [P, C.c_int64, C.c_int64, C.c_int, P, P]
        lib.orc_restore_run.argtypes = [P, P, C.c_int64, C.c_int64, C.c_double, C.c_int, C.c_int,
                                        C.c_int, C.c_double, C.c_int, C.c_int64, P, C.c_int64,
                                        C.POINTER(_Res)]
        lib.orc_jacobi_sep_run.argtypes = [P, P, P, C.c_double, C.c_double, C.c_int64, C.c_int64,
                                           C.c_double, C.c_double, C.c_int, C.c_int, C.c_double,
                                           C.c_int, C.c_int64, P, C.c_int64, C.POINTER(_Res)]
        lib.orc_box_run.argtypes = [P, C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_double,
                                    C.c_int, C.c_int64, P, C.c_int64, C.POINTER(_Res)]
        lib.orc_jacobi3d_run.argtypes = [P, C.c_int64, C.c_int64, C.c_int64, C.c_int, C.c_int,
                                         C.c_double, C.c_int, C.c_int64, P, C.c_int64,
                                         C.POINTER(_Res)]
        lib.orc_sobel_run.argtypes = [P, C.c_int64, C.c_int64, C.c_int, C.c_int64, P, C.c_int64,
                                      C.POINTER(_Res)]
        lib.orc_restore_argmin.argtypes = [P, C.c_int, C.c_double, C.c_int]
        lib.orc_restore_argmin.restype = C.c_double
        lib.orc_threads.restype = C.c_int
        lib.orc_set_threads.argtypes = [C.c_int]
        _lib = lib
    return _lib


def threads() -> int:
    return _load().orc_threads()


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _result(res: _Res, trace: np.ndarray) -> OracleResult:
    k = min(int(res.checks), len(trace))
    return OracleResult(n=int(res.n), r=float(res.r), count=int(res.count),
                        converged=bool(res.converged), run=int(res.run), checks=int(res.checks),
                        numeric_error=bool(res.numeric_error), trace=trace[:k].copy())


def jacobi_run(a: np.ndarray, *, helmholtz: bool = False, g: np.ndarray | None = None,
               alpha: float = 0.0, h: float = 1.0, reduce_op: int = RED_MAX_ABS_DELTA,
               cond: int = COND_BELOW, thr: float = 1e-6, check_every: int = 1,
               max_iter: int = 2000, trace_cap: int = 0) -> tuple[np.ndarray, OracleResult]:
    """5-point Jacobi (Laplace or Helmholtz) on an FP64 grid with a fixed ring."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64).copy()
    gp = None
    if helmholtz:
        g = np.ascontiguousarray(g, dtype=np.float64)
        assert g.shape == a.shape
        gp = _ptr(g)
    trace = np.zeros(max(trace_cap, 1), dtype=np.float64)
    res = _Res()
    rc = lib.orc_jacobi_run(int(helmholtz), _ptr(a), gp, a.shape[0], a.shape[1], float(alpha),
                            float(h), int(reduce_op), int(cond), float(thr), int(check_every),
                            int(max_iter), _ptr(trace), int(trace_cap), C.byref(res))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return a, _result(res, trace[:trace_cap])


def jacobi_sep_run(a: np.ndarray, p: np.ndarray, q: np.ndarray, c1: float, c2: float, *,
                   alpha: float, h: float, reduce_op: int = RED_L2_DELTA, cond: int = COND_BELOW,
                   thr: float = 1e-9, check_every: int = 10, max_iter: int = 5000,
                   trace_cap: int = 0) -> tuple[np.ndarray, OracleResult]:
    """The -i form of the Helmholtz sweep: g(i, j) = c2 * (c1 * (p[i] * q[j])) from the
    cell's indices (FP64)."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64).copy()
    p = np.ascontiguousarray(p, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert p.shape == (a.shape[0],) and q.shape == (a.shape[1],)
    trace = np.zeros(max(trace_cap, 1), dtype=np.float64)
    res = _Res()
    rc = lib.orc_jacobi_sep_run(_ptr(a), _ptr(p), _ptr(q), float(c1), float(c2), a.shape[0],
                                a.shape[1], float(alpha), float(h), int(reduce_op), int(cond),
                                float(thr), int(check_every), int(max_iter), _ptr(trace),
                                int(trace_cap), C.byref(res))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return a, _result(res, trace[:trace_cap])


def life_run(a: np.ndarray, *, bc: int = BC_TORUS, cond: int = COND_STABLE_FOR,
             stable_window: int = 10, check_every: int = 1, max_iter: int = 2000,
             trace_cap: int = 0) -> tuple[np.ndarray, OracleResult]:
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.uint8).copy()
    trace = np.zeros(max(trace_cap, 1), dtype=np.uint64)
    res = _Res()
    rc = lib.orc_life_run(_ptr(a), a.shape[0], a.shape[1], int(bc), int(cond), int(stable_window),
                          int(check_every), int(max_iter), _ptr(trace), int(trace_cap),
                          C.byref(res))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return a, _result(res, trace[:trace_cap])


def amf_detect(y: np.ndarray, w_max: int = 19) -> tuple[np.ndarray, np.ndarray]:
    """Returns (mask, u0): u0 is the median at flagged pixels and y elsewhere."""
    lib = _load()
    y = np.ascontiguousarray(y, dtype=np.uint8)
    mask = np.zeros_like(y)
    u0 = np.zeros_like(y)
    if lib.orc_amf_detect(_ptr(y), y.shape[0], y.shape[1], int(w_max), _ptr(mask), _ptr(u0)) != 0:
        raise ValueError("oracle rejected the arguments")
    return mask, u0


def restore_run(u: np.ndarray, mask: np.ndarray, *, beta: float = 100.0, quadratic: bool = False,
                reduce_op: int = RED_MAX_ABS_DELTA, cond: int = COND_BELOW, thr: float = 0.1,
                check_every: int = 1, max_iter: int = 200,
                trace_cap: int = 0) -> tuple[np.ndarray, OracleResult]:
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.float64).copy()
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    assert mask.shape == u.shape
    trace = np.zeros(max(trace_cap, 1), dtype=np.float64)
    res = _Res()
    rc = lib.orc_restore_run(_ptr(u), _ptr(mask), u.shape[0], u.shape[1], float(beta),
                             int(quadratic), int(reduce_op), int(cond), float(thr),
                             int(check_every), int(max_iter), _ptr(trace), int(trace_cap),
                             C.byref(res))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return u, _result(res, trace[:trace_cap])


def restore_argmin(v, beta: float = 100.0, quadratic: bool = False) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return float(_load().orc_restore_argmin(_ptr(v), len(v), float(beta), int(quadratic)))


def sobel_run(a: np.ndarray, *, check_every: int = 1, max_iter: int = 1,
              trace_cap: int = 0) -> tuple[np.ndarray, OracleResult]:
    """Sobel magnitude sweeps of a u8 image (Sect. 4.2): floor(sqrt(Gx^2 + Gy^2))
    clamped to 255, outside samples 0; the reduce is the sum of the new image."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.uint8).copy()
    trace = np.zeros(max(trace_cap, 1), dtype=np.uint64)
    res = _Res()
    rc = lib.orc_sobel_run(_ptr(a), a.shape[0], a.shape[1], int(check_every), int(max_iter),
                           _ptr(trace), int(trace_cap), C.byref(res))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return a, _result(res, trace[:trace_cap])


def box_run(a: np.ndarray, k: int, *, reduce_op: int = RED_MAX_ABS_DELTA, cond: int = COND_BELOW,
            thr: float = 1e-6, check_every: int = 1, max_iter: int = 100,
            trace_cap: int = 0) -> tuple[np.ndarray, OracleResult]:
    """Radius-k box-mean Jacobi (sigma_k): FP64, band of width k fixed."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64).copy()
    trace = np.zeros(max(trace_cap, 1), dtype=np.float64)
    res = _Res()
    rc = lib.orc_box_run(_ptr(a), a.shape[0], a.shape[1], int(k), int(reduce_op), int(cond),
                         float(thr), int(check_every), int(max_iter), _ptr(trace), int(trace_cap),
                         C.byref(res))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return a, _result(res, trace[:trace_cap])


def jacobi3d_run(a: np.ndarray, *, reduce_op: int = RED_MAX_ABS_DELTA, cond: int = COND_BELOW,
                 thr: float = 1e-6, check_every: int = 1, max_iter: int = 100,
                 trace_cap: int = 0) -> tuple[np.ndarray, OracleResult]:
    """3D 7-point Jacobi on an (nz, ny, nx) FP64 array with fixed faces."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64).copy()
    nz, ny, nx = a.shape
    trace = np.zeros(max(trace_cap, 1), dtype=np.float64)
    res = _Res()
    rc = lib.orc_jacobi3d_run(_ptr(a), nz, ny, nx, int(reduce_op), int(cond), float(thr),
                              int(check_every), int(max_iter), _ptr(trace), int(trace_cap),
                              C.byref(res))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return a, _result(res, trace[:trace_cap])
