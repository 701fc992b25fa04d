"""ctypes binding of include/lsr.h (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
computation of its own; all work runs in the HIP kernels of liblsr.so. The
library must be built (``python -m paper_1609_04567_amd.build`` or
``__graft_entry__.build()``); a missing library raises at first use, there is
no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblsr.so")

# enums of lsr.h
LSR_OK, LSR_EINVAL, LSR_ENOMEM, LSR_EBUSY, LSR_EDEVICE, LSR_ENUMERIC, LSR_ECANCELED, LSR_ENOTFOUND = range(8)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EBUSY", 4: "EDEVICE", 5: "ENUMERIC",
                6: "ECANCELED", 7: "ENOTFOUND"}
LSR_U8, LSR_F32, LSR_F64 = 1, 4, 8
LSR_BC_RING, LSR_BC_TORUS, LSR_BC_BOTTOM = 0, 1, 2
LSR_ST_LAPLACE5, LSR_ST_HELMHOLTZ5, LSR_ST_LIFE, LSR_ST_RESTORE, LSR_ST_SOBEL = 1, 2, 3, 4, 5
LSR_ST_HELMHOLTZ5_SEP, LSR_ST_BOX, LSR_ST_LAPLACE7_3D = 6, 7, 8
LSR_RED_MAX_ABS_DELTA, LSR_RED_L2_DELTA, LSR_RED_SUM, LSR_RED_MEAN_ABS_DELTA = 1, 2, 3, 4
LSR_COND_BELOW, LSR_COND_STABLE_FOR, LSR_COND_NEVER = 1, 2, 3
LSR_FLAG_BATCHED = 1


class lsr_grid(C.Structure):
    _fields_ = [("data", C.c_void_p), ("rows", C.c_int64), ("cols", C.c_int64),
                ("pitch", C.c_int64), ("dtype", C.c_int32), ("bc", C.c_int32),
                ("env0", C.c_void_p), ("env1", C.c_void_p), ("param", C.c_double * 4)]


class lsr_cond(C.Structure):
    _fields_ = [("kind", C.c_int32), ("check_every", C.c_int32), ("stable_window", C.c_int32),
                ("reserved", C.c_int32), ("threshold", C.c_double)]


class lsr_config(C.Structure):
    _fields_ = [("device", C.c_int32), ("flags", C.c_uint32), ("stream", C.c_void_p),
                ("hbm_budget_bytes", C.c_uint64)]


class lsr_job_result(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("last_reduce", C.c_double), ("last_count", C.c_uint64),
                ("converged", C.c_int32), ("status", C.c_int32), ("stable_run", C.c_int32),
                ("sweeps_per_launch", C.c_int32), ("checks", C.c_int64),
                ("device_ms", C.c_double), ("queue_ms", C.c_double), ("latency_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class lsr_tuning(C.Structure):
    _fields_ = [("tile_rows", C.c_int32), ("tb_depth", C.c_int32), ("chunk", C.c_int32),
                ("use_graph", C.c_int32), ("waves", C.c_int32), ("unroll", C.c_int32)]


class lsr_stats(C.Structure):
    _fields_ = [("pending", C.c_int64), ("ingesting", C.c_int64), ("active", C.c_int64),
                ("retiring", C.c_int64), ("unfinished", C.c_int64), ("finished_untaken", C.c_int64),
                ("pool_live_bytes", C.c_uint64), ("pool_cached_bytes", C.c_uint64),
                ("pool_budget_bytes", C.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class LsrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# Every symbol lsr.h declares, with its ctypes signature.
_SIGS = {
    "lsr_create": (C.c_int, [C.POINTER(lsr_config), C.POINTER(C.c_void_p)]),
    "lsr_destroy": (C.c_int, [C.c_void_p]),
    "lsr_set_tuning": (C.c_int, [C.c_void_p, C.POINTER(lsr_tuning)]),
    "lsr_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_int64, C.c_int32,
                               C.c_int64, C.POINTER(lsr_tuning)]),
    "lsr_tune_export": (C.c_int, [C.c_void_p, C.c_char_p, C.c_uint64, C.POINTER(C.c_uint64)]),
    "lsr_tune_import": (C.c_int, [C.c_void_p, C.c_char_p]),
    "lsr_run": (C.c_int, [C.c_void_p, C.POINTER(lsr_grid), C.c_int32, C.c_int32,
                          C.POINTER(lsr_cond), C.c_int64, C.POINTER(C.c_int64)]),
    "lsr_run_host": (C.c_int, [C.c_void_p, C.POINTER(lsr_grid), C.c_int32, C.c_int32,
                               C.POINTER(lsr_cond), C.c_int64, C.POINTER(C.c_int64)]),
    "lsr_run_restore_host": (C.c_int, [C.c_void_p, C.POINTER(lsr_grid), C.c_void_p, C.c_int32,
                                       C.c_int32, C.c_int32, C.POINTER(lsr_cond), C.c_int64,
                                       C.POINTER(C.c_int64)]),
    "lsr_run_noalloc": (C.c_int, [C.c_void_p, C.POINTER(lsr_grid), C.c_int32, C.c_int32,
                                  C.POINTER(lsr_cond), C.c_int64, C.POINTER(lsr_job_result)]),
    "lsr_result": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.POINTER(lsr_job_result)]),
    "lsr_cancel": (C.c_int, [C.c_void_p, C.c_int64]),
    "lsr_wait_any": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]),
    "lsr_get_stats": (C.c_int, [C.c_void_p, C.POINTER(lsr_stats)]),
    "lsr_amf_detect": (C.c_int, [C.c_void_p, C.POINTER(lsr_grid), C.c_void_p, C.c_void_p,
                                 C.c_int32, C.c_int32]),
    "lsr_check_args": (C.c_int, [C.POINTER(lsr_grid), C.c_int32, C.c_int32, C.POINTER(lsr_cond),
                                 C.c_int64]),
    "lsr_probe_copy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_int32,
                                 C.POINTER(C.c_double)]),
    "lsr_last_error": (C.c_char_p, []),
    "lsr_version": (C.c_char_p, []),
}

_lib = None


def lib():
    """Loads liblsr.so (raises if it is not built: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != LSR_OK:
        raise LsrError(status, lsr_last_error())


def lsr_last_error() -> str:
    return lib().lsr_last_error().decode()


def lsr_version() -> str:
    return lib().lsr_version().decode()


def lsr_create(device: int = 0, stream: int | None = None, hbm_budget_bytes: int = 0,
               flags: int = 0) -> int:
    cfg = lsr_config(device=device, flags=flags, stream=stream or None,
                     hbm_budget_bytes=hbm_budget_bytes)
    out = C.c_void_p()
    _check(lib().lsr_create(C.byref(cfg), C.byref(out)))
    return out.value


def lsr_destroy(ctx: int) -> None:
    _check(lib().lsr_destroy(ctx))


def lsr_set_tuning(ctx: int, tile_rows: int = 0, tb_depth: int = 0, chunk: int = 0,
                   use_graph: int = 0, waves: int = 0, unroll: int = 0) -> None:
    t = lsr_tuning(tile_rows, tb_depth, chunk, use_graph, waves, unroll)
    _check(lib().lsr_set_tuning(ctx, C.byref(t)))


def lsr_run(ctx: int, grid: lsr_grid, stencil_id: int, reduce_op: int, cond: lsr_cond,
            max_iter: int) -> int:
    job = C.c_int64()
    _check(lib().lsr_run(ctx, C.byref(grid), stencil_id, reduce_op, C.byref(cond), max_iter,
                         C.byref(job)))
    return job.value


def lsr_run_host(ctx: int, grid: lsr_grid, stencil_id: int, reduce_op: int, cond: lsr_cond,
                 max_iter: int) -> int:
    """lsr_run with grid->data and grid->env0 in host memory."""
    job = C.c_int64()
    _check(lib().lsr_run_host(ctx, C.byref(grid), stencil_id, reduce_op, C.byref(cond), max_iter,
                              C.byref(job)))
    return job.value


def lsr_run_restore_host(ctx: int, y: lsr_grid, u_out_ptr: int, u_dtype: int, w_max: int,
                         reduce_op: int, cond: lsr_cond, max_iter: int) -> int:
    """Detection and restoration of one host frame as one batched job."""
    job = C.c_int64()
    _check(lib().lsr_run_restore_host(ctx, C.byref(y), u_out_ptr, u_dtype, w_max, reduce_op,
                                      C.byref(cond), max_iter, C.byref(job)))
    return job.value


def lsr_run_noalloc(ctx: int, grid: lsr_grid, stencil_id: int, reduce_op: int, cond: lsr_cond,
                    max_iter: int) -> lsr_job_result:
    """lsr_run + a waiting lsr_result on the library's fixed scratch (no allocation)."""
    out = lsr_job_result()
    st = lib().lsr_run_noalloc(ctx, C.byref(grid), stencil_id, reduce_op, C.byref(cond), max_iter,
                               C.byref(out))
    if st not in (LSR_OK, LSR_ENUMERIC):
        raise LsrError(st, lsr_last_error())
    return out


def lsr_result(ctx: int, job: int, wait: bool = True) -> lsr_job_result:
    """Returns the job's result; its own status (OK/ENUMERIC/ECANCELED) is in .status."""
    out = lsr_job_result()
    st = lib().lsr_result(ctx, job, 1 if wait else 0, C.byref(out))
    if st not in (LSR_OK, LSR_ENUMERIC, LSR_ECANCELED):
        raise LsrError(st, lsr_last_error())
    return out


def lsr_wait_any(ctx: int, wait: bool = True) -> int | None:
    """Id of a finished job whose result is not taken yet; None when wait is False
    and none has finished (EBUSY). Raises ENOTFOUND when no job is outstanding."""
    job = C.c_int64()
    st = lib().lsr_wait_any(ctx, 1 if wait else 0, C.byref(job))
    if st == LSR_EBUSY:
        return None
    _check(st)
    return job.value


def lsr_get_stats(ctx: int) -> dict:
    out = lsr_stats()
    _check(lib().lsr_get_stats(ctx, C.byref(out)))
    return out.as_dict()


def lsr_cancel(ctx: int, job: int) -> None:
    _check(lib().lsr_cancel(ctx, job))


def lsr_amf_detect(ctx: int, y: lsr_grid, mask_ptr: int, u_init_ptr: int, u_dtype: int,
                   w_max: int) -> None:
    _check(lib().lsr_amf_detect(ctx, C.byref(y), mask_ptr, u_init_ptr, u_dtype, w_max))


def lsr_check_args(grid: lsr_grid, stencil_id: int, reduce_op: int, cond: lsr_cond,
                   max_iter: int) -> int:
    """Returns the status lsr_run would give for these arguments (no device needed)."""
    return lib().lsr_check_args(C.byref(grid), stencil_id, reduce_op, C.byref(cond), max_iter)


def lsr_autotune(ctx: int, stencil_id: int, dtype: int, rows: int, cols: int, check_every: int,
                 max_iter: int = 0) -> lsr_tuning:
    best = lsr_tuning()
    _check(lib().lsr_autotune(ctx, stencil_id, dtype, rows, cols, check_every, max_iter,
                              C.byref(best)))
    return best


def lsr_tune_export(ctx: int) -> str:
    need = C.c_uint64(0)
    _check(lib().lsr_tune_export(ctx, None, 0, C.byref(need)))
    buf = C.create_string_buffer(need.value)
    _check(lib().lsr_tune_export(ctx, buf, need.value, C.byref(need)))
    return buf.value.decode()


def lsr_tune_import(ctx: int, text: str) -> None:
    _check(lib().lsr_tune_import(ctx, text.encode()))


def lsr_probe_copy(ctx: int, dst_ptr: int, src_ptr: int, nbytes: int, iters: int) -> float:
    """Mean milliseconds per plain copy of nbytes (device to device)."""
    ms = C.c_double()
    _check(lib().lsr_probe_copy(ctx, dst_ptr, src_ptr, nbytes, iters, C.byref(ms)))
    return ms.value


def make_cond(kind: int, threshold: float = 0.0, check_every: int = 1,
              stable_window: int = 0) -> lsr_cond:
    return lsr_cond(kind=kind, check_every=check_every, stable_window=stable_window, reserved=0,
                    threshold=threshold)


def make_grid(data_ptr: int, rows: int, cols: int, pitch: int, dtype: int, bc: int,
              env0: int | None = None, param=(0.0, 0.0, 0.0, 0.0)) -> lsr_grid:
    p = (C.c_double * 4)(*([float(x) for x in param] + [0.0] * (4 - len(param))))
    return lsr_grid(data=data_ptr or None, rows=rows, cols=cols, pitch=pitch, dtype=dtype, bc=bc,
                    env0=env0 or None, env1=None, param=p)
