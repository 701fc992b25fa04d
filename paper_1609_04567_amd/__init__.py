"""Loop-of-stencil-reduce on MI355X (gfx950): Python side of the lsr C ABI.

``_native`` binds every entry point of include/lsr.h under its own name. The
helpers below only turn torch tensors into ``lsr_grid`` descriptors (pointer,
shape, pitch, dtype) and pass the current torch stream; every step of the
pattern runs in the HIP kernels of liblsr.so.
"""
from __future__ import annotations

from ._native import (  # noqa: F401
    LSR_BC_BOTTOM, LSR_BC_RING, LSR_BC_TORUS, LSR_COND_BELOW, LSR_COND_NEVER,
    LSR_COND_STABLE_FOR, LSR_FLAG_BATCHED, LSR_EBUSY, LSR_ECANCELED, LSR_EDEVICE, LSR_EINVAL, LSR_ENOMEM,
    LSR_ENOTFOUND, LSR_ENUMERIC, LSR_F32, LSR_F64, LSR_OK, LSR_RED_L2_DELTA,
    LSR_RED_MAX_ABS_DELTA, LSR_RED_MEAN_ABS_DELTA, LSR_RED_SUM, LSR_ST_HELMHOLTZ5,
    LSR_ST_HELMHOLTZ5_SEP, LSR_ST_BOX, LSR_ST_LAPLACE7_3D,
    LSR_ST_LAPLACE5, LSR_ST_LIFE, LSR_ST_RESTORE, LSR_ST_SOBEL, LSR_U8, LsrError, lsr_amf_detect,
    lsr_autotune, lsr_cancel, lsr_check_args, lsr_create, lsr_destroy, lsr_last_error,
    lsr_probe_copy, lsr_result, lsr_run, lsr_run_host, lsr_run_noalloc, lsr_run_restore_host,
    lsr_set_tuning, lsr_tune_export, lsr_tune_import, lsr_version, lsr_wait_any, lsr_get_stats,
    make_cond, make_grid,
)


def _dtype_code(t):
    import torch
    m = {torch.float64: LSR_F64, torch.float32: LSR_F32, torch.uint8: LSR_U8}
    if t.dtype not in m:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return m[t.dtype]


def grid_from_tensor(t, bc: int, env0=None, param=()):
    """lsr_grid over a 2-D CUDA tensor with unit column stride (row pitch = stride(0))."""
    if t.dim() != 2 or t.stride(1) != 1 or not t.is_cuda:
        raise ValueError("grid must be a 2-D device tensor with unit column stride")
    if env0 is not None and (env0.shape != t.shape or env0.stride(0) != t.stride(0)):
        raise ValueError("env0 must have the grid's shape and pitch")
    return make_grid(t.data_ptr(), t.shape[0], t.shape[1], t.stride(0), _dtype_code(t), bc,
                     env0.data_ptr() if env0 is not None else None, tuple(param))


def grid_from_host(t, bc: int, env0=None, param=()):
    """lsr_grid over a 2-D host array (a CPU torch tensor, pinned for asynchronous
    copies, or a numpy array) with unit column stride."""
    import numpy as np
    import torch

    def desc(a):
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(a)
        if a.dim() != 2 or a.stride(1) != 1 or a.is_cuda:
            raise ValueError("host grid must be a 2-D CPU array with unit column stride")
        return a
    t = desc(t)
    if env0 is not None:
        env0 = desc(env0)
        if env0.shape != t.shape or env0.stride(0) != t.stride(0):
            raise ValueError("env0 must have the grid's shape and pitch")
    return make_grid(t.data_ptr(), t.shape[0], t.shape[1], t.stride(0), _dtype_code(t), bc,
                     env0.data_ptr() if env0 is not None else None, tuple(param))


class Context:
    """An lsr context on one device, ordered against a torch stream."""

    def __init__(self, device: int = 0, stream=None, hbm_budget_bytes: int = 0,
                 batched: bool = False):
        import torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.handle = lsr_create(device, self.stream.cuda_stream, hbm_budget_bytes,
                                 LSR_FLAG_BATCHED if batched else 0)
        self._keep = {}

    def close(self):
        if self.handle:
            lsr_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def tune(self, tile_rows=0, tb_depth=0, chunk=0, use_graph=0, waves=0, unroll=0):
        lsr_set_tuning(self.handle, tile_rows, tb_depth, chunk, use_graph, waves, unroll)

    def autotune(self, stencil_id, dtype, rows, cols, check_every, max_iter=0):
        """Measures launch settings for this job description (see lsr_autotune)."""
        return lsr_autotune(self.handle, stencil_id, dtype, rows, cols, check_every, max_iter)

    def save_tuning(self, path):
        with open(path, "w") as fh:
            fh.write(lsr_tune_export(self.handle))

    def load_tuning(self, path):
        with open(path) as fh:
            lsr_tune_import(self.handle, fh.read())

    def submit(self, grid_t, stencil_id, reduce_op, cond, max_iter, bc, env0=None, param=(),
               env1=None):
        if stencil_id == LSR_ST_HELMHOLTZ5_SEP:
            import torch
            # env0 / env1 are the factor vectors p (rows) and q (cols), FP64 on the device
            for v, n in ((env0, grid_t.shape[0]), (env1, grid_t.shape[1])):
                if v is None or v.dim() != 1 or v.shape[0] != n or v.dtype != torch.float64 \
                        or not v.is_cuda or not v.is_contiguous():
                    raise ValueError("the -i form needs FP64 device vectors p (rows) and q (cols)")
            g = grid_from_tensor(grid_t, bc, None, param)
            g.env0, g.env1 = env0.data_ptr(), env1.data_ptr()
            job = lsr_run(self.handle, g, stencil_id, reduce_op, cond, max_iter)
            self._keep[job] = (grid_t, env0, env1)
            return job
        g = grid_from_tensor(grid_t, bc, env0, param)
        job = lsr_run(self.handle, g, stencil_id, reduce_op, cond, max_iter)
        self._keep[job] = (grid_t, env0)  # the caller's buffers stay alive until the result
        return job

    def submit_host(self, grid, stencil_id, reduce_op, cond, max_iter, bc, env0=None, param=()):
        """Starts a job on host buffers (lsr_run_host); grid receives the result."""
        g = grid_from_host(grid, bc, env0, param)
        job = lsr_run_host(self.handle, g, stencil_id, reduce_op, cond, max_iter)
        self._keep[job] = (grid, env0)
        return job

    def submit_restore_host(self, y, u_out, w_max=19, beta=100.0, quadratic=False,
                            reduce_op=LSR_RED_MAX_ABS_DELTA, cond=None, max_iter=200):
        """Detection + restoration of a host u8 frame y into the host array u_out
        (same shape and pitch, float32 or float64) on a batched context."""
        if cond is None:
            cond = make_cond(LSR_COND_BELOW, 0.1, 1)
        import numpy as np
        import torch
        g = grid_from_host(y, LSR_BC_BOTTOM, param=(beta, 1.0 if quadratic else 0.0))
        u = torch.from_numpy(u_out) if isinstance(u_out, np.ndarray) else u_out
        if tuple(u.shape) != (g.rows, g.cols) or u.stride(0) != g.pitch or u.is_cuda:
            raise ValueError("u_out must be a host array of y's shape and pitch")
        job = lsr_run_restore_host(self.handle, g, u.data_ptr(), _dtype_code(u), w_max, reduce_op,
                                   cond, max_iter)
        self._keep[job] = (y, u_out)
        return job

    def run_noalloc(self, grid_t, stencil_id, reduce_op, cond, max_iter, bc, env0=None, param=()):
        """The job on the library's fixed scratch, synchronously (lsr_run_noalloc)."""
        g = grid_from_tensor(grid_t, bc, env0, param)
        return lsr_run_noalloc(self.handle, g, stencil_id, reduce_op, cond, max_iter)

    def result(self, job, wait=True):
        r = lsr_result(self.handle, job, wait)
        self._keep.pop(job, None)
        return r

    def wait_any(self, wait=True):
        """Id of a finished job whose result is not taken yet (lsr_wait_any)."""
        return lsr_wait_any(self.handle, wait)

    def stats(self):
        """Queue and memory snapshot (lsr_get_stats)."""
        return lsr_get_stats(self.handle)

    def cancel(self, job):
        lsr_cancel(self.handle, job)

    def run(self, grid_t, stencil_id, reduce_op, cond, max_iter, bc, env0=None, param=(),
            env1=None):
        return self.result(self.submit(grid_t, stencil_id, reduce_op, cond, max_iter, bc, env0,
                                       param, env1))

    def amf_detect(self, y_t, w_max=19, u_dtype=None):
        """Phase-1 detection; returns (mask u8, u_init) tensors on y's device."""
        import torch
        u_dtype = u_dtype or torch.float64
        mask = torch.empty_like(y_t)
        u0 = torch.empty(y_t.shape, dtype=u_dtype, device=y_t.device)
        if u0.stride(0) != y_t.stride(0):
            raise ValueError("u_init must share y's pitch")
        g = grid_from_tensor(y_t, LSR_BC_BOTTOM)
        lsr_amf_detect(self.handle, g, mask.data_ptr(), u0.data_ptr(), _dtype_code(u0), w_max)
        return mask, u0
