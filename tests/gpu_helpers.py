"""Helpers shared by the GPU tests: run the HIP path through the C ABI on
torch tensors and compare with the oracle."""
from __future__ import annotations

import math
import sys

import numpy as np

import paper_1609_04567_amd as L


def say(msg: str) -> None:
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a: np.ndarray, pitch: int | None = None, offset: int = 0):
    """Copy a host array into a device tensor; optionally inside a wider allocation
    (row pitch `pitch`, first column at `offset`) to exercise pitched/misaligned paths."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if pitch is None and offset == 0:
        return t.to("cuda:0")
    rows, cols = a.shape
    pitch = pitch or (cols + offset)
    big = torch.zeros((rows, pitch), dtype=t.dtype, device="cuda:0")
    view = big[:, offset:offset + cols]
    view.copy_(t.to("cuda:0"))
    return view


def rel_err(x: np.ndarray, o: np.ndarray) -> float:
    den = float(np.max(np.abs(o)))
    return float(np.max(np.abs(x.astype(np.float64) - o))) / (den if den > 0 else 1.0)


def run_jacobi(ctx, a: np.ndarray, *, helm=False, g=None, alpha=0.0, h=1.0, f32=False,
               reduce_op=L.LSR_RED_MAX_ABS_DELTA, cond=L.LSR_COND_BELOW, thr=1e-6, check_every=1,
               max_iter=2000, pitch=None, offset=0):
    import torch
    dt = np.float32 if f32 else np.float64
    t = to_dev(a.astype(dt), pitch, offset)
    env = to_dev(g.astype(dt), pitch, offset) if helm else None
    st = L.LSR_ST_HELMHOLTZ5 if helm else L.LSR_ST_LAPLACE5
    r = ctx.run(t, st, reduce_op, L.make_cond(cond, thr, check_every), max_iter, L.LSR_BC_RING,
                env0=env, param=(alpha, h))
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64), r


def run_life(ctx, a: np.ndarray, *, torus=True, cond=L.LSR_COND_STABLE_FOR, window=10,
             check_every=1, max_iter=2000, pitch=None, offset=0):
    import torch
    t = to_dev(a.astype(np.uint8), pitch, offset)
    r = ctx.run(t, L.LSR_ST_LIFE, L.LSR_RED_SUM, L.make_cond(cond, 0.0, check_every, window),
                max_iter, L.LSR_BC_TORUS if torus else L.LSR_BC_BOTTOM)
    torch.cuda.synchronize()
    return t.cpu().numpy(), r


def run_restore(ctx, u0: np.ndarray, mask: np.ndarray, *, f32=False, beta=100.0, quadratic=False,
                reduce_op=L.LSR_RED_MAX_ABS_DELTA, cond=L.LSR_COND_BELOW, thr=0.1, max_iter=200):
    import torch
    dt = np.float32 if f32 else np.float64
    t = to_dev(u0.astype(dt))
    m = to_dev(mask.astype(np.uint8))
    r = ctx.run(t, L.LSR_ST_RESTORE, reduce_op, L.make_cond(cond, thr, 1), max_iter,
                L.LSR_BC_BOTTOM, env0=m, param=(beta, 1.0 if quadratic else 0.0))
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64), r


def closed_form_helmholtz(n: int, alpha: float, sweeps: int):
    """u^k = c*(1 - mu^k) u*, ||Delta^k||_2 = c*(1 - mu) mu^(k-1) (N-1)/2, evaluated
    without cancellation: 1 - mu = (8 sin^2(pi h/2) + alpha h^2)/(4 + alpha h^2)."""
    h = 1.0 / (n - 1)
    s2 = math.sin(math.pi * h / 2) ** 2
    one_m_mu = (8.0 * s2 + alpha * h * h) / (4.0 + alpha * h * h)
    lam = 8.0 / (h * h) * s2
    cstar = (2 * math.pi ** 2 + alpha) / (lam + alpha)
    lmu = math.log1p(-one_m_mu)
    coef = cstar * -math.expm1(sweeps * lmu)
    dnorm = cstar * one_m_mu * math.exp((sweeps - 1) * lmu) * (n - 1) / 2.0
    return coef, dnorm
