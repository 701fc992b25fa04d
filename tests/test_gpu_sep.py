"""GPU tests of the -i (index-aware) Helmholtz form: g(i, j) = c2 * (c1 * (p_i q_j))
evaluated from the cell's indices. With the manufactured solution's factors it
equals the array form (g read from env0) bit for bit, unfused and fused, FP64 and
FP32; with asymmetric factors it equals the oracle's -i form (FP64 bit for bit)."""
import math

import numpy as np
import pytest

import oracle as O
import paper_1609_04567_amd as L
from paper_1609_04567_amd import inputs as I
from gpu_helpers import rel_err, say, to_dev

pytestmark = pytest.mark.gpu


def _run_sep(ctx, u0, p, q, c1, c2, alpha, h, f32, cond, mi, pitch=None, off=0):
    import torch
    dt = np.float32 if f32 else np.float64
    t = to_dev(u0.astype(dt), pitch, off)
    pv = torch.from_numpy(np.ascontiguousarray(p, np.float64)).to("cuda:0")
    qv = torch.from_numpy(np.ascontiguousarray(q, np.float64)).to("cuda:0")
    r = ctx.run(t, L.LSR_ST_HELMHOLTZ5_SEP, L.LSR_RED_L2_DELTA, cond, mi, L.LSR_BC_RING,
                env0=pv, env1=qv, param=(alpha, h, c1, c2))
    torch.cuda.synchronize()
    return t.cpu().numpy(), r


def _run_env(ctx, u0, g, alpha, h, f32, cond, mi):
    import torch
    dt = np.float32 if f32 else np.float64
    t = to_dev(u0.astype(dt))
    gt = to_dev(g.astype(dt))
    r = ctx.run(t, L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA, cond, mi, L.LSR_BC_RING, env0=gt,
                param=(alpha, h))
    torch.cuda.synchronize()
    return t.cpu().numpy(), r


@pytest.mark.parametrize("n", [66, 257, 1024])
@pytest.mark.parametrize("f32", [False, True])
@pytest.mark.parametrize("depth", [0, 1])
def test_sep_equals_array_form(ctx, n, f32, depth):
    say(f"sep vs env n={n} f32={f32} depth={depth}")
    hin = I.helmholtz_input(n)
    s, h = I.helmholtz_factor(n)
    cond = L.make_cond(L.LSR_COND_BELOW, 1e-9, 10)
    ctx.tune(tb_depth=depth)
    try:
        xs, rs = _run_sep(ctx, hin.u0, s, s, 2 * math.pi ** 2 + hin.alpha, h * h, hin.alpha, h, f32,
                          cond, 430)
        xe, re = _run_env(ctx, hin.u0, hin.g, hin.alpha, h, f32, cond, 430)
    finally:
        ctx.tune()
    assert rs.status == L.LSR_OK and rs.iterations == re.iterations == 430
    assert rs.sweeps_per_launch == re.sweeps_per_launch or depth == 0
    assert np.array_equal(xs, xe)


def test_sep_asymmetric_factors_match_oracle(ctx):
    say("sep asymmetric vs oracle")
    rng = np.random.default_rng(5)
    for rows, cols, mi, every in ((130, 77, 300, 10), (515, 1000, 203, 1)):
        p = rng.uniform(-1, 1, rows)
        q = rng.uniform(0, 2, cols)
        a = rng.uniform(0, 1, (rows, cols))
        cond = L.make_cond(L.LSR_COND_BELOW, 1e-12, every)
        o, ro = O.jacobi_sep_run(a, p, q, 3.7, 0.01, alpha=2.0, h=0.1, thr=1e-12,
                                 check_every=every, max_iter=mi)
        x, r = _run_sep(ctx, a, p, q, 3.7, 0.01, 2.0, 0.1, False, cond, mi)
        assert r.iterations == ro.n and np.array_equal(x, o)
        # a pitched, misaligned grid runs on a staged copy with the same result
        x2, r2 = _run_sep(ctx, a, p, q, 3.7, 0.01, 2.0, 0.1, False, cond, mi, pitch=cols + 7, off=1)
        assert np.array_equal(x2, o)
        xf, rf = _run_sep(ctx, a, p, q, 3.7, 0.01, 2.0, 0.1, True, cond, mi)
        assert rel_err(xf, o) <= 1e-5


def test_sep_rejected_on_batched_and_host():
    import torch
    say("sep rejections")
    t = torch.zeros((16, 16), dtype=torch.float64, device="cuda:0")
    v = torch.ones(16, dtype=torch.float64, device="cuda:0")
    with L.Context(0, batched=True) as b:
        with pytest.raises(L.LsrError) as ei:
            b.submit(t, L.LSR_ST_HELMHOLTZ5_SEP, L.LSR_RED_L2_DELTA,
                     L.make_cond(L.LSR_COND_BELOW, 1e-9, 10), 10, L.LSR_BC_RING, env0=v, env1=v,
                     param=(1.0, 0.1, 1.0, 1.0))
        assert ei.value.status == L.LSR_EINVAL
