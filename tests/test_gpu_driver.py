"""GPU tests of the loop driver and the C-ABI contract around it: asynchronous
results, cancellation, stream ordering, the HBM budget, and job-table errors."""
import numpy as np
import pytest

import oracle as O
import paper_1609_04567_amd as L
from paper_1609_04567_amd import inputs as I
from gpu_helpers import say

pytestmark = pytest.mark.gpu


def _helm_job(ctx, n=4096, sweeps=2000):
    import torch
    h = I.helmholtz_input(n)
    t = torch.zeros((n, n), dtype=torch.float64, device="cuda:0")
    g = torch.from_numpy(h.g).to("cuda:0")
    job = ctx.submit(t, L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA,
                     L.make_cond(L.LSR_COND_BELOW, 1e-9, 10), sweeps, L.LSR_BC_RING, env0=g,
                     param=(1.0, h.h))
    return job, t


def _poll(ctx, job):
    out = L._native.lsr_job_result()
    return L._native.lib().lsr_result(ctx.handle, job, 0, L._native.C.byref(out))


def test_nonblocking_result_then_wait(ctx):
    # 20000 sweeps of 4096^2 take a few hundred milliseconds: the immediate poll
    # must find the job running
    say("nonblocking result")
    job, _ = _helm_job(ctx, n=4096, sweeps=20000)
    assert _poll(ctx, job) == L.LSR_EBUSY
    r = ctx.result(job)
    assert r.status == L.LSR_OK and r.iterations == 20000
    with pytest.raises(L.LsrError) as ei:
        ctx.result(job)
    assert ei.value.status == L.LSR_ENOTFOUND


def test_cancel_stops_early(ctx):
    # the cap (200000 sweeps of 8192^2, about 10 s) cannot be reached before the
    # cancel takes effect at the next chunk boundary
    say("cancel")
    job, _ = _helm_job(ctx, n=8192, sweeps=200000)
    assert _poll(ctx, job) == L.LSR_EBUSY
    ctx.cancel(job)
    r = ctx.result(job)
    assert r.status == L.LSR_ECANCELED
    assert 0 <= r.iterations < 200000 and not r.converged


def test_queued_jobs_run_in_order_and_match_oracle(ctx):
    import torch
    say("queue of jobs")
    ins = [I.laplace_input(64 + 16 * k, seed=k) for k in range(6)]
    ts = [torch.from_numpy(a).to("cuda:0") for a in ins]
    jobs = [ctx.submit(t, L.LSR_ST_LAPLACE5, L.LSR_RED_MAX_ABS_DELTA,
                       L.make_cond(L.LSR_COND_BELOW, 1e-6, 1), 300, L.LSR_BC_RING) for t in ts]
    for a, t, j in zip(ins, ts, jobs):
        r = ctx.result(j)
        o, ro = O.jacobi_run(a, thr=1e-6, max_iter=300)
        assert r.iterations == ro.n
        assert np.array_equal(t.cpu().numpy(), o)


def test_stream_ordering_with_torch_work(ctx):
    import torch
    say("stream ordering")
    a = I.laplace_input(128, seed=9)
    t = torch.zeros((128, 128), dtype=torch.float64, device="cuda:0")
    src = torch.from_numpy(a).to("cuda:0")
    torch.cuda.synchronize()
    t.copy_(src)                   # enqueued before the job on the same stream
    job = ctx.submit(t, L.LSR_ST_LAPLACE5, L.LSR_RED_MAX_ABS_DELTA,
                     L.make_cond(L.LSR_COND_BELOW, 1e-6, 1), 100, L.LSR_BC_RING)
    ctx.result(job)
    after = t * 2.0                # enqueued after the result on the same stream
    o, _ = O.jacobi_run(a, thr=1e-6, max_iter=100)
    assert np.array_equal(after.cpu().numpy(), 2.0 * o)


def test_budget_refuses_oversized_scratch():
    import torch
    say("hbm budget")
    with L.Context(0, hbm_budget_bytes=1 << 20) as c:
        t = torch.zeros((1024, 1024), dtype=torch.float64, device="cuda:0")
        with pytest.raises(L.LsrError) as ei:
            c.submit(t, L.LSR_ST_LAPLACE5, L.LSR_RED_MAX_ABS_DELTA,
                     L.make_cond(L.LSR_COND_BELOW, 1e-6, 1), 10, L.LSR_BC_RING)
        assert ei.value.status == L.LSR_EBUSY
        small = torch.zeros((64, 64), dtype=torch.float64, device="cuda:0")
        r = c.run(small, L.LSR_ST_LAPLACE5, L.LSR_RED_MAX_ABS_DELTA,
                  L.make_cond(L.LSR_COND_BELOW, 1e-6, 1), 10, L.LSR_BC_RING)
        assert r.status == L.LSR_OK


def test_invalid_run_is_rejected_synchronously(ctx):
    import torch
    say("invalid run")
    t = torch.zeros((2, 8), dtype=torch.float64, device="cuda:0")
    with pytest.raises(L.LsrError) as ei:
        ctx.submit(t, L.LSR_ST_LAPLACE5, L.LSR_RED_MAX_ABS_DELTA,
                   L.make_cond(L.LSR_COND_BELOW, 1e-6, 1), 10, L.LSR_BC_RING)
    assert ei.value.status == L.LSR_EINVAL


def test_extreme_check_periods(ctx):
    # a check period of at least max_iter checks only at the cap (a period of
    # 2^31 - 1 with a cap of 64 sweeps runs); a period whose chunk base
    # lcm(period, 2K) would pass the driver's bound is rejected at submission
    # instead of overflowing the chunk arithmetic
    import torch
    say("extreme check periods")
    a = I.laplace_input(96, seed=4)
    t = torch.from_numpy(a).to("cuda:0")
    r = ctx.run(t, L.LSR_ST_LAPLACE5, L.LSR_RED_MAX_ABS_DELTA,
                L.make_cond(L.LSR_COND_BELOW, 0.0, (1 << 31) - 1), 64, L.LSR_BC_RING)
    o, ro = O.jacobi_run(a, reduce_op=O.RED_MAX_ABS_DELTA, thr=0.0, check_every=64, max_iter=64)
    assert r.status == L.LSR_OK and r.iterations == 64 and ro.n == 64
    assert np.array_equal(t.cpu().numpy(), o)
    for every in ((1 << 31) - 1, 65537 * 2):
        with pytest.raises(L.LsrError) as ei:
            ctx.submit(t, L.LSR_ST_LAPLACE5, L.LSR_RED_MAX_ABS_DELTA,
                       L.make_cond(L.LSR_COND_BELOW, 0.0, every), 1 << 40, L.LSR_BC_RING)
        assert ei.value.status == L.LSR_EINVAL
