"""GPU tests of restoration jobs in the batched engine (phase 2 of Sect. 4.3 in
the sweep rounds, and two-phase host frames: detection on the device at
admission, then the restoration rounds).

Every restored field equals the plain path's (detection + one sweep per launch)
bit for bit, with the same iteration count; FP64 fields are within 1e-12 of the
oracle and FP32 within 1e-5; a job's result is the same alone and beside other
frames and Jacobi/Life jobs."""
import numpy as np
import pytest

import oracle as O
import paper_1609_04567_amd as L
from paper_1609_04567_amd import inputs as I
from gpu_helpers import rel_err, say

pytestmark = pytest.mark.gpu

SHAPES = [(96, 80, 0.4, 4), (130, 200, 0.3, 5), (61, 67, 0.7, 6), (257, 129, 0.4, 7)]


def _plain(y, dt, reduce_op=L.LSR_RED_MAX_ABS_DELTA, thr=0.1, quadratic=False):
    import torch
    with L.Context(0) as c:
        yt = torch.from_numpy(y).to("cuda:0")
        m, u = c.amf_detect(yt, 19, dt)
        r = c.run(u, L.LSR_ST_RESTORE, reduce_op, L.make_cond(L.LSR_COND_BELOW, thr, 1), 200,
                  L.LSR_BC_BOTTOM, env0=m, param=(100.0, 1.0 if quadratic else 0.0))
        torch.cuda.synchronize()
        return m.cpu().numpy(), u.cpu().numpy(), r


def _oracle(y, reduce_op=O.RED_MAX_ABS_DELTA, thr=0.1):
    m, u0 = O.amf_detect(y, 19)
    o, ro = O.restore_run(u0.astype(np.float64), m, reduce_op=reduce_op, thr=thr, max_iter=200)
    return m, o, ro


@pytest.mark.parametrize("dt_name", ["f64", "f32"])
def test_batched_restore_sweeps_equal_plain_and_oracle(dt_name):
    import torch
    dt = torch.float64 if dt_name == "f64" else torch.float32
    say(f"batched restore phase 2 {dt_name}")
    with L.Context(0, batched=True) as b, L.Context(0) as c:
        jobs = []
        for rows, cols, noise, seed in SHAPES:
            y = I.restore_input(rows, cols, seed=seed, noise=noise).y
            yt = torch.from_numpy(y).to("cuda:0")
            m, u = c.amf_detect(yt, 19, dt)
            torch.cuda.synchronize()
            jid = b.submit(u, L.LSR_ST_RESTORE, L.LSR_RED_MAX_ABS_DELTA,
                           L.make_cond(L.LSR_COND_BELOW, 0.1, 1), 200, L.LSR_BC_BOTTOM, env0=m,
                           param=(100.0, 0.0))
            jobs.append((y, u, m, jid))
        for y, u, m, jid in jobs:
            r = b.result(jid)
            torch.cuda.synchronize()
            mp, up, rp = _plain(y, dt)
            x = u.cpu().numpy()
            assert r.status == L.LSR_OK and r.iterations == rp.iterations
            assert np.array_equal(x, up)
            mo, o, ro = _oracle(y)
            assert r.iterations == ro.n
            assert rel_err(x.astype(np.float64), o) <= (1e-12 if dt_name == "f64" else 1e-5)


def test_two_phase_host_frames_mixed_with_other_jobs():
    import torch
    say("two-phase host frames in a mixed batch")
    with L.Context(0, batched=True) as b:
        frames = []
        for k, (rows, cols, noise, seed) in enumerate(SHAPES * 2):
            y = torch.from_numpy(I.restore_input(rows, cols, seed=seed + 10 * (k // 4),
                                                 noise=noise).y).pin_memory()
            dt = torch.float64 if k % 2 == 0 else torch.float32
            u = torch.empty((rows, cols), dtype=dt).pin_memory()
            frames.append((y, u, dt, b.submit_restore_host(y, u)))
            if k == 2:   # other kinds of job in the same rounds
                a = torch.from_numpy(I.laplace_input(300, seed=3)).to("cuda:0")
                lap = b.submit(a, L.LSR_ST_LAPLACE5, L.LSR_RED_MAX_ABS_DELTA,
                               L.make_cond(L.LSR_COND_BELOW, 1e-6, 1), 500, L.LSR_BC_RING)
                s = torch.from_numpy(I.life_input(256, seed=5)).to("cuda:0")
                lif = b.submit(s, L.LSR_ST_LIFE, L.LSR_RED_SUM,
                               L.make_cond(L.LSR_COND_STABLE_FOR, 0.0, 1, 10), 400, L.LSR_BC_TORUS)
        for y, u, dt, jid in frames:
            r = b.result(jid)
            mp, up, rp = _plain(y.numpy(), dt)
            assert r.status == L.LSR_OK and r.iterations == rp.iterations
            assert np.array_equal(u.numpy(), up)
        assert b.result(lap).status == L.LSR_OK and b.result(lif).status == L.LSR_OK
        torch.cuda.synchronize()


def test_two_phase_mean_abs_and_host_restore_job():
    import torch
    say("two-phase mean-abs; host restore job")
    y = I.restore_input(200, 160, seed=9, noise=0.5).y
    mo, o, ro = _oracle(y, reduce_op=O.RED_MEAN_ABS_DELTA, thr=0.01)
    with L.Context(0, batched=True) as b:
        yh = torch.from_numpy(y).pin_memory()
        u = torch.empty(y.shape, dtype=torch.float64).pin_memory()
        r = b.result(b.submit_restore_host(yh, u, reduce_op=L.LSR_RED_MEAN_ABS_DELTA,
                                           cond=L.make_cond(L.LSR_COND_BELOW, 0.01, 1)))
        assert r.status == L.LSR_OK and r.iterations == ro.n
        assert rel_err(u.numpy(), o) <= 1e-12
        # phase 2 alone on host buffers (lsr_run_host), batched and plain
        u0 = torch.from_numpy(O.amf_detect(y, 19)[1].astype(np.float64)).pin_memory()
        m = torch.from_numpy(mo).pin_memory()
        for ctx in (b, L.Context(0)):
            uu = u0.clone().pin_memory()
            r2 = ctx.result(ctx.submit_host(uu, L.LSR_ST_RESTORE, L.LSR_RED_MEAN_ABS_DELTA,
                                            L.make_cond(L.LSR_COND_BELOW, 0.01, 1), 200,
                                            L.LSR_BC_BOTTOM, env0=m, param=(100.0, 0.0)))
            assert r2.iterations == ro.n and rel_err(uu.numpy(), o) <= 1e-12
            if ctx is not b:
                ctx.close()


def test_two_phase_rejections():
    import torch
    say("two-phase argument checks")
    y = torch.zeros((16, 16), dtype=torch.uint8).pin_memory()
    u = torch.zeros((16, 16), dtype=torch.float64).pin_memory()
    with L.Context(0) as c:
        with pytest.raises(L.LsrError) as ei:
            c.submit_restore_host(y, u)
        assert ei.value.status == L.LSR_EINVAL
    with L.Context(0, batched=True) as b:
        for kw in (dict(w_max=4), dict(w_max=33), dict(beta=0.0)):
            with pytest.raises(L.LsrError) as ei:
                b.submit_restore_host(y, u, **kw)
            assert ei.value.status == L.LSR_EINVAL
