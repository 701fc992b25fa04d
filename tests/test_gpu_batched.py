"""GPU tests of the batched engine (continuous batching, LSR_FLAG_BATCHED).

Every job of a mixed batch is compared with the oracle (FP64 Jacobi fields
bit-identical, FP32 storage within 1e-5 of the FP64 oracle, Life bit-exact,
iteration counts exact); a job's result is bit-identical alone and in a mix;
jobs queue for memory under a small HBM budget and still finish correctly; a
short job submitted while a long one runs finishes first.
"""
import time

import numpy as np
import pytest

import oracle as O
import paper_1609_04567_amd as L
from paper_1609_04567_amd import inputs as I
from gpu_helpers import rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bctx():
    import torch
    c = L.Context(0, batched=True)
    yield c
    torch.cuda.synchronize()
    c.close()


def _job(kind, side, seed, f32=False, max_iter=None):
    """(tensors, submit kwargs, oracle closure) for one job of the mixed stream recipe."""
    import torch
    dt = np.float32 if f32 else np.float64
    if kind == "laplace":
        a = I.laplace_input(side, seed=seed)
        t = torch.from_numpy(a.astype(dt)).to("cuda:0")
        mi = max_iter or 2000
        kw = dict(stencil_id=L.LSR_ST_LAPLACE5, reduce_op=L.LSR_RED_MAX_ABS_DELTA,
                  cond=L.make_cond(L.LSR_COND_BELOW, 1e-6, 1), max_iter=mi, bc=L.LSR_BC_RING)
        ora = lambda: O.jacobi_run(a, thr=1e-6, max_iter=mi)
        return t, kw, ora, None
    if kind == "helmholtz":
        h = I.helmholtz_input(side)
        t = torch.from_numpy(h.u0.astype(dt)).to("cuda:0")
        g = torch.from_numpy(h.g.astype(dt)).to("cuda:0")
        mi = max_iter or 5000
        kw = dict(stencil_id=L.LSR_ST_HELMHOLTZ5, reduce_op=L.LSR_RED_L2_DELTA,
                  cond=L.make_cond(L.LSR_COND_BELOW, 1e-9, 10), max_iter=mi, bc=L.LSR_BC_RING,
                  env0=g, param=(h.alpha, h.h))
        ora = lambda: O.jacobi_run(h.u0, helmholtz=True, g=h.g, alpha=h.alpha, h=h.h,
                                   reduce_op=O.RED_L2_DELTA, thr=1e-9, check_every=10, max_iter=mi)
        return t, kw, ora, g
    s = I.life_input(side, seed=seed)
    t = torch.from_numpy(s).to("cuda:0")
    mi = max_iter or 2000
    kw = dict(stencil_id=L.LSR_ST_LIFE, reduce_op=L.LSR_RED_SUM,
              cond=L.make_cond(L.LSR_COND_STABLE_FOR, 0.0, 1, 10), max_iter=mi, bc=L.LSR_BC_TORUS)
    ora = lambda: O.life_run(s, stable_window=10, max_iter=mi)
    return t, kw, ora, None


def _submit(ctx, t, kw):
    return ctx.submit(t, kw["stencil_id"], kw["reduce_op"], kw["cond"], kw["max_iter"], kw["bc"],
                      env0=kw.get("env0"), param=kw.get("param", ()))


MIX = [("laplace", 128, 1, False, 600), ("laplace", 200, 2, True, 600),
       ("helmholtz", 129, 0, False, 700), ("helmholtz", 257, 0, True, 500),
       ("life", 128, 3, False, 2000), ("life", 160, 4, False, 900), ("life", 130, 5, False, 500),
       ("laplace", 333, 6, False, 300), ("laplace", 67, 7, True, 400),
       # grids whose two buffers fit in LDS run whole in one workgroup
       ("helmholtz", 97, 0, False, 700), ("helmholtz", 140, 0, True, 500),
       ("laplace", 60, 8, False, 900)]


def test_mixed_batch_matches_oracle(bctx):
    import torch
    say("batched mix vs oracle")
    jobs = []
    for kind, side, seed, f32, mi in MIX:
        t, kw, ora, keep = _job(kind, side, seed, f32, mi)
        jobs.append((kind, f32, t, ora, _submit(bctx, t, kw), keep))
    for kind, f32, t, ora, job, _ in jobs:
        r = bctx.result(job)
        torch.cuda.synchronize()
        o, ro = ora()
        x = t.cpu().numpy()
        assert r.status == L.LSR_OK, (kind, r.status)
        assert r.iterations == ro.n, (kind, r.iterations, ro.n)
        if kind == "life":
            assert np.array_equal(x, o) and r.last_count == ro.count
        elif f32:
            assert rel_err(x, o) <= 1e-5
        else:
            assert np.array_equal(x, o)
            assert abs(r.last_reduce - ro.r) <= 1e-12 * ro.r
        assert r.latency_ms >= r.queue_ms >= 0.0


def test_alone_and_in_mix_are_identical(bctx):
    import torch
    say("alone vs mix")
    target = ("helmholtz", 300, 0, True, 400)
    t0, kw0, _, k0 = _job(*target)
    r_alone = bctx.result(_submit(bctx, t0, kw0))
    alone = t0.cpu().numpy().copy()
    others = [_job(k, s, sd, f, mi) for (k, s, sd, f, mi) in MIX]
    t1, kw1, _, k1 = _job(*target)
    ids = [_submit(bctx, t, kw) for (t, kw, _, _) in others[:4]]
    jid = _submit(bctx, t1, kw1)
    ids += [_submit(bctx, t, kw) for (t, kw, _, _) in others[4:]]
    r_mix = bctx.result(jid)
    for i in ids:
        bctx.result(i)
    torch.cuda.synchronize()
    assert np.array_equal(t1.cpu().numpy(), alone)
    assert r_mix.iterations == r_alone.iterations and r_mix.last_reduce == r_alone.last_reduce


def test_admission_waits_for_memory():
    import torch
    say("admission under a small budget")
    side = 512
    # pool blocks per job: partner 2 MiB, partials 4 KiB, state 4 KiB; the budget
    # holds two jobs' scratch but not three
    per_job = side * side * 8 + 4096 + 4096
    with L.Context(0, hbm_budget_bytes=2 * per_job + 200_000, batched=True) as c:
        ins = [I.laplace_input(side, seed=k) for k in range(5)]
        ts = [torch.from_numpy(a).to("cuda:0") for a in ins]
        ids = [c.submit(t, L.LSR_ST_LAPLACE5, L.LSR_RED_MAX_ABS_DELTA,
                        L.make_cond(L.LSR_COND_BELOW, 1e-6, 1), 200, L.LSR_BC_RING) for t in ts]
        rs = [c.result(i) for i in ids]
        torch.cuda.synchronize()
        for a, t, r in zip(ins, ts, rs):
            o, ro = O.jacobi_run(a, thr=1e-6, max_iter=200)
            assert r.status == L.LSR_OK and r.iterations == ro.n and np.array_equal(t.cpu().numpy(), o)
        # at most two jobs fit at once, so the later ones waited in the queue
        assert max(r.queue_ms for r in rs[2:]) > min(r.queue_ms for r in rs[:2])


def test_late_short_job_overtakes_long_job(bctx):
    import torch
    say("late arrival")
    h = I.helmholtz_input(2048)
    tl = torch.zeros((2048, 2048), dtype=torch.float32, device="cuda:0")
    g = torch.from_numpy(h.g.astype(np.float32)).to("cuda:0")
    long_id = bctx.submit(tl, L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA,
                          L.make_cond(L.LSR_COND_BELOW, 1e-9, 10), 5000, L.LSR_BC_RING, env0=g,
                          param=(h.alpha, h.h))
    time.sleep(0.02)
    a = I.laplace_input(96, seed=3)
    ts = torch.from_numpy(a).to("cuda:0")
    short_id = bctx.submit(ts, L.LSR_ST_LAPLACE5, L.LSR_RED_MAX_ABS_DELTA,
                           L.make_cond(L.LSR_COND_BELOW, 1e-6, 1), 300, L.LSR_BC_RING)
    rs = bctx.result(short_id)
    t_short = time.perf_counter()
    rl = bctx.result(long_id)
    t_long = time.perf_counter()
    assert rs.status == L.LSR_OK and rl.status == L.LSR_OK and rl.iterations == 5000
    assert t_short <= t_long and rs.latency_ms < rl.latency_ms
    o, _ = O.jacobi_run(a, thr=1e-6, max_iter=300)
    assert np.array_equal(ts.cpu().numpy(), o)


def test_cancel_pending_and_running(bctx):
    import torch
    say("batched cancel")
    h = I.helmholtz_input(1024)
    mk = lambda: (torch.zeros((1024, 1024), dtype=torch.float64, device="cuda:0"),
                  torch.from_numpy(h.g).to("cuda:0"))
    cond = L.make_cond(L.LSR_COND_BELOW, 1e-9, 10)
    # two million sweeps of 1024^2 take seconds: both jobs are still running or
    # queued when the cancels arrive
    (t1, g1), (t2, g2) = mk(), mk()
    j1 = bctx.submit(t1, L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA, cond, 2_000_000, L.LSR_BC_RING,
                     env0=g1, param=(h.alpha, h.h))
    j2 = bctx.submit(t2, L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA, cond, 2_000_000, L.LSR_BC_RING,
                     env0=g2, param=(h.alpha, h.h))
    out = L._native.lsr_job_result()
    assert L._native.lib().lsr_result(bctx.handle, j1, 0, L._native.C.byref(out)) == L.LSR_EBUSY
    bctx.cancel(j2)
    bctx.cancel(j1)
    for j in (j1, j2):
        r = bctx.result(j)
        assert r.status == L.LSR_ECANCELED
        assert 0 <= r.iterations < 2_000_000 and not r.converged


def test_restoration_with_nothing_flagged_stops_at_once(bctx):
    """A restoration job with an all-zero mask on a batched context: no pixel
    changes, so the first check (r = 0 < 0.1) stops it and the field is unchanged."""
    import torch
    say("restore on batched, empty mask")
    u0 = torch.arange(256, dtype=torch.float64, device="cuda:0").reshape(16, 16)
    u = u0.clone()
    m = torch.zeros((16, 16), dtype=torch.uint8, device="cuda:0")
    r = bctx.result(bctx.submit(u, L.LSR_ST_RESTORE, L.LSR_RED_MAX_ABS_DELTA,
                                L.make_cond(L.LSR_COND_BELOW, 0.1), 10, L.LSR_BC_BOTTOM, env0=m,
                                param=(100.0, 0.0)))
    torch.cuda.synchronize()
    assert r.status == L.LSR_OK and r.iterations == 1 and r.converged and r.last_reduce == 0.0
    assert torch.equal(u, u0)


def test_stops_inside_rounds_are_replayed(bctx):
    """Jobs whose checks fall inside a fused round (check every sweep, a cap that is
    not a multiple of the depth) stop at exactly the oracle's sweep, alone and mixed."""
    import torch
    say("batched stops inside rounds")
    a = I.laplace_input(96, 100, seed=21)
    h = I.helmholtz_input(131)
    cases = []
    for thr in (3e-3, 2.44e-3, 1.98e-3):      # stop at sweeps 81, 97, 117 (check every sweep)
        t = torch.from_numpy(a).to("cuda:0")
        kw = dict(stencil_id=L.LSR_ST_LAPLACE5, reduce_op=L.LSR_RED_MAX_ABS_DELTA,
                  cond=L.make_cond(L.LSR_COND_BELOW, thr, 1), max_iter=3000, bc=L.LSR_BC_RING)
        cases.append((t, kw, lambda thr=thr: O.jacobi_run(a, thr=thr, max_iter=3000), None))
    for cap in (123, 7):
        t = torch.from_numpy(h.u0).to("cuda:0")
        g = torch.from_numpy(h.g).to("cuda:0")
        kw = dict(stencil_id=L.LSR_ST_HELMHOLTZ5, reduce_op=L.LSR_RED_L2_DELTA,
                  cond=L.make_cond(L.LSR_COND_BELOW, 1e-12, 10), max_iter=cap, bc=L.LSR_BC_RING,
                  env0=g, param=(h.alpha, h.h))
        ora = lambda cap=cap: O.jacobi_run(h.u0, helmholtz=True, g=h.g, alpha=h.alpha, h=h.h,
                                           reduce_op=O.RED_L2_DELTA, thr=1e-12, check_every=10,
                                           max_iter=cap)
        cases.append((t, kw, ora, g))
    ids = [_submit(bctx, t, kw) for (t, kw, _, _) in cases]
    for (t, kw, ora, _), jid in zip(cases, ids):
        r = bctx.result(jid)
        torch.cuda.synchronize()
        o, ro = ora()
        assert r.status == L.LSR_OK and r.iterations == ro.n, (r.iterations, ro.n)
        assert bool(r.converged) == ro.converged
        assert np.array_equal(t.cpu().numpy(), o)
        assert abs(r.last_reduce - ro.r) <= 1e-12 * ro.r


# (rows, cols, torus, cond, check_every, max_iter): every large Life job takes the
# fused family (8 generations per round), also rows that do not hold a multiple of
# 16 cells (dead border: masked padding; torus: edge lanes gathered from the
# wrapped columns)
FUSED_LIFE = [(320, 512, True, L.LSR_COND_STABLE_FOR, 1, 700),
              (300, 1000, False, L.LSR_COND_STABLE_FOR, 1, 700),   # rows end in padding
              (130, 3003, False, L.LSR_COND_NEVER, 1, 61),
              (999, 333, False, L.LSR_COND_STABLE_FOR, 2, 500),
              (300, 1008, False, L.LSR_COND_STABLE_FOR, 1, 900),   # a 16-column second window
              (257, 2000, True, L.LSR_COND_STABLE_FOR, 3, 400),
              (200, 1984, False, L.LSR_COND_NEVER, 1, 123),        # cap inside a round
              (333, 496, True, L.LSR_COND_NEVER, 5, 61),
              (300, 500, True, L.LSR_COND_STABLE_FOR, 1, 300),     # torus, not a multiple of 16
              (257, 1000, True, L.LSR_COND_STABLE_FOR, 3, 400),
              (600, 301, True, L.LSR_COND_NEVER, 1, 77),
              (130, 2001, True, L.LSR_COND_STABLE_FOR, 1, 500),
              (2000, 131, True, L.LSR_COND_NEVER, 2, 100)]


def test_fused_life_rounds_match_oracle(bctx):
    """Life jobs on the fused batched family (8 generations per round, counts of
    every checked generation inside a round, a stop inside a round replayed one
    generation at a time) equal the oracle bit for bit: field, stop generation and
    live count, also on dead borders and tori whose rows end in padding."""
    import torch
    say("batched fused life")
    cases = []
    for k, (rows, cols, torus, cond, every, mi) in enumerate(FUSED_LIFE):
        a = I.life_input(rows, cols, seed=40 + k)
        t = torch.from_numpy(a).to("cuda:0")
        c = L.make_cond(cond, 0.0, every, 10)
        jid = bctx.submit(t, L.LSR_ST_LIFE, L.LSR_RED_SUM, c, mi,
                          L.LSR_BC_TORUS if torus else L.LSR_BC_BOTTOM)
        cases.append((rows, cols, torus, cond, every, mi, a, t, jid))
    for rows, cols, torus, cond, every, mi, a, t, jid in cases:
        r = bctx.result(jid)
        torch.cuda.synchronize()
        o, ro = O.life_run(a, bc=O.BC_TORUS if torus else O.BC_BOTTOM,
                           cond=O.COND_STABLE_FOR if cond == L.LSR_COND_STABLE_FOR else O.COND_NEVER,
                           stable_window=10, check_every=every, max_iter=mi)
        name = (rows, cols, torus, every, mi)
        assert r.status == L.LSR_OK, name
        assert r.sweeps_per_launch == 8, name
        assert r.iterations == ro.n and r.last_count == ro.count, (name, r.iterations, ro.n)
        assert np.array_equal(t.cpu().numpy(), o), name


def test_fused_life_stop_inside_a_round(bctx):
    """A still life plus a blinker on a wide dead-border grid: the live count is
    constant from generation 0, so a stable window of 10 stops at generation 10,
    inside the second fused round; the engine replays generations 9 and 10."""
    import torch
    say("batched fused life, stop inside a round")
    cells = [(5, 5), (5, 6), (6, 5), (6, 6),           # block
             (40, 991), (40, 992), (40, 993)]         # blinker across the first window seam
    for window, stop in ((10, 10), (5, 5), (17, 17)):
        a = I.life_pattern(96, 1024, cells)
        t = torch.from_numpy(a).to("cuda:0")
        r = bctx.run(t, L.LSR_ST_LIFE, L.LSR_RED_SUM, L.make_cond(L.LSR_COND_STABLE_FOR, 0.0, 1, window),
                     500, L.LSR_BC_BOTTOM)
        torch.cuda.synchronize()
        o, ro = O.life_run(a, bc=O.BC_BOTTOM, stable_window=window, max_iter=500)
        assert ro.n == stop and r.iterations == stop and r.sweeps_per_launch == 8
        assert r.last_count == 7 and np.array_equal(t.cpu().numpy(), o)


SMALL_LIFE = [(1, 1), (1, 7), (2, 2), (3, 3), (5, 1), (7, 131), (64, 99), (33, 250), (250, 33),
              (200, 203), (280, 280)]


def test_small_life_grids_in_lds_match_oracle(bctx):
    """Life grids whose two buffers fit in LDS run their whole loop in one workgroup
    (one 32-bit word of 4 cells per thread, ghost bytes for the torus wrap): every
    width modulo 4, single rows and columns, both borders, equal to the oracle in
    field, stop generation and count."""
    import torch
    say("batched small life shapes")
    cases = []
    for k, (rows, cols) in enumerate(SMALL_LIFE):
        for torus in (True, False):
            a = I.life_input(rows, cols, seed=rows * 1000 + cols, density=0.4)
            t = torch.from_numpy(a).to("cuda:0")
            jid = bctx.submit(t, L.LSR_ST_LIFE, L.LSR_RED_SUM,
                              L.make_cond(L.LSR_COND_STABLE_FOR, 0.0, 1 + k % 3, 10), 300,
                              L.LSR_BC_TORUS if torus else L.LSR_BC_BOTTOM)
            cases.append((rows, cols, torus, 1 + k % 3, a, t, jid))
    for rows, cols, torus, every, a, t, jid in cases:
        r = bctx.result(jid)
        torch.cuda.synchronize()
        o, ro = O.life_run(a, bc=O.BC_TORUS if torus else O.BC_BOTTOM, stable_window=10,
                           check_every=every, max_iter=300)
        name = (rows, cols, torus, every)
        assert r.status == L.LSR_OK, name
        assert r.iterations == ro.n and r.last_count == ro.count, (name, r.iterations, ro.n)
        assert np.array_equal(t.cpu().numpy(), o), name


@pytest.mark.parametrize("f32", [True, False])
def test_reduce_kind_leaves_the_field_unchanged(f32):
    """The tiles with a job's usual reduce compiled in (Helmholtz L2, Laplace max
    |delta|) and the general tile (any other reduce) compute the same field bit for
    bit, on a batched context (depth 5, checks inside the rounds for Laplace) and on
    a plain one (two-wavefront launches at depths 5 and 10)."""
    import torch
    say(f"reduce kinds, same field f32={f32}")
    dt = torch.float32 if f32 else torch.float64
    h = I.helmholtz_input(300)
    lap = I.laplace_input(300, seed=4)
    cases = [(L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA, 10), (L.LSR_ST_HELMHOLTZ5, L.LSR_RED_MAX_ABS_DELTA, 10),
             (L.LSR_ST_LAPLACE5, L.LSR_RED_MAX_ABS_DELTA, 1), (L.LSR_ST_LAPLACE5, L.LSR_RED_L2_DELTA, 1),
             (L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA, 1), (L.LSR_ST_HELMHOLTZ5, L.LSR_RED_MAX_ABS_DELTA, 1)]
    fields = {}
    for batched in (True, False):
        with L.Context(0, batched=batched) as c:
            for st, red, every in cases:
                helm = st == L.LSR_ST_HELMHOLTZ5
                t = torch.from_numpy(h.u0 if helm else lap).to("cuda:0").to(dt)
                g = torch.from_numpy(h.g).to("cuda:0").to(dt) if helm else None
                r = c.run(t, st, red, L.make_cond(L.LSR_COND_NEVER, 0.0, every), 200, L.LSR_BC_RING,
                          env0=g, param=(h.alpha, h.h) if helm else ())
                torch.cuda.synchronize()
                assert r.status == L.LSR_OK and r.iterations == 200
                fields[(batched, st, red, every)] = t.cpu().numpy()
    for batched in (True, False):
        for st, every in ((L.LSR_ST_HELMHOLTZ5, 10), (L.LSR_ST_LAPLACE5, 1), (L.LSR_ST_HELMHOLTZ5, 1)):
            a = fields[(batched, st, L.LSR_RED_L2_DELTA, every)]
            b = fields[(batched, st, L.LSR_RED_MAX_ABS_DELTA, every)]
            assert np.array_equal(a, b), (batched, st, every)
