"""The autotuner through the C ABI: it measures candidates on the device, later
automatic jobs of the same key take its winner (results still match the oracle
exactly), and its table round-trips through JSON."""
import json

import numpy as np
import pytest

import oracle as O
import paper_1609_04567_amd as L
from paper_1609_04567_amd import inputs as I
from gpu_helpers import run_jacobi, run_life, say

pytestmark = pytest.mark.gpu


@pytest.fixture()
def tctx():
    c = L.Context(0)
    yield c
    c.close()


def test_helmholtz_tuned_job_matches_oracle(tctx):
    say("autotune helmholtz 300^2 fp64")
    best = tctx.autotune(L.LSR_ST_HELMHOLTZ5, L.LSR_F64, 300, 300, 10, 160)
    say(f"  winner tile_rows={best.tile_rows} depth={best.tb_depth} waves={best.waves} "
        f"unroll={best.unroll}")
    table = json.loads(L.lsr_tune_export(tctx.handle))
    assert table["arch"].startswith("gfx")
    (e,) = table["entries"]
    assert (e["stencil"], e["dtype"], e["bc"], e["rows_log2"], e["cols_log2"], e["check_every"]) == \
        (L.LSR_ST_HELMHOLTZ5, L.LSR_F64, L.LSR_BC_RING, 9, 9, 10)
    assert (e["tile_rows"], e["tb_depth"], e["waves"], e["unroll"]) == \
        (best.tile_rows, best.tb_depth, best.waves, best.unroll) and e["us_per_sweep"] > 0
    h = I.helmholtz_input(300)
    o, ro = O.jacobi_run(h.u0, helmholtz=True, g=h.g, alpha=1.0, h=h.h, reduce_op=O.RED_L2_DELTA,
                         thr=1e-9, check_every=10, max_iter=160)
    x, r = run_jacobi(tctx, h.u0, helm=True, g=h.g, alpha=1.0, h=h.h, reduce_op=L.LSR_RED_L2_DELTA,
                      thr=1e-9, check_every=10, max_iter=160)
    assert r.iterations == 160 and np.array_equal(x, o)
    assert r.sweeps_per_launch == max(best.tb_depth, 1)


def test_life_tuned_job_matches_oracle(tctx):
    say("autotune life 200x208")
    tctx.autotune(L.LSR_ST_LIFE, L.LSR_U8, 200, 208, 1, 300)
    # both boundaries are measured and keyed separately
    keys = sorted(e["bc"] for e in json.loads(L.lsr_tune_export(tctx.handle))["entries"])
    assert keys == [L.LSR_BC_TORUS, L.LSR_BC_BOTTOM]
    a = I.life_input(200, 208, seed=3)
    for torus, bc in ((True, O.BC_TORUS), (False, O.BC_BOTTOM)):
        o, ro = O.life_run(a, bc=bc, stable_window=10, max_iter=300)
        x, r = run_life(tctx, a, torus=torus, window=10, max_iter=300)
        assert r.iterations == ro.n and np.array_equal(x, o)


_ENTRY = {"stencil": 3, "dtype": 1, "bc": 1, "rows_log2": 8, "cols_log2": 8, "check_every": 1,
          "tile_rows": 0, "tb_depth": 8, "waves": 0, "unroll": 0, "us_per_sweep": 1.0}


@pytest.mark.parametrize("bad", [{"stencil": 4}, {"stencil": 9}, {"tb_depth": 7}, {"tb_depth": 3, "stencil": 2,
                                  "dtype": 8, "bc": 0}, {"bc": 0}, {"dtype": 8}, {"tile_rows": -2},
                                 {"tile_rows": 100000}, {"waves": 2}, {"check_every": 0},
                                 {"tb_depth": 2.5}])
def test_import_rejects_entries_the_library_cannot_run(tctx, bad):
    say(f"tune import rejects {bad}")
    base = {"arch": json.loads(L.lsr_tune_export(tctx.handle))["arch"], "entries": [dict(_ENTRY)]}
    L.lsr_tune_import(tctx.handle, json.dumps(base))       # the valid entry is taken
    good = L.lsr_tune_export(tctx.handle)
    e = dict(_ENTRY)
    e.update(bad)
    with pytest.raises(L.LsrError) as ei:
        L.lsr_tune_import(tctx.handle, json.dumps({"arch": base["arch"], "entries": [e]}))
    assert ei.value.status == L.LSR_EINVAL
    assert L.lsr_tune_export(tctx.handle) == good         # the table is unchanged


def test_table_round_trips_and_rejects_other_arch(tctx):
    say("autotune table round trip")
    tctx.autotune(L.LSR_ST_LAPLACE5, L.LSR_F32, 130, 100, 1, 200)
    text = L.lsr_tune_export(tctx.handle)
    other = L.Context(0)
    try:
        L.lsr_tune_import(other.handle, text)
        assert L.lsr_tune_export(other.handle) == text
        bad = text.replace(json.loads(text)["arch"], "gfx000")
        with pytest.raises(L.LsrError):
            L.lsr_tune_import(other.handle, bad)
        assert L.lsr_tune_export(other.handle) == text
    finally:
        other.close()


def test_batched_context_tunes_its_own_families():
    """On a batched context the autotuner measures the engine's settings (fused
    depth where it divides the check period, band rows; Life band rows), later
    jobs of the key run with the winner, and their fields equal the default
    geometry's bit for bit (Life: and the oracle's)."""
    import torch
    say("batched autotune")
    h = I.helmholtz_input(300)
    life = I.life_input(200, seed=6)
    c = L.Context(0, batched=True)
    try:
        with pytest.raises(L.LsrError) as ei:
            c.autotune(L.LSR_ST_RESTORE, L.LSR_F32, 64, 64, 1)
        assert ei.value.status == L.LSR_EINVAL
        # a job still running on the context: the tuner would change its settings
        big = torch.zeros((2048, 2048), dtype=torch.float32, device="cuda:0")
        busy = c.submit(big, L.LSR_ST_LAPLACE5, L.LSR_RED_MAX_ABS_DELTA,
                        L.make_cond(L.LSR_COND_NEVER, 0.0, 1), 4000, L.LSR_BC_RING)
        with pytest.raises(L.LsrError) as ei:
            c.autotune(L.LSR_ST_LAPLACE5, L.LSR_F32, 300, 300, 1, 40)
        assert ei.value.status == L.LSR_EBUSY
        assert c.result(busy).status == L.LSR_OK
        best = c.autotune(L.LSR_ST_HELMHOLTZ5, L.LSR_F32, 300, 300, 10, 160)
        assert best.tb_depth in (5, 2) and best.tile_rows in (8, 16, 24, 32, 48, 64)
        assert best.waves == 0 and best.unroll == 0
        lb = c.autotune(L.LSR_ST_LIFE, L.LSR_U8, 200, 200, 1, 240)
        assert lb.tb_depth in (1, 8) and lb.tile_rows in (8, 16, 32, 64, 128)
        entries = json.loads(L.lsr_tune_export(c.handle))["entries"]
        assert len(entries) == 3   # Helmholtz, Life torus, Life dead border
        t = torch.from_numpy(h.u0.astype(np.float32)).to("cuda:0")
        g = torch.from_numpy(h.g.astype(np.float32)).to("cuda:0")
        r = c.run(t, L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA,
                  L.make_cond(L.LSR_COND_BELOW, 1e-9, 10), 160, L.LSR_BC_RING, env0=g,
                  param=(h.alpha, h.h))
        assert r.sweeps_per_launch == best.tb_depth
        s = torch.from_numpy(life).to("cuda:0")
        rl = c.run(s, L.LSR_ST_LIFE, L.LSR_RED_SUM, L.make_cond(L.LSR_COND_STABLE_FOR, 0.0, 1, 10),
                   300, L.LSR_BC_TORUS)
        torch.cuda.synchronize()
        xt, xs = t.cpu().numpy(), s.cpu().numpy()
    finally:
        c.close()
    with L.Context(0, batched=True) as d:
        t2 = torch.from_numpy(h.u0.astype(np.float32)).to("cuda:0")
        g2 = torch.from_numpy(h.g.astype(np.float32)).to("cuda:0")
        r2 = d.run(t2, L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA,
                   L.make_cond(L.LSR_COND_BELOW, 1e-9, 10), 160, L.LSR_BC_RING, env0=g2,
                   param=(h.alpha, h.h))
        torch.cuda.synchronize()
        assert r2.iterations == r.iterations == 160
        assert np.array_equal(t2.cpu().numpy(), xt)
    o, ro = O.life_run(life, bc=O.BC_TORUS, cond=O.COND_STABLE_FOR, stable_window=10, max_iter=300)
    assert rl.iterations == ro.n and np.array_equal(xs, o)


def test_batched_jobs_take_the_table_entry():
    """A batched context reads the same tuning table: an imported entry for a job's
    key sets its fused depth and band height inside the rounds, and the field is
    bit-identical to the one the default geometry gives (every level evaluates the
    same update with the same rounding keys)."""
    import torch
    say("batched job with an imported tuning entry")
    h = I.helmholtz_input(300)
    out = {}
    for tuned in (False, True):
        c = L.Context(0, batched=True)
        try:
            if tuned:
                table = json.loads(L.lsr_tune_export(c.handle))
                table["entries"] = [{"stencil": L.LSR_ST_HELMHOLTZ5, "dtype": L.LSR_F32,
                                     "bc": L.LSR_BC_RING, "rows_log2": 9, "cols_log2": 9, "check_every": 10,
                                     "tile_rows": 16, "tb_depth": 2, "waves": 0, "unroll": 0,
                                     "us_per_sweep": 1.0}]
                L.lsr_tune_import(c.handle, json.dumps(table))
            t = torch.from_numpy(h.u0.astype(np.float32)).to("cuda:0")
            g = torch.from_numpy(h.g.astype(np.float32)).to("cuda:0")
            r = c.run(t, L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA,
                      L.make_cond(L.LSR_COND_BELOW, 1e-9, 10), 160, L.LSR_BC_RING, env0=g,
                      param=(h.alpha, h.h))
            torch.cuda.synchronize()
            out[tuned] = (t.cpu().numpy(), r)
        finally:
            c.close()
    (x0, r0), (x1, r1) = out[False], out[True]
    assert r0.sweeps_per_launch == 5 and r1.sweeps_per_launch == 2
    assert r0.iterations == r1.iterations == 160
    assert np.array_equal(x0, x1)
    assert abs(r1.last_reduce - r0.last_reduce) <= 1e-12 * abs(r0.last_reduce)
