"""Benchmark of the loop-of-stencil-reduce hot path on one MI355X.

Default workload (the configuration the headline metric is quoted on): the
Helmholtz Jacobi solver, 8192 x 8192 FP64 grid including the boundary ring,
alpha = 1, manufactured solution sin(pi x) sin(pi y); the L2 norm of the update
is reduced every 10 sweeps, stop below 1e-9 or at 5000 sweeps (it always reaches
the cap: the closed form gives ||update|| ~ 3.2e-4 there). One step = one whole
lsr_run job (5000 sweeps with the reduce fused in, 10 per launch at the automatic
depth, and 500 on-device checks) from a zero interior that is already resident in
HBM.

value = whole-job GLUP/s (interior cells x sweeps / wall time of the step,
host API overhead included). roofline: the fused kernel's compulsory traffic per
launch (24 B per interior cell: read u and g, write u, once per launch whatever
the number of sweeps it fuses), divided by its mean launch time measured with HIP
events on the library's own stream (the job's device time over its launches, so
it also carries the small finalize kernels and launch gaps), against 8 TB/s.
plain_sweep: the same job run with one sweep per launch, outside the timed
region, and its own fraction of 8 TB/s.

Other workloads (--workload): laplace (256^2 FP64, 2000 sweeps), life (16384^2
u8 torus, 2000 generations, 8 per launch; its roofline is the vector ALU's), restore (4096^2 two-phase restoration, FP64 and
FP32), served (a prefix of the mixed job stream through the batched engine in
FP32 storage, against the plain per-grid FP64 path on the same jobs).

--gpus N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# 32-bit vector lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
PEAK_VALU_TOPS = 39.32
# lane operations of the fused Life kernel's level body per cell and generation,
# per 16 cells: column sums 8, byte shifts 8 + 2 lane shifts, 3x3 totals 4, the
# rule 16, the count 6 (44 instructions of its compiled loop)
LIFE_OPS_PER_CELL = 44 / 16
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_hash(files=("jacobi.hip", "jacobi_tb.hip", "tile_jacobi.hpp",
                              "common.hpp")) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1609_04567_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name: str, files=None):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None when the
    kernel source changed since they were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        d = json.load(fh)
    e = d.get(name)
    h = kernel_source_hash(files) if files else kernel_source_hash()
    if not e or e.get("source_hash") != h:
        return None
    return e.get("bytes_per_launch")


def base_line(metric, value, unit, steps, warmup, ms_per_step, dtype, config, higher=True):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": ms_per_step, "higher_is_better": higher,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": config}


def copy_probe(L, ctx, torch, dev):
    nb = 1 << 30
    src = torch.empty(nb, dtype=torch.uint8, device=dev)
    dst = torch.empty(nb, dtype=torch.uint8, device=dev)
    ms = L.lsr_probe_copy(ctx.handle, dst.data_ptr(), src.data_ptr(), nb, 20)
    return round(2 * nb / (ms * 1e-3) / 1e9, 1)


def roofline(alg_bytes_per_launch, per_launch_s, traffic):
    achieved = alg_bytes_per_launch / per_launch_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic}


# ---------------------------------------------------------------------------
def run_helmholtz(args, L, I, torch):
    n, sweeps = args.n or 8192, args.sweeps or 5000
    dev = "cuda:0"
    h = I.helmholtz_input(n)
    g = torch.from_numpy(h.g).to(dev)
    grids = [torch.zeros((n, n), dtype=torch.float64, device=dev)
             for _ in range(args.steps + args.warmup)]
    ustar = torch.from_numpy(h.ustar).to(dev)
    cond = L.make_cond(L.LSR_COND_BELOW, 1e-9, 10)
    ctx = L.Context(0)
    ctx.tune(tile_rows=args.tile_rows, tb_depth=args.tb, chunk=args.chunk, use_graph=args.graph,
             waves=args.waves, unroll=args.unroll)
    copy_gbs = copy_probe(L, ctx, torch, dev)
    tuned = None
    if args.autotune:
        t0 = time.perf_counter()
        b = ctx.autotune(L.LSR_ST_HELMHOLTZ5, L.LSR_F64, n, n, 10, sweeps)
        tuned = {"tile_rows": b.tile_rows, "tb_depth": b.tb_depth, "waves": b.waves,
                 "unroll": b.unroll, "tuning_s": round(time.perf_counter() - t0, 2)}
        print(f"autotune: {tuned}", file=sys.stderr, flush=True)

    if args.form == "sep":
        # the -i form: g from the cell's indices and the factor vectors (same result)
        sv, hh = I.helmholtz_factor(n)
        fac = torch.from_numpy(sv).to(dev)

        def step(t):
            return ctx.run(t, L.LSR_ST_HELMHOLTZ5_SEP, L.LSR_RED_L2_DELTA, cond, sweeps,
                           L.LSR_BC_RING, env0=fac, env1=fac,
                           param=(h.alpha, h.h, 2 * math.pi ** 2 + h.alpha, hh * hh))
    else:
        def step(t):
            return ctx.run(t, L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA, cond, sweeps, L.LSR_BC_RING,
                           env0=g, param=(h.alpha, h.h))

    for k in range(args.warmup):
        r = step(grids[k])
        print(f"warmup {k}: n={r.iterations} device_ms={r.device_ms:.1f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step(grids[args.warmup + k]) for k in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for k, r in enumerate(results):
        print(f"step {k}: n={r.iterations} device_ms={r.device_ms:.1f}", file=sys.stderr, flush=True)
        assert r.status == L.LSR_OK and r.iterations == sweeps
    value = (n - 2) ** 2 * sweeps * args.steps / wall / 1e9
    # closed form of the last step, u^n = c*(1 - mu^n) u*, with 1 - mu written
    # without cancellation (it is 7.7e-8 at N = 8192)
    hh = 1.0 / (n - 1)
    s2 = math.sin(math.pi * hh / 2) ** 2
    one_m_mu = (8.0 * s2 + hh * hh) / (4.0 + hh * hh)
    lam = 8.0 / (hh * hh) * s2
    coef = (2 * math.pi ** 2 + 1.0) / (lam + 1.0) * -math.expm1(sweeps * math.log1p(-one_m_mu))
    err = float((grids[-1] - coef * ustar).abs().max() / (coef * ustar).abs().max())
    dev_ms = sum(r.device_ms for r in results)
    spl = int(results[-1].sweeps_per_launch)   # sweeps fused per launch (1 = unfused)
    per_launch_s = dev_ms * 1e-3 / (sweeps // spl * args.steps)
    out = base_line("GLUP/s", round(value, 3), "GLUP/s", args.steps, args.warmup,
                    round(wall / args.steps * 1e3, 3), "f64",
                    {"workload": f"helmholtz-jacobi5 {n}x{n} fp64, L2 of update every 10 sweeps, "
                                 f"stop <1e-9 or {sweeps} sweeps", "rows": n, "cols": n,
                     "sweeps": sweeps, "check_every": 10, "sweeps_per_launch": spl,
                     "parallelism": "single-gpu"})
    # a launch reads u and g and writes u once, whatever number of sweeps it fuses
    kname = f"jacobi5_helmholtz_f64_{n}" if spl == 1 else f"jacobi5_tb{spl}_helmholtz_f64_{n}"
    bpc = 24.0 if args.form == "array" else 16.0   # the -i form reads no g array
    if args.form == "sep":
        kname += "_sep"
        out["config"]["workload"] += ", right-hand side from the indices (-i form)"
    out["roofline"] = roofline(bpc * (n - 2) ** 2, per_launch_s, measured_traffic(kname))
    out["roofline"]["basis"] = (f"compulsory bytes of one launch of {spl} fused sweeps: {bpc:.0f} B "
                                "per interior cell (u read and written once"
                                + (", g read once" if bpc == 24.0 else "") +
                                "), over the launch's mean device time")
    out["copy_probe_gbs"] = copy_gbs
    if tuned:
        out["autotuned"] = tuned
    # bytes an unfused sweep would move per update, at the achieved update rate
    out["effective_gbs"] = round(value * 24.0, 1)
    out["effective"] = {"gbs": round(value * 24.0, 1), "frac": round(value * 24.0 / PEAK_HBM_GBS, 4),
                        "basis": "24 B per cell update (an unfused sweep's traffic) x the whole "
                                 "job's update rate; above 1 because fused sweeps reuse data on chip"}
    out["accuracy"] = {"closed_form_max_rel_err": err, "iterations": int(results[-1].iterations),
                       "last_l2_update": results[-1].last_reduce}
    if spl > 1 and not args.no_plain:
        # the same job with one sweep per launch (outside the timed region): the plain
        # sweep's own fraction of HBM bandwidth, 24 bytes per update
        pctx = L.Context(0)
        pctx.tune(tb_depth=1)
        ps = 500
        grids[0].zero_()
        rp = pctx.run(grids[0], L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA, cond, ps, L.LSR_BC_RING,
                      env0=g, param=(h.alpha, h.h))
        assert rp.status == L.LSR_OK and rp.iterations == ps and rp.sweeps_per_launch == 1
        sweep_s = rp.device_ms * 1e-3 / ps
        out["plain_sweep"] = {"glups": round((n - 2) ** 2 / sweep_s / 1e9, 1), "sweeps": ps,
                              "roofline": roofline(24.0 * (n - 2) ** 2, sweep_s,
                                                   measured_traffic(f"jacobi5_helmholtz_f64_{n}"))}
        pctx.close()
    if not args.no_cpu:
        import oracle as O
        t0 = time.perf_counter()
        _, r = O.jacobi_run(h.u0, helmholtz=True, g=h.g, alpha=h.alpha, h=h.h,
                            reduce_op=O.RED_L2_DELTA, thr=1e-9, check_every=10,
                            max_iter=args.cpu_sweeps)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round((n - 2) ** 2 * r.n / dt / 1e9, 4), "unit": "GLUP/s",
                               "cores": O.threads(), "kind": "oracle",
                               "sample": f"first {r.n} sweeps of the {n}x{n} job ({dt:.1f} s)"}
        # the same oracle on one core, over a shorter prefix
        cores = O.threads()
        O.set_threads(1)
        k1 = max(1, args.cpu_sweeps // 75)
        t0 = time.perf_counter()
        _, r1 = O.jacobi_run(h.u0, helmholtz=True, g=h.g, alpha=h.alpha, h=h.h,
                             reduce_op=O.RED_L2_DELTA, thr=1e-9, check_every=10, max_iter=k1)
        dt1 = time.perf_counter() - t0
        O.set_threads(cores)
        out["cpu_baseline_1core"] = {"value": round((n - 2) ** 2 * r1.n / dt1 / 1e9, 4),
                                     "unit": "GLUP/s", "cores": 1, "kind": "oracle",
                                     "sample": f"first {r1.n} sweeps ({dt1:.1f} s)",
                                     "all_core_speedup": round(out["cpu_baseline"]["value"] /
                                                               ((n - 2) ** 2 * r1.n / dt1 / 1e9), 2),
                                     "all_cores": cores}
    ctx.close()
    return out


def run_laplace(args, L, I, torch):
    import numpy as np
    n, sweeps = args.n or 256, args.sweeps or 2000
    a = I.laplace_input(n, seed=1)
    grids = [torch.from_numpy(a).to("cuda:0") for _ in range(args.steps + args.warmup)]
    ctx = L.Context(0)
    ctx.tune(tile_rows=args.tile_rows, tb_depth=args.tb, chunk=args.chunk, use_graph=args.graph,
             waves=args.waves, unroll=args.unroll)
    cond = L.make_cond(L.LSR_COND_BELOW, 1e-6, 1)
    step = lambda t: ctx.run(t, L.LSR_ST_LAPLACE5, L.LSR_RED_MAX_ABS_DELTA, cond, sweeps,
                             L.LSR_BC_RING)
    for k in range(args.warmup):
        step(grids[k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step(grids[args.warmup + k]) for k in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert all(r.iterations == sweeps for r in results)
    value = (n - 2) ** 2 * sweeps * args.steps / wall / 1e9
    per_launch_s = sum(r.device_ms for r in results) * 1e-3 / (sweeps * args.steps)
    out = base_line("GLUP/s", round(value, 4), "GLUP/s", args.steps, args.warmup,
                    round(wall / args.steps * 1e3, 3), "f64",
                    {"workload": f"laplace-jacobi5 {n}x{n} fp64, max|update| every sweep, "
                                 f"stop <1e-6 or {sweeps}", "rows": n, "cols": n, "sweeps": sweeps})
    out["sweeps_per_s"] = round(sweeps * args.steps / wall, 1)
    out["roofline"] = roofline(16.0 * (n - 2) ** 2, per_launch_s, None)
    out["roofline"]["note"] = "1 MiB working set: cache-resident and launch-bound; HBM % is context"
    if not args.no_cpu:
        import oracle as O
        cores = O.threads()
        O.set_threads(1)
        t0 = time.perf_counter()
        o, ro = O.jacobi_run(a, thr=1e-6, max_iter=sweeps)
        dt = time.perf_counter() - t0
        O.set_threads(cores)
        out["cpu_baseline"] = {"value": round((n - 2) ** 2 * ro.n / dt / 1e9, 4), "unit": "GLUP/s",
                               "cores": 1, "kind": "oracle", "sample": f"the whole job ({dt:.2f} s)"}
        out["accuracy"] = {"bit_identical_to_oracle": bool(np.array_equal(grids[-1].cpu().numpy(), o))}
    ctx.close()
    return out


def run_life(args, L, I, torch):
    import numpy as np
    n, gens = args.n or 16384, args.sweeps or 2000
    s = I.life_input(n, seed=3)
    grids = [torch.from_numpy(s).to("cuda:0") for _ in range(args.steps + args.warmup)]
    ctx = L.Context(0)
    ctx.tune(tile_rows=args.tile_rows, tb_depth=args.tb, chunk=args.chunk, use_graph=args.graph)
    copy_gbs = copy_probe(L, ctx, torch, "cuda:0")
    cond = L.make_cond(L.LSR_COND_STABLE_FOR, 0.0, 1, 10)
    step = lambda t: ctx.run(t, L.LSR_ST_LIFE, L.LSR_RED_SUM, cond, gens, L.LSR_BC_TORUS)
    for k in range(args.warmup):
        step(grids[k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step(grids[args.warmup + k]) for k in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lups = sum(n * n * r.iterations for r in results)
    spl = int(results[-1].sweeps_per_launch)   # generations fused per launch
    launches = sum(-(-r.iterations // spl) for r in results)
    per_launch_s = sum(r.device_ms for r in results) * 1e-3 / launches
    value = lups / wall / 1e9
    out = base_line("GLUP/s", round(value, 2), "GLUP/s", args.steps, args.warmup,
                    round(wall / args.steps * 1e3, 3), "u8",
                    {"workload": f"life-b3s23 {n}x{n} u8 torus, live count every generation, "
                                 f"stop when unchanged for 10 or {gens}", "rows": n, "cols": n,
                     "generations": gens, "generations_per_launch": spl})
    # a launch reads and writes every cell once, whatever number of generations it fuses
    if spl == 1:
        kname, files = f"life_swar_{n}", ("life.hip", "tile_life.hpp", "common.hpp")
        out["roofline"] = roofline(2.0 * n * n, per_launch_s, measured_traffic(kname, files))
    else:
        # fused generations are bound by the vector ALU: LIFE_OPS_PER_CELL 32-bit
        # lane operations per cell and generation against the chip's lane rate
        kname, files = f"life_tb{spl}_{n}", ("life_tb.hip", "tile_life_tb.hpp", "tile_life.hpp", "common.hpp")
        achieved = n * n * spl * LIFE_OPS_PER_CELL / per_launch_s / 1e12
        out["roofline"] = {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK_VALU_TOPS,
                           "unit": "Tops/s", "frac": round(achieved / PEAK_VALU_TOPS, 4),
                           "traffic": measured_traffic(kname, files)}
        out["hbm_per_launch"] = roofline(2.0 * n * n, per_launch_s, None)
    out["copy_probe_gbs"] = copy_gbs
    # bytes an unfused generation would move per cell, at the achieved update rate
    out["effective_gbs"] = round(value * 2.0, 1)
    out["result"] = {"iterations": int(results[-1].iterations), "count": int(results[-1].last_count)}
    golden = os.path.join(ROOT, "tests", "golden", f"life_{n}_torus_seed3.txt")
    if gens == 2000 and os.path.exists(golden):
        # the oracle's full run of this workload (stop generation, final count,
        # SHA-256 of the final grid), written by tests/golden/make_life_golden.py
        vals = {}
        with open(golden) as fh:
            for line in fh:
                if line.strip() == "trajectory":
                    break
                if not line.startswith("#") and line.strip():
                    k, v = line.split()
                    vals[k] = v
        digest = hashlib.sha256(grids[-1].cpu().numpy().tobytes()).hexdigest()
        out["accuracy"] = {"oracle_n": int(vals["n"]), "oracle_count": int(vals["count"]),
                           "bit_identical_to_oracle": bool(
                               digest == vals["sha256"] and
                               int(results[-1].iterations) == int(vals["n"]) and
                               int(results[-1].last_count) == int(vals["count"]))}
    if not args.no_cpu:
        import oracle as O
        k = 10
        t0 = time.perf_counter()
        O.life_run(s, cond=O.COND_NEVER, max_iter=k)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(n * n * k / dt / 1e9, 4), "unit": "GLUP/s",
                               "cores": O.threads(), "kind": "oracle",
                               "sample": f"first {k} generations ({dt:.1f} s)"}
        cores = O.threads()
        O.set_threads(1)
        t0 = time.perf_counter()
        O.life_run(s, cond=O.COND_NEVER, max_iter=1)
        dt1 = time.perf_counter() - t0
        O.set_threads(cores)
        out["cpu_baseline_1core"] = {"value": round(n * n / dt1 / 1e9, 4), "unit": "GLUP/s",
                                     "cores": 1, "kind": "oracle", "all_cores": cores,
                                     "sample": f"first generation ({dt1:.1f} s)"}
    ctx.close()
    return out


def run_restore(args, L, I, torch):
    import numpy as np
    n = args.n or 4096
    rin = I.restore_input(n, seed=4, noise=0.4)
    y = torch.from_numpy(rin.y).to("cuda:0")
    ctx = L.Context(0)
    out_runs = {}
    for dtname, dt in (("f64", torch.float64), ("f32", torch.float32)):
        for k in range(args.warmup):
            m, u = ctx.amf_detect(y, 19, dt)
            ctx.run(u, L.LSR_ST_RESTORE, L.LSR_RED_MAX_ABS_DELTA, L.make_cond(L.LSR_COND_BELOW, 0.1, 1),
                    200, L.LSR_BC_BOTTOM, env0=m, param=(100.0, 0.0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m, u = ctx.amf_detect(y, 19, dt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = ctx.run(u, L.LSR_ST_RESTORE, L.LSR_RED_MAX_ABS_DELTA,
                    L.make_cond(L.LSR_COND_BELOW, 0.1, 1), 200, L.LSR_BC_BOTTOM, env0=m,
                    param=(100.0, 0.0))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        flagged = int(m.sum())
        out_runs[dtname] = {"detect_ms": round((t1 - t0) * 1e3, 3),
                            "restore_ms": round((t2 - t1) * 1e3, 3), "iterations": int(r.iterations),
                            "flagged": flagged,
                            "flagged_px_per_s": round(flagged * r.iterations / (t2 - t1), 1),
                            "px_per_s": round(n * n * r.iterations / (t2 - t1), 1),
                            "field": u.cpu().numpy().astype(np.float64),
                            "mask": m.cpu().numpy()}
    err = float(np.max(np.abs(out_runs["f32"]["field"] - out_runs["f64"]["field"])) /
                np.max(np.abs(out_runs["f64"]["field"])))
    oracle_cmp = None
    if not args.no_cpu:
        # the oracle's full two-phase run on the same image: the CPU baseline, and the
        # reference for the detection mask and both restored fields
        import oracle as O
        t0 = time.perf_counter()
        m_o, u_o = O.amf_detect(rin.y, 19)
        t1 = time.perf_counter()
        o, ro = O.restore_run(u_o.astype(np.float64), m_o, thr=0.1, max_iter=200)
        t2 = time.perf_counter()
        den = float(np.max(np.abs(o)))
        oracle_cmp = {
            "mask_bit_exact": bool(np.array_equal(out_runs["f64"]["mask"], m_o) and
                                   np.array_equal(out_runs["f32"]["mask"], m_o)),
            "f64_max_rel_err": float(np.max(np.abs(out_runs["f64"]["field"] - o))) / den,
            "f32_max_rel_err": float(np.max(np.abs(out_runs["f32"]["field"] - o))) / den,
            "iterations_oracle": int(ro.n),
            "iterations_equal": bool(out_runs["f64"]["iterations"] == ro.n ==
                                     out_runs["f32"]["iterations"])}
        cpu = {"value": round(n * n * ro.n / (t2 - t0) / 1e9, 4), "unit": "GLUP/s",
               "cores": O.threads(), "kind": "oracle",
               "sample": f"the whole job: detection {t1 - t0:.2f} s, {ro.n} restoration "
                         f"sweeps {t2 - t1:.2f} s"}
        # the same oracle on one core: detection and the first sweep of the job
        cores = O.threads()
        O.set_threads(1)
        t0 = time.perf_counter()
        O.amf_detect(rin.y, 19)
        t1 = time.perf_counter()
        O.restore_run(u_o.astype(np.float64), m_o, thr=0.1, max_iter=1)
        t2 = time.perf_counter()
        O.set_threads(cores)
        cpu1 = {"value": round(n * n / (t2 - t0) / 1e9, 4), "unit": "GLUP/s", "cores": 1,
                "kind": "oracle", "all_cores": cores,
                "sample": f"detection {t1 - t0:.2f} s and one restoration sweep {t2 - t1:.2f} s"}
    for v in out_runs.values():
        v.pop("field")
        v.pop("mask")
    wall = (out_runs["f64"]["detect_ms"] + out_runs["f64"]["restore_ms"]) / 1e3
    out = base_line("GLUP/s", round(n * n * out_runs["f64"]["iterations"] / wall / 1e9, 3), "GLUP/s",
                    1, args.warmup, round(wall * 1e3, 3), "f64",
                    {"workload": f"two-phase restoration {n}x{n} u8, 40% impulses, w_max 19, "
                                 f"beta 100, stop max|change| < 0.1 or 200", "rows": n, "cols": n})
    out["runs"] = out_runs
    out["f32_vs_f64_max_rel"] = err
    if oracle_cmp:
        out["accuracy"] = oracle_cmp
        out["cpu_baseline"] = cpu
        out["cpu_baseline_1core"] = cpu1
    ctx.close()
    return out


# ---------------------------------------------------------------------------
# ---------------------------------------------------------------------------
# Served mixed stream: jobs are generated on the host at their arrival into
# pinned buffers, submitted with lsr_run_host (the context allocates their device
# copies under its HBM budget, copies them in at admission and the result out at
# retirement), collected in completion order with lsr_wait_any, checked, and
# freed. At most --host-gib of host buffers are outstanding at a time.
# ---------------------------------------------------------------------------
def _job_kw(L, I, spec, h=None):
    if spec.kind == I.KIND_LAPLACE:
        return dict(stencil_id=L.LSR_ST_LAPLACE5, reduce_op=L.LSR_RED_MAX_ABS_DELTA,
                    cond=L.make_cond(L.LSR_COND_BELOW, 1e-6, 1), max_iter=2000, bc=L.LSR_BC_RING)
    if spec.kind == I.KIND_HELMHOLTZ:
        return dict(stencil_id=L.LSR_ST_HELMHOLTZ5, reduce_op=L.LSR_RED_L2_DELTA,
                    cond=L.make_cond(L.LSR_COND_BELOW, 1e-9, 10), max_iter=5000,
                    bc=L.LSR_BC_RING, param=(1.0, h))
    return dict(stencil_id=L.LSR_ST_LIFE, reduce_op=L.LSR_RED_SUM,
                cond=L.make_cond(L.LSR_COND_STABLE_FOR, 0.0, 1, 10), max_iter=2000,
                bc=L.LSR_BC_TORUS)


def _job_bytes(I, spec, f32):
    esz = 1 if spec.kind == I.KIND_LIFE else (4 if f32 else 8)
    return spec.side * spec.side * esz * (2 if spec.kind == I.KIND_HELMHOLTZ else 1)


def _make_host_job(L, I, torch, spec, f32):
    """Pinned host grid (and env) of one job of the stream, filled by the seeded recipe."""
    n = spec.side
    if spec.kind == I.KIND_LIFE:
        grid = torch.empty((n, n), dtype=torch.uint8, pin_memory=True)
        I.life_fill(grid.numpy(), spec.seed)
        return grid, None, _job_kw(L, I, spec)
    dt = torch.float32 if f32 else torch.float64
    grid = torch.empty((n, n), dtype=dt, pin_memory=True)
    if spec.kind == I.KIND_LAPLACE:
        I.laplace_fill(grid.numpy(), spec.seed)
        return grid, None, _job_kw(L, I, spec)
    env = torch.empty((n, n), dtype=dt, pin_memory=True)
    h = I.helmholtz_fill(grid.numpy(), env.numpy())
    return grid, env, _job_kw(L, I, spec, h)


def _digest(a):
    import xxhash
    return xxhash.xxh3_128_hexdigest(memoryview(a).cast("B"))


def _helm_closed_form_err(x, n_side, sweeps):
    """max|x - u^n| / max|u^n| with u^n = c*(1 - mu^n) u* the closed form of the
    manufactured Helmholtz solve (alpha = 1), a block of rows at a time."""
    import numpy as np
    from paper_1609_04567_amd import inputs as I
    hh = 1.0 / (n_side - 1)
    s2 = math.sin(math.pi * hh / 2) ** 2
    one_m_mu = (8.0 * s2 + hh * hh) / (4.0 + hh * hh)
    lam = 8.0 / (hh * hh) * s2
    coef = (2 * math.pi ** 2 + 1.0) / (lam + 1.0) * -math.expm1(sweeps * math.log1p(-one_m_mu))
    sv, _ = I.helmholtz_factor(n_side)
    worst, den = 0.0, coef * float(np.max(sv)) ** 2
    step = max(1, (1 << 16) // n_side)
    for r0 in range(0, n_side, step):
        r1 = min(n_side, r0 + step)
        ref = np.outer(coef * sv[r0:r1], sv)
        worst = max(worst, float(np.max(np.abs(x[r0:r1].astype(np.float64) - ref))))
    return worst / den


class _StreamRun:
    """Feeds a job stream to a context and collects it.

    Generator threads build jobs in index order into pinned buffers while the
    outstanding host bytes stay under a limit; the submitter submits job k as soon
    as it is built (closed loop) or at its scheduled arrival time (open loop); a
    collector takes results in completion order (lsr_wait_any) and hands each job
    to a pool of checker threads, which run `check(k, job, result)` and free it."""

    def __init__(self, L, I, torch, ctx, specs, f32, host_bytes, gen_threads=6, check_threads=6,
                 arrivals=None, check=None, variants=None):
        import concurrent.futures as cf
        self.L, self.I, self.torch, self.ctx = L, I, torch, ctx
        self.specs, self.f32 = specs, f32
        self.variants = variants or [f32]      # one submission per precision in the list
        self.limit = host_bytes
        self.arrivals = arrivals
        self.check = check
        self.cv = threading.Condition()
        self.ready = {}
        self.out_bytes = 0
        self.next_gen = 0
        self.submitted = 0
        self.collected = 0
        self.total = len(specs) * len(self.variants)
        self.lag = []
        self.error = None
        self.gen_threads = gen_threads
        self.pool = cf.ThreadPoolExecutor(max_workers=check_threads)
        self.jobs = {}

    def _gen(self):
        try:
            while True:
                with self.cv:
                    # host bytes are reserved in job order: a later job that fits
                    # must not take the room an earlier one waits for, since jobs
                    # are submitted in order (a job larger than the limit still
                    # runs, alone)
                    def fits():
                        k = self.next_gen
                        if self.error or k >= len(self.specs):
                            return True
                        need = sum(_job_bytes(self.I, self.specs[k], v) for v in self.variants)
                        return self.out_bytes == 0 or self.out_bytes + need <= self.limit
                    self.cv.wait_for(fits)
                    k = self.next_gen
                    if k >= len(self.specs) or self.error:
                        return
                    self.next_gen += 1
                    spec = self.specs[k]
                    self.out_bytes += sum(_job_bytes(self.I, spec, v) for v in self.variants)
                built = [(_make_host_job(self.L, self.I, self.torch, spec, v), v,
                          _job_bytes(self.I, spec, v)) for v in self.variants]
                with self.cv:
                    self.ready[k] = built
                    self.cv.notify_all()
        except BaseException as e:   # surfaced by run()
            with self.cv:
                self.error = e
                self.cv.notify_all()

    def _collect(self):
        L = self.L
        try:
            while self.collected < self.total:
                with self.cv:
                    self.cv.wait_for(lambda: self.error or self.submitted > self.collected)
                    if self.error:
                        return
                jid = self.ctx.wait_any(True)
                r = self.ctx.result(jid)
                with self.cv:
                    k, v, job, need = self.jobs.pop(jid)
                    self.collected += 1
                    done = self.collected
                self.pool.submit(self._finish, k, v, job, r, need)
                if done % 250 == 0:   # progress of long streams
                    print(f"  {done} / {self.total} results", file=sys.stderr, flush=True)
        except BaseException as e:
            with self.cv:
                self.error = e
                self.cv.notify_all()

    def _finish(self, k, v, job, r, need):
        try:
            if self.check:
                self.check(k, v, job, r)
        except BaseException as e:
            with self.cv:
                self.error = e
                self.cv.notify_all()
        finally:
            with self.cv:
                self.out_bytes -= need
                self.cv.notify_all()

    def _stall_guard(self, stall_s=120.0):
        """Ends the process (exit status 3) with a description of the stream's and the
        context's state when no result has arrived for stall_s seconds."""
        last, t_last = -1, time.monotonic()
        while True:
            time.sleep(5.0)
            with self.cv:
                done = self.collected >= self.total or self.error is not None
                c = self.collected
            if done:
                return
            if c != last:
                last, t_last = c, time.monotonic()
                continue
            if time.monotonic() - t_last < stall_s:
                continue
            with self.cv:
                oldest = sorted(self.jobs.items())[:8]
                state = {"submitted": self.submitted, "collected": self.collected,
                         "total": self.total, "out_bytes": self.out_bytes,
                         "next_gen": self.next_gen, "ready": sorted(self.ready)[:8],
                         "in_flight": [(jid, k, v, self.specs[k].kind, self.specs[k].side)
                                       for jid, (k, v, _, _) in oldest]}
            print(f"STALL: no result for {stall_s:.0f} s: {state}", file=sys.stderr, flush=True)
            try:
                print(f"STALL: context {self.ctx.stats()}", file=sys.stderr, flush=True)
            except Exception as e:   # the report must not hide the stall
                print(f"STALL: stats failed: {e}", file=sys.stderr, flush=True)
            os._exit(3)

    def run(self):
        """Runs the stream; returns the wall time from the first submission to the
        last result (checks of the last jobs excluded)."""
        threading.Thread(target=self._stall_guard, daemon=True).start()
        gens = [threading.Thread(target=self._gen, daemon=True) for _ in range(self.gen_threads)]
        for g in gens:
            g.start()
        col = threading.Thread(target=self._collect, daemon=True)
        col.start()
        t0 = None
        for k, spec in enumerate(self.specs):
            with self.cv:
                self.cv.wait_for(lambda: self.error or k in self.ready)
                if self.error:
                    break
                built = self.ready.pop(k)
            if t0 is None:
                t0 = time.perf_counter()
            if self.arrivals is not None:
                d = t0 + self.arrivals[k] - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                self.lag.append(max(0.0, time.perf_counter() - t0 - self.arrivals[k]))
            for (grid, env, kw), v, need in built:
                jid = self.ctx.submit_host(grid, kw["stencil_id"], kw["reduce_op"], kw["cond"],
                                           kw["max_iter"], kw["bc"], env0=env,
                                           param=kw.get("param", ()))
                with self.cv:
                    self.jobs[jid] = (k, v, (grid, env, kw), need)
                    self.submitted += 1
                    self.cv.notify_all()
        col.join()
        wall = time.perf_counter() - (t0 or time.perf_counter())
        self.pool.shutdown(wait=True)
        for g in gens:
            g.join()
        if self.error:
            raise self.error
        return wall


def _pct(v, q):
    import numpy as np
    return round(float(np.percentile(np.asarray(v), q)), 2) if len(v) else None


def run_served(args, L, I, torch):
    """The mixed stream of 20000 jobs (60% Laplace, 25% Helmholtz, 15% Life; side
    log-uniform in [128, 4096]; each job generated on the host at its arrival).

    Legs (--legs, comma separated):
      closed   batched engine, FP32 storage, closed loop (as many jobs in flight as
               --host-gib of host buffers allow): jobs/s, latency percentiles, a
               digest of every result, the closed-form error of every Helmholtz job.
      poisson  the same at Poisson arrivals of lambda x the closed-loop rate for each
               lambda in --lambdas (--rate gives the closed-loop rate when that leg
               is not in this run).
      verify   untimed: every Laplace and Helmholtz job again in FP32 and in FP64 on
               one batched context; each FP32 field's error against its FP64 field
               (FP64 fields are bit-identical to the oracle's, FP32 digests equal the
               closed leg's).
      plain    the plain FP64 path: one job after another on a plain context
               (fused launches where they apply): jobs/s and a digest of every result.
      oracle   the CPU oracle on a seeded sample (every 97th job up to side 1024 and
               every 997th of any side): its time (the CPU baseline), and the FP32 /
               FP64 / Life results of those jobs against it.
    """
    import numpy as np
    count = args.jobs
    specs = I.job_stream(count)
    legs = [x for x in args.legs.split(",") if x]
    gib = int(args.host_gib * (1 << 30))
    recs = {k: {"kind": s.kind, "side": s.side} for k, s in enumerate(specs)}
    prior = False
    if args.prior_records:
        # per-job records of earlier legs of the same stream (another run of this
        # workload): their digests and counts join the cross-checks below
        with open(args.prior_records) as fh:
            for k, v in json.load(fh).items():
                if int(k) in recs:
                    recs[int(k)].update(v)
        prior = True
    keep_fields = {}
    sample = {k for k, s in enumerate(specs)
              if (k % 97 == 0 and s.side <= 1024) or k % 997 == 0}
    out = None
    sat = args.rate or None

    # --autotune: the batched engine's settings for every key of the stream (kind,
    # size class = bit length of the side, check period), measured on a batched
    # context before the legs and loaded into each batched context they use
    tune_json, tune_info = None, None
    if args.autotune:
        t0 = time.perf_counter()
        kinds = [(L.LSR_ST_LAPLACE5, L.LSR_F32, 1), (L.LSR_ST_HELMHOLTZ5, L.LSR_F32, 10),
                 (L.LSR_ST_LIFE, L.LSR_U8, 1)]
        classes = sorted({s.side.bit_length() for s in specs})
        chosen = {}
        with L.Context(0, batched=True) as tctx:
            for b in classes:
                side = min(max(s.side for s in specs), int(round(2 ** (b - 0.5))))
                for st, dt, every in kinds:
                    best = tctx.autotune(st, dt, side, side, every)
                    chosen[f"{st}/{b}"] = (best.tb_depth, best.tile_rows)
            tune_json = L.lsr_tune_export(tctx.handle)
        tune_info = {"keys": len(chosen), "seconds": round(time.perf_counter() - t0, 1),
                     "depth_tile_rows": chosen}
        print(f"autotune: {tune_info}", file=sys.stderr, flush=True)

    def batched_ctx():
        c = L.Context(0, batched=True)
        if tune_json:
            L.lsr_tune_import(c.handle, tune_json)
        return c

    def lup_of(k, n):
        s = specs[k]
        return (s.side - (0 if s.kind == I.KIND_LIFE else 2)) ** 2 * n

    # -- closed loop, batched FP32 --------------------------------------------
    if "closed" in legs:
        bctx = batched_ctx()
        done_lup = [0]

        def check(k, v, job, r):
            grid = job[0].numpy()
            rec = recs[k]
            rec.update(n=int(r.iterations), r32=float(r.last_reduce), count=int(r.last_count),
                       lat_ms=round(r.latency_ms, 3), queue_ms=round(r.queue_ms, 3),
                       status=int(r.status), d32=_digest(grid))
            done_lup[0] += lup_of(k, r.iterations)
            if specs[k].kind == I.KIND_HELMHOLTZ:
                rec["cf_err32"] = _helm_closed_form_err(grid, specs[k].side, r.iterations)
            if k in sample and specs[k].kind != I.KIND_LIFE:
                keep_fields[(k, "f32")] = grid.copy()

        run = _StreamRun(L, I, torch, bctx, specs, True, gib, check=check)
        wall = run.run()
        bctx.close()
        sat = count / wall
        lat = [recs[k]["lat_ms"] for k in recs]
        print(f"closed loop: {count} jobs in {wall:.1f} s = {sat:.2f} jobs/s", file=sys.stderr,
              flush=True)
        out = base_line("jobs/s", round(sat, 3), "jobs/s", 1, 0, round(wall * 1e3, 1), "f32",
                        {"workload": f"served mixed stream, {count} jobs (60% Laplace, 25% "
                                     "Helmholtz, 15% Life; side log-uniform 128..4096), host "
                                     "ingest, FP32 storage with FP64 reduce, batched engine",
                         "jobs": count, "host_window_gib": args.host_gib})
        out["batched_glup_s"] = round(done_lup[0] / wall / 1e9, 2)
        out["latency_closed_loop_ms"] = {"p50": _pct(lat, 50), "p99": _pct(lat, 99)}
        cf = [recs[k]["cf_err32"] for k in recs if "cf_err32" in recs[k]]
        out["helmholtz_closed_form"] = {"jobs": len(cf), "max_rel_err": max(cf) if cf else None,
                                        "within_1e-5": int(sum(e <= 1e-5 for e in cf))}
        bad = [k for k in recs if recs[k].get("status", 0) != L.LSR_OK]
        out["status_not_ok"] = len(bad)
    if out is None:
        out = base_line("jobs/s", None, "jobs/s", 1, 0, None, "f32",
                        {"workload": f"served mixed stream, {count} jobs", "jobs": count})

    # -- Poisson arrivals ------------------------------------------------------
    if "poisson" in legs:
        if not sat:
            raise SystemExit("--legs poisson needs the closed leg or --rate")
        out["poisson"] = []
        for lam in [float(x) for x in args.lambdas.split(",")]:
            rate = lam * sat
            arr = I.poisson_arrivals(specs, rate)
            lat = []
            bctx = batched_ctx()

            def check(k, v, job, r, lat=lat):
                lat.append(r.latency_ms)

            run = _StreamRun(L, I, torch, bctx, specs, True, gib, arrivals=arr, check=check)
            wall = run.run()
            bctx.close()
            lag = np.array(run.lag) * 1e3
            e = {"lambda_x_sat": lam, "rate_jobs_s": round(rate, 3), "wall_s": round(wall, 2),
                 "served_jobs_s": round(count / wall, 3), "p50_ms": _pct(lat, 50),
                 "p99_ms": _pct(lat, 99), "submit_lag_p99_ms": _pct(lag, 99)}
            out["poisson"].append(e)
            print(f"poisson {e}", file=sys.stderr, flush=True)

    # -- verification: FP32 against FP64, every Laplace and Helmholtz job -----------
    if "verify" in legs:
        vspecs = [(k, s) for k, s in enumerate(specs) if s.kind != I.KIND_LIFE]
        bctx = batched_ctx()
        pend = {}
        lock = threading.Lock()

        def check(i, v, job, r):
            k = vspecs[i][0]
            grid = job[0].numpy()
            with lock:
                pend.setdefault(k, {})[v] = (grid, r)
                pair = pend.pop(k) if len(pend[k]) == 2 else None
            if pair is None:
                return
            (x32, r32), (x64, r64) = pair[True], pair[False]
            rec = recs[k]
            den = float(np.max(np.abs(x64)))
            rec["err32"] = float(np.max(np.abs(x32.astype(np.float64) - x64))) / (den or 1.0)
            rec["n64"] = int(r64.iterations)
            rec["n32v"] = int(r32.iterations)
            rec["d32v"] = _digest(x32)
            rec["d64v"] = _digest(x64)
            if k in sample:
                keep_fields[(k, "f32")] = x32.copy()
                keep_fields[(k, "f64")] = x64.copy()

        run = _StreamRun(L, I, torch, bctx, [s for _, s in vspecs], True, gib, check=check,
                         variants=[True, False])
        t0 = time.perf_counter()
        run.run()
        bctx.close()
        errs = [recs[k]["err32"] for k, _ in vspecs]
        same_n = sum(recs[k]["n64"] == recs[k]["n32v"] for k, _ in vspecs)
        v = {"jobs": len(vspecs), "wall_s": round(time.perf_counter() - t0, 1),
             "max_rel_err_f32_vs_f64": max(errs), "p99_rel_err": float(np.percentile(errs, 99)),
             "within_1e-5": int(sum(e <= 1e-5 for e in errs)), "iteration_counts_equal": same_n}
        if "closed" in legs:
            v["f32_digest_equal_to_closed_leg"] = int(sum(recs[k]["d32v"] == recs[k]["d32"]
                                                          for k, _ in vspecs))
            v["iterations_equal_to_closed_leg"] = int(sum(recs[k]["n32v"] == recs[k]["n"]
                                                          for k, _ in vspecs))
        out["verify"] = v
        print(f"verify {v}", file=sys.stderr, flush=True)

    # -- plain FP64 path ------------------------------------------------------
    if "plain" in legs:
        pctx = L.Context(0)
        done = []

        def check(k, v, job, r):
            grid = job[0].numpy()
            recs[k].update(n64p=int(r.iterations), d64p=_digest(grid))
            done.append(k)
            if k in sample and specs[k].kind != I.KIND_LIFE:
                keep_fields[(k, "f64p")] = grid.copy()

        # one job at a time on the device; the host prepares the next ones meanwhile
        run = _StreamRun(L, I, torch, pctx, specs, False, min(gib, 4 << 30), check=check)
        wall = run.run()
        pctx.close()
        pj = count / wall
        out["plain_fp64_jobs_s"] = round(pj, 3)
        if sat:
            out["speedup_vs_plain_fp64"] = round(sat / pj, 3)
        if "closed" in legs or prior:
            out["life_equal_batched_vs_plain"] = int(sum(
                recs[k].get("d32") == recs[k]["d64p"] and recs[k].get("n") == recs[k]["n64p"]
                for k in recs if specs[k].kind == I.KIND_LIFE))
            out["life_jobs"] = int(sum(specs[k].kind == I.KIND_LIFE for k in recs))
        if "verify" in legs or prior:
            out["f64_batched_equal_plain"] = int(sum(
                recs[k].get("d64v") == recs[k]["d64p"] and recs[k].get("n64") == recs[k]["n64p"]
                for k in recs if specs[k].kind != I.KIND_LIFE))
            out["jacobi_jobs"] = int(sum(specs[k].kind != I.KIND_LIFE for k in recs))
        print(f"plain fp64: {pj:.2f} jobs/s", file=sys.stderr, flush=True)

    # -- CPU oracle on the seeded sample (the CPU baseline) --------------------------
    if "oracle" in legs:
        import oracle as O
        res, t_or, lup_or = [], 0.0, 0
        for k in sorted(sample):
            s = specs[k]
            t0 = time.perf_counter()
            if s.kind == I.KIND_LAPLACE:
                a = I.laplace_input(s.side, seed=s.seed)
                o, ro = O.jacobi_run(a, thr=1e-6, max_iter=2000)
            elif s.kind == I.KIND_HELMHOLTZ:
                h = I.helmholtz_input(s.side)
                o, ro = O.jacobi_run(h.u0, helmholtz=True, g=h.g, alpha=h.alpha, h=h.h,
                                     reduce_op=O.RED_L2_DELTA, thr=1e-9, check_every=10,
                                     max_iter=5000)
            else:
                a = I.life_input(s.side, seed=s.seed)
                o, ro = O.life_run(a, stable_window=10, max_iter=2000)
            dt = time.perf_counter() - t0
            t_or += dt
            lup_or += lup_of(k, ro.n)
            e = {"job": k, "kind": s.kind, "side": s.side, "n_oracle": ro.n, "oracle_s": round(dt, 3)}
            rec = recs[k]
            if s.kind == I.KIND_LIFE:
                d = _digest(o)
                if "d32" in rec:
                    e["batched_equal"] = rec["d32"] == d and rec["n"] == ro.n
                if "d64p" in rec:
                    e["plain_equal"] = rec["d64p"] == d and rec["n64p"] == ro.n
            else:
                den = float(np.max(np.abs(o))) or 1.0
                if (k, "f32") in keep_fields:
                    x = keep_fields[(k, "f32")]
                    e["f32_rel_err"] = float(np.max(np.abs(x.astype(np.float64) - o))) / den
                    e["f32_n_equal"] = rec.get("n", rec.get("n32v")) == ro.n
                for tag in ("f64", "f64p"):
                    if (k, tag) in keep_fields:
                        e[f"{tag}_bit_equal"] = bool(np.array_equal(keep_fields[(k, tag)], o))
            res.append(e)
        oracle_glups = lup_or / t_or / 1e9
        # jobs/s of the oracle over the whole stream, extrapolated from its GLUP/s on
        # the sample and the stream's total cell updates (the closed leg's counts)
        total_lup = sum(lup_of(k, recs[k]["n"]) for k in recs if "n" in recs[k])
        out["cpu_baseline"] = {
            "value": round(count / (total_lup / (oracle_glups * 1e9)), 4) if total_lup else None,
            "unit": "jobs/s", "cores": O.threads(), "kind": "oracle",
            "sample": (f"{len(res)} jobs (every 97th up to side 1024, every 997th), "
                       f"{t_or:.1f} s, {oracle_glups:.2f} GLUP/s; jobs/s extrapolated to the "
                       "whole stream's cell updates")}
        out["oracle_sample"] = {
            "jobs": len(res),
            "f32_max_rel_err": max([e["f32_rel_err"] for e in res if "f32_rel_err" in e],
                                   default=None),
            "f32_n_equal": sum(bool(e.get("f32_n_equal")) for e in res),
            "f64_bit_equal": sum(bool(e.get("f64_bit_equal")) for e in res),
            "f64p_bit_equal": sum(bool(e.get("f64p_bit_equal")) for e in res),
            "life_batched_equal": sum(bool(e.get("batched_equal")) for e in res),
            "life_plain_equal": sum(bool(e.get("plain_equal")) for e in res),
            "by_kind": {kd: sum(e["kind"] == kd for e in res) for kd in
                        (I.KIND_LAPLACE, I.KIND_HELMHOLTZ, I.KIND_LIFE)}}
    if tune_info:
        out["autotune"] = tune_info
    if args.records:
        with open(args.records, "w") as fh:
            json.dump({str(k): v for k, v in recs.items()}, fh)
    return out


# ---------------------------------------------------------------------------
def run_video(args, L, I, torch):
    """Restoration of noisy video streams (the 100-frame streams of Sect. 4.3's
    table: VGA 640x480, 720p 1280x720 and 2048x1080 at 30% and 70% impulses;
    synthetic frames of moving blobs). Each frame is one two-phase job on a batched
    context (lsr_run_restore_host: H2D of the frame, detection, restoration sweeps
    in the engine's rounds beside the other frames, D2H of the result), stopping on
    the mean absolute change below 1e-3 (the paper's criterion) or 200 sweeps.
    Frames are generated on the host ahead of time and submitted as fast as the
    engine admits them; results come back in completion order and are taken in
    frame order, as the ordered farm of the paper's pipeline delivers them."""
    import numpy as np
    nframes = args.frames
    streams = [(480, 640, "VGA"), (720, 1280, "720p"), (1080, 2048, "2048x1080")]
    dt = torch.float32 if args.video_dtype == "f32" else torch.float64
    cond = L.make_cond(L.LSR_COND_BELOW, 1e-3, 1)
    runs = []
    sample = sorted({0, nframes // 2, nframes - 1})
    keep = {}
    for rows, cols, name in streams:
        for noise in (0.3, 0.7):
            frames = [torch.from_numpy(I.video_frame(rows, cols, f, noise=noise).y).pin_memory()
                      for f in range(nframes)]
            outs = [torch.empty((rows, cols), dtype=dt).pin_memory() for _ in range(nframes)]
            bctx = L.Context(0, batched=True)
            # warm-up frame (first use of the kernels and the pool)
            bctx.result(bctx.submit_restore_host(frames[0], outs[0],
                                                 reduce_op=L.LSR_RED_MEAN_ABS_DELTA, cond=cond))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ids = [bctx.submit_restore_host(frames[f], outs[f], reduce_op=L.LSR_RED_MEAN_ABS_DELTA,
                                            cond=cond) for f in range(nframes)]
            res = [bctx.result(i) for i in ids]   # in frame order
            wall = time.perf_counter() - t0
            bctx.close()
            its = [int(r.iterations) for r in res]
            assert all(r.status == L.LSR_OK for r in res)
            runs.append({"video": f"{name}, {int(noise * 100)}%", "frames": nframes,
                         "wall_s": round(wall, 4), "fps": round(nframes / wall, 1),
                         "mpx_per_s": round(nframes * rows * cols / wall / 1e6, 1),
                         "iterations_min_max": [min(its), max(its)],
                         "latency_p50_ms": _pct([r.latency_ms for r in res], 50)})
            print(f"video {runs[-1]}", file=sys.stderr, flush=True)
            for f in sample:
                keep[(name, noise, f)] = (frames[f].numpy().copy(), outs[f].numpy().copy(),
                                          its[f])
    out = base_line("frames/s", round(min(r["fps"] for r in runs), 1), "frames/s", 1, 1, None,
                    args.video_dtype,
                    {"workload": f"two-phase restoration of {nframes}-frame video streams (VGA, "
                                 "720p, 2048x1080 at 30% and 70% impulses), mean |change| < 1e-3 "
                                 "or 200 sweeps, batched engine, host frames", "frames": nframes})
    out["streams"] = runs
    if not args.no_cpu:
        # per-frame parity with the oracle on frames sampled from each stream, and the
        # oracle's own time on them (the CPU baseline)
        import oracle as O
        worst, n_eq, masks_eq, t_or, px = 0.0, 0, 0, 0.0, 0
        for (name, noise, f), (y, u, n_gpu) in keep.items():
            t0 = time.perf_counter()
            m_o, u_o = O.amf_detect(y, 19)
            o, ro = O.restore_run(u_o.astype(np.float64), m_o, reduce_op=O.RED_MEAN_ABS_DELTA,
                                  thr=1e-3, max_iter=200)
            t_or += time.perf_counter() - t0
            px += y.size
            worst = max(worst, float(np.max(np.abs(u.astype(np.float64) - o)) / np.max(np.abs(o))))
            n_eq += int(n_gpu == ro.n)
        out["accuracy"] = {"frames_checked": len(keep), "max_rel_err_vs_oracle": worst,
                           "iterations_equal": n_eq,
                           "tolerance": 1e-5 if args.video_dtype == "f32" else 1e-12}
        out["cpu_baseline"] = {"value": round(len(keep) / t_or, 3), "unit": "frames/s",
                               "cores": O.threads(), "kind": "oracle",
                               "sample": f"{len(keep)} frames sampled from the six streams "
                                         f"({px / 1e6:.1f} Mpx, {t_or:.1f} s)"}
    return out


# ---------------------------------------------------------------------------
def run_sobel(args, L, I, torch):
    """The streaming Sobel edge detector (Sect. 4.2's table): square images of side
    512, 4096 and 16384 (synthetic: moving-blob frames without noise, plus a
    checkerboard of sharp edges), first one at a time through a plain context (host
    image in, host edges out: H2D, one sweep, D2H), then a stream of 100 images,
    each drawn from the three by a seeded draw, through the batched engine, whose
    copy stream overlaps the H2D and D2H copies of one image with the sweeps of
    others. The single-iteration pattern is bound by the copies: the line reports
    images/s of the stream and the PCIe bytes it moved per second."""
    import numpy as np
    sides = [512, 4096, 16384][: args.sobel_sizes]
    cond = L.make_cond(L.LSR_COND_NEVER, 0.0, 1, 1)
    src = {}
    for n in sides:
        img = I.video_frame(n, n, 0, seed=12, noise=0.0).clean
        img[(np.arange(n)[:, None] // 64 + np.arange(n)[None, :] // 64) % 2 == 1] //= 4
        src[n] = torch.from_numpy(img).pin_memory()
    single = {}
    with L.Context(0) as c:
        for n in sides:
            g = src[n].clone().pin_memory()
            c.result(c.submit_host(g, L.LSR_ST_SOBEL, L.LSR_RED_SUM, cond, 1, L.LSR_BC_BOTTOM))
            best = 1e9
            for _ in range(3):
                g.copy_(src[n])
                t0 = time.perf_counter()
                r = c.result(c.submit_host(g, L.LSR_ST_SOBEL, L.LSR_RED_SUM, cond, 1,
                                           L.LSR_BC_BOTTOM))
                best = min(best, time.perf_counter() - t0)
            single[n] = {"ms": round(best * 1e3, 3), "kernel_ms": round(r.device_ms, 3)}
    # the stream: 100 images drawn from the three, each in its own pinned buffer
    draws = I.uniform01(13, 0, args.frames)
    order = [sides[min(int(u * len(sides)), len(sides) - 1)] for u in draws]
    bufs = [src[n].clone().pin_memory() for n in order]
    nbytes = sum(n * n for n in order)
    with L.Context(0, batched=True) as b:
        warm = src[sides[0]].clone().pin_memory()
        b.result(b.submit_host(warm, L.LSR_ST_SOBEL, L.LSR_RED_SUM, cond, 1, L.LSR_BC_BOTTOM))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ids = [b.submit_host(g, L.LSR_ST_SOBEL, L.LSR_RED_SUM, cond, 1, L.LSR_BC_BOTTOM)
               for g in bufs]
        res = [b.result(i) for i in ids]
        wall = time.perf_counter() - t0
    assert all(r.status == L.LSR_OK for r in res)
    out = base_line("images/s", round(len(order) / wall, 2), "images/s", 1, 1,
                    round(wall * 1e3, 2), "u8",
                    {"workload": f"streaming Sobel: {len(order)} images drawn from sides "
                                 f"{sides} (host in, host out), batched engine",
                     "images": len(order), "sides": sides})
    out["stream_pcie_gbs"] = round(2 * nbytes / wall / 1e9, 2)
    out["single_image"] = {str(n): v for n, v in single.items()}
    if not args.no_cpu:
        import oracle as O
        ok, t_or = 0, 0.0
        ref = {}
        for n in sides:
            t1 = time.perf_counter()
            o, ro = O.sobel_run(src[n].numpy(), max_iter=1)
            t_or += time.perf_counter() - t1
            ref[n] = (_digest(o), int(ro.count))
        for n, g, r in zip(order, bufs, res):
            ok += int(_digest(g.numpy()) == ref[n][0] and int(r.last_count) == ref[n][1])
        out["accuracy"] = {"images_bit_identical_to_oracle": ok, "images": len(order)}
        out["cpu_baseline"] = {"value": round(len(sides) / t_or, 3), "unit": "images/s",
                               "cores": O.threads(), "kind": "oracle",
                               "sample": f"one image of each side ({t_or:.1f} s)"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="helmholtz",
                    choices=["helmholtz", "laplace", "life", "restore", "served", "video",
                             "sobel"])
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--sweeps", type=int, default=0)
    ap.add_argument("--jobs", type=int, default=20000)
    ap.add_argument("--legs", default="closed,poisson,verify,plain,oracle",
                    help="served workload: which legs to run (see run_served)")
    ap.add_argument("--lambdas", default="0.5,0.8,1.0,1.2")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="closed-loop jobs/s for the poisson leg when closed is not run")
    ap.add_argument("--host-gib", type=float, default=12.0,
                    help="host buffers outstanding at a time in the served legs")
    ap.add_argument("--records", default="", help="served: write per-job records (JSON) here")
    ap.add_argument("--prior-records", default="",
                    help="served: per-job records of an earlier run of other legs, for cross-checks")
    ap.add_argument("--frames", type=int, default=100, help="video: frames per stream")
    ap.add_argument("--video-dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--sobel-sizes", type=int, default=3, help="sobel: how many of 512, 4096, 16384")
    ap.add_argument("--cpu-sweeps", type=int, default=1500)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the one-sweep-per-launch measurement beside a fused run")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--unroll", type=int, default=0)
    ap.add_argument("--tb", type=int, default=0, help="Jacobi sweeps fused per launch (0 = auto)")
    ap.add_argument("--form", default="array", choices=["array", "sep"],
                    help="helmholtz: right-hand side read from an array, or the -i form (from the "
                         "indices and two factor vectors)")
    ap.add_argument("--autotune", action="store_true",
                    help="measure launch settings for the job before timing it (helmholtz)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this build runs on one GPU "
              "(the multi-GPU row split is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1609_04567_amd as L
    from paper_1609_04567_amd import inputs as I

    fn = {"helmholtz": run_helmholtz, "laplace": run_laplace, "life": run_life,
          "restore": run_restore, "served": run_served, "video": run_video,
          "sobel": run_sobel}[args.workload]
    print(json.dumps(fn(args, L, I, torch)), flush=True)


if __name__ == "__main__":
    main()
