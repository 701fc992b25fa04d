"""GPU parity: two-phase restoration (detection bit-exact, restoration to 1e-12 in
FP64 and 1e-5 in FP32 against the FP64 oracle).

At 4096^2 the oracle checks sampled windows: detection is local (a window of at
most w_max), and k restoration sweeps only reach k pixels, so an oracle run on a
crop with a margin of k (bottom boundary at the crop edge) is exact in its centre.
"""
import numpy as np
import pytest

import oracle as O
import paper_1609_04567_amd as L
from paper_1609_04567_amd import inputs as I
from gpu_helpers import rel_err, run_restore, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,noise,wmax", [((8, 8), 0.4, 19), ((13, 11), 0.7, 7),
                                              ((256, 256), 0.4, 19), ((300, 517), 0.7, 19),
                                              ((64, 64), 0.9, 3), ((40, 50), 0.4, 31)])
def test_amf_detect_bit_exact(ctx, shape, noise, wmax):
    import torch
    say(f"amf {shape} noise={noise} wmax={wmax}")
    r = I.restore_input(*shape, seed=4, noise=noise)
    m_o, u_o = O.amf_detect(r.y, wmax)
    y = torch.from_numpy(r.y).to("cuda:0")
    for dt in (torch.uint8, torch.float32, torch.float64):
        m, u = ctx.amf_detect(y, wmax, dt)
        torch.cuda.synchronize()
        assert np.array_equal(m.cpu().numpy(), m_o)
        assert np.array_equal(u.cpu().numpy().astype(np.float64), u_o.astype(np.float64))


@pytest.mark.parametrize("shape,noise,wmax,frame", [((480, 640), 0.7, 19, 3), ((480, 640), 0.3, 19, 50),
                                                    ((130, 97), 0.7, 5, 7), ((61, 200), 0.9, 9, 1)])
def test_amf_detect_bit_exact_on_video_frames(ctx, shape, noise, wmax, frame):
    """Video frames (smooth integer plateaus, where windows often grow past 5x5):
    the comparator-network windows, the radix windows and their hand-over."""
    import torch
    say(f"amf video frame {shape} noise={noise} wmax={wmax}")
    r = I.video_frame(*shape, frame, noise=noise)
    m_o, u_o = O.amf_detect(r.y, wmax)
    y = torch.from_numpy(r.y).to("cuda:0")
    m, u = ctx.amf_detect(y, wmax, torch.uint8)
    torch.cuda.synchronize()
    assert np.array_equal(m.cpu().numpy(), m_o)
    assert np.array_equal(u.cpu().numpy(), u_o)


@pytest.mark.parametrize("shape", [(8, 8), (64, 64), (128, 200), (257, 255)])
@pytest.mark.parametrize("red", [L.LSR_RED_MAX_ABS_DELTA, L.LSR_RED_MEAN_ABS_DELTA])
def test_restore_f64_matches_oracle(ctx, shape, red):
    say(f"restore f64 {shape} red={red}")
    r = I.restore_input(*shape, seed=4, noise=0.4)
    m, u0 = O.amf_detect(r.y, 19)
    ored = O.RED_MAX_ABS_DELTA if red == L.LSR_RED_MAX_ABS_DELTA else O.RED_MEAN_ABS_DELTA
    thr = 0.1 if red == L.LSR_RED_MAX_ABS_DELTA else 1e-3
    o, ro = O.restore_run(u0.astype(np.float64), m, reduce_op=ored, thr=thr, max_iter=200)
    x, res = run_restore(ctx, u0, m, reduce_op=red, thr=thr, max_iter=200)
    assert res.status == L.LSR_OK
    assert res.iterations == ro.n and bool(res.converged) == ro.converged
    assert rel_err(x, o) <= 1e-12
    assert abs(res.last_reduce - ro.r) <= 1e-9 * max(ro.r, 1e-12)


def test_restore_f32_within_1e5(ctx):
    say("restore f32 256^2")
    r = I.restore_input(256, seed=4, noise=0.4)
    m, u0 = O.amf_detect(r.y, 19)
    o, ro = O.restore_run(u0.astype(np.float64), m, thr=0.1, max_iter=200)
    x, res = run_restore(ctx, u0, m, f32=True, thr=0.1, max_iter=200)
    err = rel_err(x, o)
    say(f"  f32 restore rel err {err:.3e}, n {res.iterations} vs {ro.n}")
    assert err <= 1e-5
    assert res.iterations == ro.n


def test_restore_fixed_points_and_quadratic(ctx):
    say("restore fixed points")
    i = np.arange(20, dtype=np.float64)[:, None]
    j = np.arange(24, dtype=np.float64)[None, :]
    u = 30.0 + 3.0 * i + 2.0 * j
    m = np.zeros(u.shape, dtype=np.uint8)
    m[1:-1, 1:-1] = 1
    x, res = run_restore(ctx, u, m, thr=0.1)
    assert res.iterations == 1 and res.converged and np.max(np.abs(x - u)) < 1e-12
    rr = I.restore_input(32, seed=7)
    m2, u2 = O.amf_detect(rr.y, 19)
    o, ro = O.restore_run(u2.astype(np.float64), m2, quadratic=True, cond=O.COND_NEVER, max_iter=5)
    x2, r2 = run_restore(ctx, u2, m2, quadratic=True, cond=L.LSR_COND_NEVER, max_iter=5)
    assert r2.iterations == 5 and rel_err(x2, o) <= 1e-12


def test_full_4096_pipeline_sampled_windows(ctx):
    import torch
    say("restoration 4096^2: detect + restore, sampled windows")
    n = 4096
    rin = I.restore_input(n, seed=4, noise=0.4)
    y = torch.from_numpy(rin.y).to("cuda:0")
    mask, u = ctx.amf_detect(y, 19, torch.float64)
    res = ctx.run(u, L.LSR_ST_RESTORE, L.LSR_RED_MAX_ABS_DELTA,
                  L.make_cond(L.LSR_COND_BELOW, 0.1, 1), 200, L.LSR_BC_BOTTOM, env0=mask,
                  param=(100.0, 0.0))
    torch.cuda.synchronize()
    k = int(res.iterations)
    say(f"  stopped at n={k} r={res.last_reduce:.4f}")
    assert res.status == L.LSR_OK and res.converged and 3 <= k <= 200
    mk = mask.cpu().numpy()
    x = u.cpu().numpy()
    assert np.all(mk[rin.impulse] == 1)
    w, K = 40, 9
    for (r0, c0) in [(0, 0), (2000, 3000), (n - w, n - w), (1234, 0), (4000, 2100)]:
        # detection: crop with margin w_max/2 (clipped at the image edge, where the
        # crop edge is the true edge)
        a0, b0 = max(0, r0 - K), max(0, c0 - K)
        a1, b1 = min(n, r0 + w + K), min(n, c0 + w + K)
        m_o, u_o = O.amf_detect(rin.y[a0:a1, b0:b1], 19)
        assert np.array_equal(mk[r0:r0 + w, c0:c0 + w], m_o[r0 - a0:r0 - a0 + w, c0 - b0:c0 - b0 + w])
        # restoration: k sweeps from the detected start on a crop with margin k
        A0, B0 = max(0, r0 - k - 1), max(0, c0 - k - 1)
        A1, B1 = min(n, r0 + w + k + 1), min(n, c0 + w + k + 1)
        m_crop, u_crop = _detect_crop(rin.y, A0, A1, B0, B1, K)
        o, _ = O.restore_run(u_crop.astype(np.float64), m_crop, cond=O.COND_NEVER, max_iter=k)
        assert rel_err(x[r0:r0 + w, c0:c0 + w],
                       o[r0 - A0:r0 - A0 + w, c0 - B0:c0 - B0 + w]) <= 1e-12, (r0, c0)


def _detect_crop(y, A0, A1, B0, B1, K):
    """Detection on [A0:A1, B0:B1] exactly as on the full image (computed on a crop
    widened by K and cut back)."""
    n0, n1 = y.shape
    a0, b0 = max(0, A0 - K), max(0, B0 - K)
    a1, b1 = min(n0, A1 + K), min(n1, B1 + K)
    m, u = O.amf_detect(y[a0:a1, b0:b1], 19)
    return (np.ascontiguousarray(m[A0 - a0:A1 - a0, B0 - b0:B1 - b0]),
            np.ascontiguousarray(u[A0 - a0:A1 - a0, B0 - b0:B1 - b0]))


@pytest.mark.parametrize("pattern", ["all", "none", "checker", "rows"])
@pytest.mark.parametrize("shape", [(33, 70), (100, 129), (16, 64)])
def test_restore_mask_extremes_match_oracle(ctx, pattern, shape):
    """Every pixel flagged (a wavefront's list full), none flagged, and patterns
    whose flagged pixels fall unevenly over the wavefronts of a tile, on shapes
    with partial bands and partial column strips."""
    say(f"restore mask {pattern} {shape}")
    r = I.restore_input(*shape, seed=5, noise=0.4)
    _, u0 = O.amf_detect(r.y, 19)
    ii, jj = np.indices(shape)
    m = {"all": np.ones(shape), "none": np.zeros(shape), "checker": (ii + jj) % 2,
         "rows": (ii % 5 == 1) | (jj % 7 == 3)}[pattern].astype(np.uint8)
    o, ro = O.restore_run(u0.astype(np.float64), m, thr=0.1, max_iter=50)
    x, res = run_restore(ctx, u0, m, thr=0.1, max_iter=50)
    assert res.status == L.LSR_OK
    assert res.iterations == ro.n and bool(res.converged) == ro.converged
    assert rel_err(x, o) <= 1e-12


def test_detection_matches_hand_derived_golden(ctx):
    """The GPU detection on the hand-derived cases of tests/golden/amf_hand.txt."""
    import torch
    from test_oracle_restore import _amf_hand_cases
    say("detection hand golden")
    for name, c in _amf_hand_cases().items():
        y = torch.from_numpy(c["y"]).to("cuda:0")
        m, u = ctx.amf_detect(y, c["w"], torch.uint8)
        torch.cuda.synchronize()
        assert np.array_equal(m.cpu().numpy(), c["mask"]), name
        assert np.array_equal(u.cpu().numpy(), c["init"]), name
