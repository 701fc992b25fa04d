"""Seeded synthetic inputs for the loop-of-stencil-reduce workloads.

This module is shared by the tests, the benchmark and the CPU oracle's callers.
It holds no arithmetic of the method itself (no sweep, no reduce, no stopping
test): it only draws random numbers and lays out grids. Both the HIP path and the
oracle read the exact bytes produced here.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based generator:
draw i of the stream with seed s is ``mix(s + (i + 1) * GAMMA)``, so any slice of
a stream can be produced independently. A 64-bit draw becomes a double in [0, 1)
as ``(x >> 11) * 2**-53``.

The paper's own inputs (the Helmholtz matrices of Sect. 4.1, the images and
videos of Sect. 4.2 and 4.3) are not available; these recipes are stand-ins of
the same shape and structure:

* ``laplace_input``: square FP64 grid, fixed boundary ring drawn U[0,1), interior 0.
* ``helmholtz_input``: manufactured solution u* = sin(pi x) sin(pi y) on the unit
  square, right-hand side f = (2 pi^2 + alpha) u*, boundary u* = 0, interior 0;
  the env passed to the sweep is g = h^2 f.
* ``life_input``: random soup, a cell is alive iff its draw is below the density.
* ``restore_input``: smooth 8-bit image (sum of Gaussian blobs) plus salt-and-pepper
  impulses at a given rate.
* ``job_stream``: a mixed stream of Laplace / Helmholtz / Life jobs with
  log-uniform sides, for the served form.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Draws start .. start+count-1 of the SplitMix64 stream with this seed (uint64)."""
    out = np.empty(count, dtype=np.uint64)
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        for lo in range(0, count, _CHUNK):
            hi = min(count, lo + _CHUNK)
            idx = np.arange(start + lo + 1, start + hi + 1, dtype=np.uint64)
            out[lo:hi] = _mix(s + idx * GAMMA)
    return out


def uniform01(seed: int, start: int, count: int) -> np.ndarray:
    """Doubles in [0, 1): (draw >> 11) * 2**-53."""
    out = np.empty(count, dtype=np.float64)
    for lo in range(0, count, _CHUNK):
        hi = min(count, lo + _CHUNK)
        x = splitmix64(seed, start + lo, hi - lo)
        out[lo:hi] = (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return out


# ---------------------------------------------------------------------------
# Jacobi / Laplace: fixed boundary ring U[0,1), interior 0.
# ---------------------------------------------------------------------------
def uniform01_at(seed: int, index: np.ndarray) -> np.ndarray:
    """Doubles in [0, 1) for arbitrary draw indices of the stream (counter-based)."""
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        x = _mix(s + (index.astype(np.uint64) + np.uint64(1)) * GAMMA)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _ring_index(rows: int, cols: int):
    """Raster indices of the ring cells and their (row, col) positions."""
    top = np.arange(cols, dtype=np.int64)
    bot = (rows - 1) * cols + top
    mid = np.arange(1, rows - 1, dtype=np.int64) * cols
    idx = np.concatenate([top, bot, mid, mid + (cols - 1)])
    return idx, idx // cols, idx % cols


def laplace_fill(out: np.ndarray, seed: int = 1) -> np.ndarray:
    """Writes the Laplace recipe into a 2-D array of any float dtype (values are
    computed in FP64, then stored): ring cell (i, j) takes draw i*cols + j of the
    stream, every other cell 0."""
    rows, cols = out.shape
    out[...] = 0
    idx, r, c = _ring_index(rows, cols)
    out[r, c] = uniform01_at(seed, idx)
    return out


def laplace_input(rows: int, cols: int | None = None, seed: int = 1) -> np.ndarray:
    """FP64 grid; ring cells take draw (i*cols + j) of the stream, interior cells are 0.

    The side includes the ring, so only (rows-2) x (cols-2) cells are updated.
    """
    cols = rows if cols is None else cols
    return laplace_fill(np.empty((rows, cols), dtype=np.float64), seed)


def harmonic_input(rows: int, cols: int, kind: str) -> np.ndarray:
    """Integer-valued discrete harmonic polynomials on the index lattice (FP64)."""
    i = np.arange(rows, dtype=np.float64)[:, None]
    j = np.arange(cols, dtype=np.float64)[None, :]
    if kind == "x2-y2":
        return np.ascontiguousarray(i * i - j * j)
    if kind == "xy":
        return np.ascontiguousarray(i * j + 0.0 * j)
    if kind == "x3-3xy2":
        return np.ascontiguousarray(i * i * i - 3.0 * i * j * j)
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# Helmholtz: manufactured solution on the unit square.
# ---------------------------------------------------------------------------
@dataclass
class HelmholtzInput:
    u0: np.ndarray      # initial iterate: ring = u* (= 0), interior 0
    g: np.ndarray       # env: h^2 * f
    ustar: np.ndarray   # sin(pi x) sin(pi y) on the lattice (ring exactly 0)
    s: np.ndarray       # the 1-D factor sin(pi x_i)
    alpha: float
    h: float


def helmholtz_factor(n: int):
    """The 1-D factor s_i = sin(pi x_i), x_i = i/(N-1), with exact zeros at both ends, and h."""
    h = 1.0 / (n - 1)
    x = np.arange(n, dtype=np.float64) * h
    s = np.sin(np.pi * x)
    s[0] = 0.0
    s[-1] = 0.0
    return s, h


def helmholtz_input(n: int, alpha: float = 1.0) -> HelmholtzInput:
    """N x N lattice including the ring, x_i = i/(N-1), h = 1/(N-1)."""
    s, h = helmholtz_factor(n)
    ustar = np.ascontiguousarray(np.outer(s, s))
    f = (2.0 * np.pi * np.pi + alpha) * ustar
    g = np.ascontiguousarray((h * h) * f)
    u0 = np.zeros((n, n), dtype=np.float64)
    return HelmholtzInput(u0=u0, g=g, ustar=ustar, s=s, alpha=float(alpha), h=float(h))


def helmholtz_fill(u0: np.ndarray, g: np.ndarray, alpha: float = 1.0) -> float:
    """Writes the Helmholtz recipe into two N x N arrays of any float dtype: u0 = 0
    and g = h^2 f, evaluated per element in FP64 exactly as helmholtz_input does
    (a block of rows at a time), then stored. Returns h."""
    n = u0.shape[0]
    s, h = helmholtz_factor(n)
    u0[...] = 0
    c = 2.0 * np.pi * np.pi + alpha
    hh = h * h
    step = max(1, (1 << 16) // n)
    for r0 in range(0, n, step):
        r1 = min(n, r0 + step)
        blk = np.outer(s[r0:r1], s)
        np.multiply(c, blk, out=blk)
        np.multiply(hh, blk, out=blk)
        g[r0:r1] = blk
    return h


# ---------------------------------------------------------------------------
# Game of Life soup.
# ---------------------------------------------------------------------------
def _mixed_blocks(seed: int, start: int, count: int, blk: int = 1 << 16):
    """Yields (offset, uint64 view) covering draws start .. start+count-1 of the stream,
    a block at a time (the view is reused between blocks)."""
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    z = np.empty(blk, dtype=np.uint64)
    t = np.empty(blk, dtype=np.uint64)
    with np.errstate(over="ignore"):
        for lo in range(0, count, blk):
            m = min(blk, count - lo)
            zz, tt = z[:m], t[:m]
            zz[...] = np.arange(start + lo + 1, start + lo + m + 1, dtype=np.uint64)
            np.multiply(zz, GAMMA, out=zz)
            np.add(zz, s, out=zz)
            for sh, mul in ((30, _M1), (27, _M2)):
                np.right_shift(zz, np.uint64(sh), out=tt)
                np.bitwise_xor(zz, tt, out=zz)
                np.multiply(zz, mul, out=zz)
            np.right_shift(zz, np.uint64(31), out=tt)
            np.bitwise_xor(zz, tt, out=zz)
            yield lo, zz


def _below_limit(p: float) -> np.uint64:
    """The draw x satisfies (x >> 11) * 2**-53 < p iff x < this limit (0 < p < 1): the
    scaling by a power of two is exact, so the test is (x >> 11) < ceil(p * 2**53)."""
    return np.uint64(math.ceil(p * 2.0 ** 53) << 11)


def life_fill(out: np.ndarray, seed: int = 3, density: float = 0.3) -> np.ndarray:
    """Writes the Life soup into a 2-D uint8 array: cell (i, j) is 1 iff draw
    i*cols + j, as a double in [0, 1), is below the density (tested on the integer
    draw, see _below_limit)."""
    rows, cols = out.shape
    if not out.flags.c_contiguous or out.dtype != np.uint8:
        raise ValueError("life_fill writes a C-contiguous uint8 array")
    flat = out.reshape(-1)
    if density >= 1.0 or density <= 0.0:
        flat[...] = 1 if density >= 1.0 else 0
        return out
    lim = _below_limit(density)
    for lo, zz in _mixed_blocks(seed, 0, rows * cols):
        np.less(zz, lim, out=flat[lo:lo + len(zz)].view(np.bool_))
    return out


def life_input(rows: int, cols: int | None = None, seed: int = 3, density: float = 0.3) -> np.ndarray:
    """uint8 grid, cell (i, j) alive (1) iff draw i*cols + j is below the density."""
    cols = rows if cols is None else cols
    return life_fill(np.empty((rows, cols), dtype=np.uint8), seed, density)


def life_pattern(rows: int, cols: int, cells) -> np.ndarray:
    g = np.zeros((rows, cols), dtype=np.uint8)
    for (i, j) in cells:
        g[i % rows, j % cols] = 1
    return g


# ---------------------------------------------------------------------------
# Impulse-noise restoration input.
# ---------------------------------------------------------------------------
@dataclass
class RestoreInput:
    y: np.ndarray        # noisy uint8 image
    clean: np.ndarray    # uint8 image before noise, values in [16, 239]
    impulse: np.ndarray  # bool, where noise was injected


def restore_input(rows: int, cols: int | None = None, seed: int = 4, noise: float = 0.4,
                  blobs: int = 8) -> RestoreInput:
    """Sum of Gaussian blobs mapped to [16, 239], then salt (255) / pepper (0) impulses.

    Draw layout: blob b uses draws 4b..4b+3 (amplitude in [-1,1), centre row,
    centre column, width in [W/16, W/4) with W = max(rows, cols)); pixel p (raster
    order) uses draws 4*blobs + 2p (impulse iff < noise) and 4*blobs + 2p + 1
    (salt iff < 0.5, else pepper).
    """
    cols = rows if cols is None else cols
    w = float(max(rows, cols))
    d = uniform01(seed, 0, 4 * blobs)
    r = np.arange(rows, dtype=np.float64)[:, None]
    c = np.arange(cols, dtype=np.float64)[None, :]
    field = np.zeros((rows, cols), dtype=np.float64)
    for b in range(blobs):
        amp = 2.0 * d[4 * b] - 1.0
        cr = d[4 * b + 1] * rows
        cc = d[4 * b + 2] * cols
        sig = w / 16.0 + d[4 * b + 3] * (w / 4.0 - w / 16.0)
        field += amp * np.exp(-((r - cr) ** 2 + (c - cc) ** 2) / (2.0 * sig * sig))
    lo, hi = field.min(), field.max()
    scale = 223.0 / (hi - lo) if hi > lo else 0.0
    clean = np.rint(16.0 + (field - lo) * scale).astype(np.uint8)
    npx = rows * cols
    y = clean.reshape(-1).copy()
    imp = np.zeros(npx, dtype=bool)
    base = 4 * blobs
    for lo_p in range(0, npx, _CHUNK):
        hi_p = min(npx, lo_p + _CHUNK)
        u = uniform01(seed, base + 2 * lo_p, 2 * (hi_p - lo_p)).reshape(-1, 2)
        hit = u[:, 0] < noise
        salt = u[:, 1] < 0.5
        seg = y[lo_p:hi_p]
        seg[hit & salt] = 255
        seg[hit & ~salt] = 0
        imp[lo_p:hi_p] = hit
    return RestoreInput(y=y.reshape(rows, cols), clean=clean, impulse=imp.reshape(rows, cols))


# ---------------------------------------------------------------------------
# Mixed job stream for the served form.
# ---------------------------------------------------------------------------
KIND_LAPLACE, KIND_HELMHOLTZ, KIND_LIFE = "laplace", "helmholtz", "life"


@dataclass
class JobSpec:
    index: int
    kind: str
    side: int
    seed: int          # seed of the job's own grid-content stream
    arrival_u: float   # U[0,1) draw turned into an inter-arrival gap by the caller


def job_stream(count: int, base_seed: int = 5, side_lo: int = 128, side_hi: int = 4096,
               p_laplace: float = 0.6, p_helm: float = 0.25) -> list[JobSpec]:
    """Job j draws from its own stream seeded with draw j of the base stream.

    Draw 0 picks the kind (Laplace if < p_laplace, Helmholtz if < p_laplace+p_helm,
    else Life), draw 1 the side round(exp(U(ln lo, ln hi))), draw 2 (raw) the
    grid-content seed, draw 3 the arrival-gap uniform.
    """
    seeds = splitmix64(base_seed, 0, count)
    jobs = []
    llo, lhi = math.log(side_lo), math.log(side_hi)
    for j in range(count):
        sj = int(seeds[j])
        u = uniform01(sj, 0, 2)
        raw = splitmix64(sj, 2, 2)
        if u[0] < p_laplace:
            kind = KIND_LAPLACE
        elif u[0] < p_laplace + p_helm:
            kind = KIND_HELMHOLTZ
        else:
            kind = KIND_LIFE
        side = int(round(math.exp(llo + u[1] * (lhi - llo))))
        side = min(max(side, side_lo), side_hi)
        arr = float((raw[1] >> np.uint64(11)).astype(np.float64) * (2.0 ** -53))
        jobs.append(JobSpec(index=j, kind=kind, side=side, seed=int(raw[0]), arrival_u=arr))
    return jobs


def poisson_arrivals(jobs: list[JobSpec], rate: float) -> np.ndarray:
    """Arrival times (s) from the jobs' own uniforms: gap = -ln(1 - U) / rate."""
    gaps = np.array([-math.log1p(-j.arrival_u) / rate for j in jobs], dtype=np.float64)
    return np.cumsum(gaps)


# ---------------------------------------------------------------------------
# Noisy video stream (restoration of a stream of frames).
# ---------------------------------------------------------------------------
def video_frame(rows: int, cols: int, f: int, seed: int = 8, noise: float = 0.3,
                blobs: int = 8) -> RestoreInput:
    """Frame f of a synthetic video: a sum of separable Gaussian blobs whose centres
    move at constant velocities, mapped to [16, 239], then salt-and-pepper impulses.

    Draw layout: blob b uses draws 6b..6b+5 (amplitude in [-1,1), centre row, centre
    column, width in [W/16, W/4), row and column velocity in [-2, 2) pixels per
    frame); blob b of frame f is amp * exp(-(r - cr)^2 / 2s^2) exp(-(c - cc)^2 / 2s^2)
    (an outer product) with the centre moved by f times the velocity. Each frame is
    mapped to [16, 239] on its own (round half to even). Pixel p of frame f uses
    draws 6*blobs + 2*(f*rows*cols + p) (impulse iff < noise) and the next one (salt
    iff < 0.5, else pepper)."""
    w = float(max(rows, cols))
    d = uniform01(seed, 0, 6 * blobs)
    r = np.arange(rows, dtype=np.float64)
    c = np.arange(cols, dtype=np.float64)
    field = np.zeros((rows, cols), dtype=np.float64)
    for b in range(blobs):
        amp = 2.0 * d[6 * b] - 1.0
        sig = w / 16.0 + d[6 * b + 3] * (w / 4.0 - w / 16.0)
        cr = d[6 * b + 1] * rows + f * (4.0 * d[6 * b + 4] - 2.0)
        cc = d[6 * b + 2] * cols + f * (4.0 * d[6 * b + 5] - 2.0)
        er = amp * np.exp(-(r - cr) ** 2 / (2.0 * sig * sig))
        ec = np.exp(-(c - cc) ** 2 / (2.0 * sig * sig))
        field += np.outer(er, ec)
    lo, hi = field.min(), field.max()
    scale = 223.0 / (hi - lo) if hi > lo else 0.0
    clean = np.rint(16.0 + (field - lo) * scale).astype(np.uint8)
    npx = rows * cols
    if noise <= 0.0:   # no impulse can be drawn
        return RestoreInput(y=clean.copy(), clean=clean, impulse=np.zeros((rows, cols), dtype=bool))
    hit = np.empty(npx, dtype=bool)
    salt = np.empty(npx, dtype=bool)
    lim_hit = _below_limit(noise) if noise < 1.0 else None
    lim_salt = _below_limit(0.5)
    for lo2, zz in _mixed_blocks(seed, 6 * blobs + 2 * f * npx, 2 * npx):
        p0 = lo2 // 2
        m = len(zz) // 2
        if lim_hit is None:
            hit[p0:p0 + m] = noise >= 1.0
        else:
            np.less(zz[0::2], lim_hit, out=hit[p0:p0 + m])
        np.less(zz[1::2], lim_salt, out=salt[p0:p0 + m])
    y = clean.reshape(-1).copy()
    y[hit & salt] = 255
    y[hit & ~salt] = 0
    return RestoreInput(y=y.reshape(rows, cols), clean=clean, impulse=hit.reshape(rows, cols))
