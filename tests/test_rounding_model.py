"""CPU model of the FP32 Helmholtz update's stochastic rounding (tile_jacobi.hpp:
hash32, add_round_stochastic, the FP32 branch of jacobi_update), replayed in numpy
float32 arithmetic, checked against exact rational arithmetic.

* Fast2Sum gives the exact remainder whenever |c| <= |p|, which the update's
  operands satisfy for |0.25 - rd| <= 1/8 (the range lsr_run accepts for FP32).
* The rounded value is fl(p + c) or one ulp step from it towards p + c, and
  averaged over the 256 byte values it equals p + c to within 1/512 ulp.
* Each lane's four cells share one hash and take distinct bytes of it.
"""
from fractions import Fraction

import numpy as np

F = np.float32
ULP_MASK = np.uint32(0x7F800000)


def hash32(x):
    x = np.uint32(x)
    x ^= x >> np.uint32(16)
    x = np.uint32((int(x) * 0x7FEB352D) & 0xFFFFFFFF)
    x ^= x >> np.uint32(15)
    x = np.uint32((int(x) * 0x846CA68B) & 0xFFFFFFFF)
    x ^= x >> np.uint32(16)
    return x


def kernel_ulp(hi):
    """2^(e - 23) for the exponent e of hi, as the kernel forms it from the bits."""
    bits = np.array([hi], F).view(np.uint32)[0] & ULP_MASK
    return F(np.array([bits], np.uint32).view(F)[0] * F(2.0 ** -23))


def round_stochastic(p, c, bits8):
    p, c = F(p), F(c)
    hi = F(p + c)
    rem = F(c - F(hi - p))
    ulp = kernel_ulp(hi)
    u = F(F(F(bits8) + F(0.5)) * F(1.0 / 256))
    return F(hi + np.copysign(ulp, rem)) if abs(rem) > F(u * ulp) else hi


def update_operands(sn, gv, rd):
    """p and c of the FP32 update: t + e = sn + gv exactly, p = t/4, c = e/4 - (1/4 - rd) t."""
    sn, gv = F(sn), F(gv)
    tt = F(sn + gv)
    bb = F(tt - sn)
    te = F(F(sn - F(tt - bb)) + F(gv - bb))
    rd_lo = F(0.25 - rd)
    return F(F(0.25) * tt), F(F(F(0.25) * te) - F(rd_lo * tt)), tt, te


def test_fast2sum_remainder_is_exact_in_the_accepted_range():
    rng = np.random.default_rng(7)
    for rd in (0.125, 0.2, 0.25 - 2.0 ** -20, 0.25, 0.3, 0.375):
        for _ in range(400):
            sn = F(rng.uniform(-4, 4) * 10.0 ** rng.integers(-6, 3))
            gv = F(rng.uniform(-1, 1) * 10.0 ** rng.integers(-12, 1))
            p, c, tt, te = update_operands(sn, gv, rd)
            assert Fraction(float(tt)) + Fraction(float(te)) == Fraction(float(sn)) + Fraction(float(gv))
            assert abs(c) <= abs(p)
            hi = F(p + c)
            rem = F(c - F(hi - p))
            assert Fraction(float(hi)) + Fraction(float(rem)) == Fraction(float(p)) + Fraction(float(c))


def test_rounding_moves_by_at_most_one_step_and_is_unbiased():
    rng = np.random.default_rng(11)
    for trial in range(60):
        p = F(rng.uniform(0.5, 4.0) * 10.0 ** rng.integers(-4, 3))
        if trial < 4:
            p = F(2.0 ** (trial - 1))   # p + c next to a power of two
        c = F(p * F(rng.uniform(-0.4, 0.4)) * F(2.0 ** -20))
        exact = Fraction(float(p)) + Fraction(float(c))
        hi = F(p + c)
        ulp = kernel_ulp(hi)
        step = F(hi + np.copysign(ulp, F(c - F(hi - p))))
        vals = [round_stochastic(p, c, k) for k in range(256)]
        assert all(v in (hi, step) for v in vals)
        # the step and its probability use the same ulp, so the mean is the exact sum
        mean = sum(Fraction(float(v)) for v in vals) / 256
        assert abs(mean - exact) <= Fraction(float(ulp)) / 512


def test_a_lane_shares_one_hash_across_its_four_cells():
    row, sweep = 37, 1234
    keys = set()
    for col in range(64, 68):
        key = (row * 0x9E3779B1 ^ (col >> 2) * 0x85EBCA77 ^ sweep * 0xC2B2AE3D) & 0xFFFFFFFF
        keys.add(key)
    assert len(keys) == 1
    h = int(hash32(keys.pop()))
    assert len({(h >> (8 * (col & 3))) & 0xFF for col in range(64, 68)}) >= 3
