"""The comparator networks of csrc/select_networks.hpp (the detection's minimum,
lower median and maximum of full 3x3, 5x5 and 7x7 windows); the first two checked
exhaustively by the 0-1 principle: a comparator network puts the rank-r element into a register for
every input iff it does so for every input of zeros and ones. All 2^9 and 2^25
0-1 inputs are run bit-parallel (one bit per input, 64 inputs per word); the 3x3
network is also checked against a fresh run of its generator."""
import os
import re

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_1609_04567_amd", "csrc")
HEADER = os.path.join(CSRC, "select_networks.hpp")


def _parse(count):
    text = open(HEADER).read()
    m = re.search(r"constexpr int kSel%dMin = (\d+), kSel%dMed = (\d+), kSel%dMax = (\d+);"
                  % (count, count, count), text)
    outs = [int(x) for x in m.groups()]
    body = text[text.index("void select%d(" % count):]
    body = body[:body.index("\n}\n")]
    ops = [(int(a), int(b)) for a, b in
           re.findall(r"min\(v\[(\d+)\], v\[(\d+)\]\)", body)]
    return ops, outs


def _wires(count):
    """Bit k of input x, for every x in [0, 2^count), as uint64 words."""
    nwords = max(1, (1 << count) // 64)
    idx = np.arange(nwords, dtype=np.uint64)
    low = [0xAAAAAAAAAAAAAAAA, 0xCCCCCCCCCCCCCCCC, 0xF0F0F0F0F0F0F0F0,
           0xFF00FF00FF00FF00, 0xFFFF0000FFFF0000, 0xFFFFFFFF00000000]
    full = np.uint64(0xFFFFFFFFFFFFFFFF)
    w = []
    for k in range(count):
        if k < 6:
            w.append(np.full(nwords, low[k], dtype=np.uint64))
        else:
            w.append(np.where((idx >> np.uint64(k - 6)) & np.uint64(1), full, np.uint64(0)))
    if count < 6:   # fewer inputs than a word: keep the first 2^count bits
        mask = np.uint64((1 << (1 << count)) - 1)
        w = [x & mask for x in w]
    return w


def _at_least(w, m):
    """Bit-parallel [number of ones among the wires >= m]."""
    # counts as bit slices, then a comparison with m
    nbits = max(1, len(w).bit_length())
    cnt = [np.zeros_like(w[0]) for _ in range(nbits)]
    for x in w:
        carry = x
        for b in range(nbits):
            cnt[b], carry = cnt[b] ^ carry, cnt[b] & carry
    # cnt >= m  <=>  not (cnt < m); compare from the top bit
    gt = np.zeros_like(w[0])
    eq = ~np.zeros_like(w[0])
    for b in reversed(range(nbits)):
        mb = (m >> b) & 1
        if mb:
            eq = eq & cnt[b]
        else:
            gt = gt | (eq & cnt[b])
            eq = eq & ~cnt[b]
    return gt | eq


@pytest.mark.parametrize("count", [9, 25])
def test_network_selects_min_median_max_for_every_01_input(count):
    ops, (rmin, rmed, rmax) = _parse(count)
    assert ops, "no comparators parsed"
    v = _wires(count)
    for a, b in ops:
        v[a], v[b] = v[a] & v[b], v[a] | v[b]
    rank = (count - 1) // 2
    # the rank-r element of a 0-1 input is 1 iff it has at least count - r ones
    assert np.array_equal(v[rmin], _at_least(_wires(count), count))
    assert np.array_equal(v[rmed], _at_least(_wires(count), count - rank))
    assert np.array_equal(v[rmax], _at_least(_wires(count), 1))


@pytest.mark.parametrize("count", [9, 25, 49])
def test_network_on_random_bytes(count):
    ops, (rmin, rmed, rmax) = _parse(count)
    rng = np.random.default_rng(count)
    x = rng.integers(0, 256, size=(count, 20000))
    x[:, :5000] = rng.integers(0, 3, size=(count, 5000))     # many ties
    v = [x[k].copy() for k in range(count)]
    for a, b in ops:
        v[a], v[b] = np.minimum(v[a], v[b]), np.maximum(v[a], v[b])
    s = np.sort(x, axis=0)
    assert np.array_equal(v[rmin], s[0])
    assert np.array_equal(v[rmed], s[(count - 1) // 2])
    assert np.array_equal(v[rmax], s[-1])


def test_generator_sorts_and_reproduces_the_3x3_network():
    """The generator's Batcher network sorts every 0-1 input of 16 wires, and its
    3x3 selection network is the header's (the 5x5 one takes half a minute to
    regenerate; the header's is checked exhaustively above)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("gen_select", os.path.join(CSRC, "gen_select.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    pairs = gen.batcher_pairs(16)
    x = np.array([[(i >> k) & 1 for k in range(16)] for i in range(1 << 16)], dtype=np.uint8)
    for a, b in pairs:
        lo, hi = np.minimum(x[:, a], x[:, b]), np.maximum(x[:, a], x[:, b])
        x[:, a], x[:, b] = lo, hi
    assert (np.diff(x.astype(np.int8), axis=1) >= 0).all()
    ops, outs = gen.selection_network(9, 16, [0, 4, 8])
    assert (ops, outs) == _parse(9)
    # the 7x7 network is the backward-pruned Batcher network (no greedy step): an
    # exact pruning, since a dropped comparator writes nothing that reaches an output
    ops, outs = gen.selection_network(49, 64, [0, 24, 48], greedy=False)
    assert (ops, outs) == _parse(49)


def test_49_network_on_random_01_inputs():
    """2^20 random 0-1 inputs (bit-parallel, 64 per word), each wire's bit drawn
    with a per-word probability so every count of ones is well covered."""
    ops, (rmin, rmed, rmax) = _parse(49)
    rng = np.random.default_rng(11)
    nwords = 1 << 14
    p = rng.uniform(0.2, 0.8, size=nwords)   # density of ones of each word's 64 inputs
    bits = rng.random((49, nwords, 64)) < p[None, :, None]
    weights = (1 << np.arange(64, dtype=np.uint64)).astype(np.uint64)
    w = [(bits[k].astype(np.uint64) * weights).sum(axis=1, dtype=np.uint64) for k in range(49)]
    v = list(w)
    for a, b in ops:
        v[a], v[b] = v[a] & v[b], v[a] | v[b]
    assert np.array_equal(v[rmin], _at_least(w, 49))
    assert np.array_equal(v[rmed], _at_least(w, 25))
    assert np.array_equal(v[rmax], _at_least(w, 1))


def test_49_network_on_structured_inputs():
    """All-equal runs, two-valued inputs with every count of ones at every
    position shift, and sorted / reversed byte ramps (the cases a selection
    network gets wrong first)."""
    ops, (rmin, rmed, rmax) = _parse(49)
    rng = np.random.default_rng(7)
    cases = []
    for ones in range(50):
        for _ in range(40):
            x = np.zeros(49, dtype=np.int64)
            x[rng.permutation(49)[:ones]] = 1
            cases.append(x)
    cases += [np.arange(49), np.arange(49)[::-1], np.full(49, 7)]
    x = np.array(cases).T
    v = [x[k].copy() for k in range(49)]
    for a, b in ops:
        v[a], v[b] = np.minimum(v[a], v[b]), np.maximum(v[a], v[b])
    s = np.sort(x, axis=0)
    assert np.array_equal(v[rmin], s[0])
    assert np.array_equal(v[rmed], s[24])
    assert np.array_equal(v[rmax], s[-1])
