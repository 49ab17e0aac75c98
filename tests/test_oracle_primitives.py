"""Pins of the oracle's determinism primitives: Philox4x32-10 against the
published known-answer vectors, the deterministic log/exp/pow against the C
library to a few ulp, and the keyed permutation that forms the candidate
pairs, a Feistel network on Z_m x Z_m with modular addition (bijectivity,
uniformity of the ordered pairs it forms at several cell sizes and pair
positions, and of single positions in a large cell)."""
import math
import os

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(orc):
    for ctr, key, want in _kat():
        got = orc.philox(key, ctr)
        assert [int(x) for x in got] == want


def _ulps(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    ia = a.view(np.int64)
    ib = b.view(np.int64)
    return np.abs(ia - ib)


def test_detlog_matches_libm(orc):
    rng = np.random.default_rng(1)
    xs = np.concatenate([
        np.exp(rng.uniform(-700, 700, 4000)),
        rng.uniform(0.5, 2.0, 4000),
        1.0 + rng.uniform(-1e-6, 1e-6, 1000),
        np.array([1e-310, 5e-324, 2.0, 0.5, math.e, 10.0, 1e300]),
    ])
    got = np.array([orc.detlog(x) for x in xs])
    want = np.log(xs)
    nz = np.abs(want) > 1e-300
    assert np.max(_ulps(got[nz], want[nz])) <= 2
    assert orc.detlog(1.0) == 0.0
    assert orc.detlog(0.0) == -math.inf


def test_detexp_matches_libm(orc):
    rng = np.random.default_rng(2)
    xs = np.concatenate([rng.uniform(-700, 700, 6000), rng.uniform(-1, 1, 2000), np.array([0.0, 1.0, -1.0])])
    got = np.array([orc.detexp(x) for x in xs])
    want = np.exp(xs)
    assert np.max(_ulps(got, want)) <= 2
    assert orc.detexp(0.0) == 1.0
    assert orc.detexp(800.0) == math.inf
    assert orc.detexp(-800.0) == 0.0


def test_detpow_matches_libm(orc):
    rng = np.random.default_rng(3)
    x = np.exp(rng.uniform(-40, 40, 3000))
    y = rng.uniform(0.0, 2.0, 3000)
    got = np.array([orc.detpow(a, b) for a, b in zip(x, y)])
    want = x ** y
    rel = np.abs(got - want) / want
    bound = 4e-16 * (1.0 + np.abs(y * np.log(x)))
    assert np.all(rel <= bound)
    assert orc.detpow(0.0, 0.26) == 0.0
    assert orc.detpow(1.0, 0.76) == 1.0


@pytest.mark.parametrize("n", list(range(2, 70)) + [255, 256, 257, 1000, 4096, 10000])
def test_feistel_is_permutation(orc, n):
    keys = np.concatenate([orc.philox((7, 9), (b, 0xFFFFFFFF, n, 3)) for b in range(4)])
    perm = [orc.feistel_index(n, keys, i) for i in range(n)]
    assert sorted(perm) == list(range(n))


@pytest.mark.parametrize("n,k", [(5, 0), (8, 0), (20, 0), (100, 0), (65, 7), (9, 2)])
def test_feistel_pairs_are_uniform(orc, n, k):
    # over many keys, candidate pair k, (pi(2k), pi(2k+1)), of a cell must hit
    # each ordered pair equally often (m = 3, 3, 5, 10, 9, 3: both round counts)
    counts = np.zeros((n, n), np.int64)
    for s in range(max(28000, 40 * n * (n - 1))):
        keys = np.concatenate([orc.philox((11, 0), (b, 0xFFFFFFFF, 5, s)) for b in range(4)])
        p, q = orc.feistel_index(n, keys, 2 * k), orc.feistel_index(n, keys, 2 * k + 1)
        assert p != q
        counts[p, q] += 1
    obs = counts[~np.eye(n, dtype=bool)]
    assert stats.chisquare(obs).pvalue > 1e-4


def test_feistel_positions_are_uniform_in_a_large_cell(orc):
    # a single position of the permutation (as a third body takes it) is
    # uniform over a 300-particle cell (m = 18, one cycle-walk step in ~8)
    n = 300
    counts = np.zeros(n, np.int64)
    for s in range(30000):
        keys = np.concatenate([orc.philox((3, 1), (b, 0xFFFFFFFF, 9, s)) for b in range(4)])
        counts[orc.feistel_index(n, keys, 123)] += 1
    assert stats.chisquare(counts).pvalue > 1e-4
