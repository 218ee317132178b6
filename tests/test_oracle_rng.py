"""Pins for the oracle's counter-based generator and the test matrices it draws.

The Philox bijection is pinned to numpy's own Philox4x64-10 (a library
implementation of the same published generator); the Gaussian and SRFT draws
are pinned by distributional facts: normality, the closed-form moment of a
pseudo-inverted Gaussian (Proposition 10.2), sampling without replacement.
"""

import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _numpy_philox_block(counter, key):
    # numpy's Philox increments the 256-bit counter before each block, so the
    # first block it returns for counter c is the bijection applied to c + 1.
    c = np.array(counter, dtype=np.uint64).copy()
    # step back by one (no borrow in the cases used here)
    assert c[0] > 0
    c[0] -= np.uint64(1)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=c)
    return [int(v) for v in bg.random_raw(4)]


@pytest.mark.parametrize("counter,key", [
    ((1, 0, 0, 0), (0, 0)),
    ((5, 7, 0, 0), (0x09094061, 0)),
    ((123456789, 3, 2, 0), (42, 0)),
    ((2**40 + 17, 2**63 + 5, 2**62, 99), (2**64 - 1, 2**63)),
])
def test_philox_matches_numpy(counter, key):
    ours = philox.philox4x64(*[np.uint64(c) for c in counter], key[0], key[1])
    ours = [int(np.asarray(v).reshape(())) for v in ours]
    assert ours == _numpy_philox_block(counter, key)


def test_philox_vectorized_equals_scalar():
    t = np.arange(1, 200, dtype=np.uint64)
    vec = philox.philox4x64(t, np.uint64(3), np.uint64(0), 0, 77)
    for i in (0, 1, 50, 198):
        sc = philox.philox4x64(t[i], np.uint64(3), np.uint64(0), 0, 77)
        assert [int(v[i]) for v in vec] == [int(np.asarray(s).reshape(())) for s in sc]


def test_uniform_bounds():
    u = philox.uniform_from_word(np.array([0, 2**64 - 1, 2**63], dtype=np.uint64))
    assert u[0] == 2.0 ** -53
    assert u[1] == 1.0 - 2.0 ** -53
    assert u[2] == 0.5 + 2.0 ** -53
    assert np.all((u > 0) & (u < 1))


def test_gaussian_is_standard_normal():
    g = philox.gaussian_omega(4000, 37, seed=2024, stream=0).ravel()
    assert abs(g.mean()) < 4.0 / np.sqrt(g.size)
    assert abs(g.var() - 1.0) < 6.0 * np.sqrt(2.0 / g.size)
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # no two entries of one quad are the same variable
    assert len(np.unique(g)) == g.size


def test_gaussian_columns_independent():
    g = philox.gaussian_omega(20000, 8, seed=5, stream=0)
    C = np.corrcoef(g.T)
    off = C[~np.eye(8, dtype=bool)]
    assert np.max(np.abs(off)) < 5.0 / np.sqrt(20000)


def test_gaussian_layout_is_quad_major():
    # Entry (i, j) lives in quad t = i*ceil(l/4) + j//4, lane j % 4: the first
    # row of a wide draw equals the first quads of the flat stream.
    n, l = 3, 10
    g = philox.gaussian_omega(n, l, seed=11, stream=4)
    flat = philox.gaussian_omega(1, n * 12, seed=11, stream=4).reshape(n, 12)
    np.testing.assert_array_equal(g, flat[:, :l])


def test_gaussian_streams_and_seeds_differ():
    a = philox.gaussian_omega(50, 8, seed=1, stream=0)
    b = philox.gaussian_omega(50, 8, seed=1, stream=10)
    c = philox.gaussian_omega(50, 8, seed=2, stream=0)
    assert not np.any(a == b) and not np.any(a == c)


def test_pinv_gaussian_moment_prop_10_2():
    # Proposition 10.2: for a k x (k+p) standard Gaussian G, E ||G^+||_F^2 = k/(p-1).
    k, p, trials = 6, 5, 3000
    vals = []
    for t in range(trials):
        G = philox.gaussian_omega(k, k + p, seed=1000 + t, stream=0)
        vals.append(np.linalg.norm(np.linalg.pinv(G), "fro") ** 2)
    vals = np.array(vals)
    expect = k / (p - 1.0)
    se = vals.std() / np.sqrt(trials)
    assert abs(vals.mean() - expect) < 4 * se + 0.02 * expect


def test_srft_signs():
    d = philox.srft_signs(100000, seed=9, stream=0)
    assert set(np.unique(d)) == {-1.0, 1.0}
    assert abs(d.mean()) < 4.0 / np.sqrt(d.size)


def test_srft_sample_without_replacement():
    for seed in range(20):
        R = philox.srft_sample(257, 64, seed=seed, stream=0)
        assert len(set(R.tolist())) == 64
        assert R.min() >= 0 and R.max() < 257
    R = philox.srft_sample(16, 16, seed=3, stream=0)
    assert sorted(R.tolist()) == list(range(16))


def test_srft_sample_uniform():
    # Each coordinate is equally likely to be drawn first, and to be drawn at all.
    n, l, trials = 12, 3, 6000
    first = np.zeros(n)
    anyhit = np.zeros(n)
    for s in range(trials):
        R = philox.srft_sample(n, l, seed=s, stream=0)
        first[R[0]] += 1
        anyhit[R] += 1
    assert stats.chisquare(first).pvalue > 1e-3
    assert stats.chisquare(anyhit).pvalue > 1e-3


def test_golden_draws_unchanged():
    # Frozen draws written by tests/golden/make_golden.py (oracle only): a change
    # to the generator contract shows up here before it desynchronizes anything.
    data = np.loadtxt(os.path.join(GOLDEN, "omega_seed09094061_n6_l7.txt"))
    np.testing.assert_array_equal(philox.gaussian_omega(6, 7, seed=0x09094061, stream=0), data)
    sr = np.loadtxt(os.path.join(GOLDEN, "srft_seed09094061_n32_l8.txt"))
    np.testing.assert_array_equal(philox.srft_signs(32, seed=0x09094061, stream=0), sr[0])
    np.testing.assert_array_equal(philox.srft_sample(32, 8, seed=0x09094061, stream=0),
                                  sr[1, :8].astype(np.int64))
