"""Pins of the oracle's noise sources.

Philox4x64-10 (Salmon et al. 2011) is pinned against numpy's independent
implementation of the same generator: numpy advances its 256-bit counter
before producing a block, so the block for counter c is numpy's first block
when it is seeded with c - 1.  Philox4x32-10 (the same paper; the DPD pair
noise) is pinned against rocRAND's host implementation.  The Gaussian draws
are pinned by their moments.
"""
import numpy as np
import pytest

import oracle
import rocrand_ref


def numpy_block(counter, key):
    c = sum(int(v) << (64 * i) for i, v in enumerate(counter))
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.asarray(key, dtype=np.uint64), counter=words)
    return bg.random_raw(4)


@pytest.mark.parametrize("counter,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([1, 0, 0, 0], [5, 7]),
    ([12345, 678, 0, 0], [1001, 0]),
    ([0, 1, 0, 0], [2**63 + 5, 3]),          # carry across words in numpy's decrement
    ([2**64 - 1, 2**32, 9, 2**60], [2**64 - 1, 2**64 - 1]),
])
def test_philox_matches_numpy(counter, key):
    assert np.array_equal(oracle.philox(counter, key), numpy_block(counter, key))


def test_philox_many_counters_match_numpy():
    g = np.random.default_rng(0)
    for _ in range(50):
        ctr = [int(x) for x in g.integers(0, 2**63, size=4)]
        key = [int(x) for x in g.integers(0, 2**63, size=2)]
        assert np.array_equal(oracle.philox(ctr, key), numpy_block(ctr, key))


def test_gauss3_moments_and_independence():
    n = 40000
    z = np.array([oracle.gauss3(1234, 0, 17, t) for t in range(n)])
    m = z.mean(axis=0)
    v = z.var(axis=0)
    assert np.all(np.abs(m) < 5 / np.sqrt(n))
    assert np.all(np.abs(v - 1) < 5 * np.sqrt(2.0 / n))
    k4 = (z ** 4).mean(axis=0)
    assert np.all(np.abs(k4 - 3) < 5 * np.sqrt(96.0 / n))
    c = np.corrcoef(z.T)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 5 / np.sqrt(n))
    # different steps and streams give different draws
    assert not np.array_equal(oracle.gauss3(1234, 0, 17, 5), oracle.gauss3(1234, 0, 18, 5))
    assert not np.array_equal(oracle.gauss3(1234, 0, 17, 5), oracle.gauss3(1234, 1, 17, 5))


def test_gauss3_tail_probability():
    n = 30000
    z = np.array([oracle.gauss3(99, 0, 3, t) for t in range(n)]).ravel()
    frac = np.mean(np.abs(z) > 2.0)
    # P(|z| > 2) = 0.0455 for a standard normal
    assert abs(frac - 0.0455003) < 5 * np.sqrt(0.0455 * 0.9545 / z.size)


def test_philox32_matches_rocrand():
    g = np.random.default_rng(3)
    ctrs = [[0, 0, 0, 0], [1, 0, 0, 0], [0xFFFFFFFF] * 4, [0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
            [7, 0xFFFFFFFF, 1, 0]] + [list(g.integers(0, 2**32, size=4)) for _ in range(40)]
    keys = [[0, 0], [5, 7], [0xFFFFFFFF] * 2, [0xA4093822, 0x299F31D0], [1, 2]] + \
        [list(g.integers(0, 2**32, size=2)) for _ in range(40)]
    ref = rocrand_ref.blocks(ctrs, keys)
    if ref is None:
        pytest.skip("hipcc or the rocRAND header is not available")
    mine = np.array([oracle.philox32(c, k) for c, k in zip(ctrs, keys)])
    assert np.array_equal(mine, ref)
