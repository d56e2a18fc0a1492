"""The counter-based instance generator (host side).

The device writes the same instances (tsylv_generate, serving requests that
carry only a seed); these tests pin the host definition: its Philox4x64-10
against numpy's own Philox bit generator, the element-to-counter map and the
Box-Muller step against a scalar rewrite of the definition, and the recipe's
structure and moments.
"""

import math

import numpy as np
import pytest

from paper_2405_09233_amd import workloads as wl


def _numpy_block(key, ctr):
    """Block `ctr` of numpy's Philox: it advances its 256-bit counter before
    it produces a block, so start it one below."""
    v = (sum(int(c) << (64 * i) for i, c in enumerate(ctr)) - 1) % 2**256
    start = np.array([(v >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=start)
    return [int(x) for x in bg.random_raw(4)]


def test_philox_matches_numpy_bit_generator():
    """numpy's Philox is Philox4x64-10."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        key = [int(x) for x in rng.integers(0, 2**64, size=2, dtype=np.uint64)]
        ctr = [int(x) for x in rng.integers(0, 2**64, size=4, dtype=np.uint64)]
        ref = _numpy_block(key, ctr)
        got = [int(w[0]) for w in wl.philox4x64(*[np.array([c], np.uint64) for c in ctr], *key)]
        assert got == ref


def test_philox_vectorised_over_counters():
    """One call over many counters equals the blocks one by one (counter 0
    included)."""
    e = np.array([0, 1, 2, 12345, 2**40 + 7], dtype=np.uint64)
    words = wl.philox4x64(e, np.full(5, 3, np.uint64), np.zeros(5, np.uint64),
                          np.zeros(5, np.uint64), 99, 2)
    for i, c in enumerate(e):
        assert [int(w[i]) for w in words] == _numpy_block([99, 2], [int(c), 3, 0, 0])


def _scalar_normal(seed, tid, rows, i, j, k):
    """One element of the stream, written out with Python integers."""
    w = _numpy_block([seed, tid], [i + rows * j, k // 4, 0, 0])
    u = [((x >> 12) + 0.5) / 2.0**52 for x in w]
    h = (k % 4) // 2
    r = math.sqrt(-2.0 * math.log(u[2 * h]))
    t = 2.0 * math.pi * u[2 * h + 1]
    return r * (math.cos(t) if k % 2 == 0 else math.sin(t))


@pytest.mark.parametrize("rows,cols,p", [(5, 3, 1), (4, 4, 6), (3, 7, 9)])
def test_element_map_and_box_muller(rows, cols, p):
    T = wl.philox_normal_tensor(17, 2, rows, cols, p)
    assert T.shape == (rows, cols, p) and T.flags.f_contiguous
    for i in range(rows):
        for j in range(cols):
            for k in range(p):
                assert abs(T[i, j, k] - _scalar_normal(17, 2, rows, i, j, k)) <= 1e-14


def test_uniforms_stay_inside_the_open_interval():
    """The extreme words map to 2^-53 and 1 - 2^-53, both exact."""
    lo = ((np.uint64(0) >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0**-52
    hi = ((np.uint64(2**64 - 1) >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0**-52
    assert lo == 2.0**-53 and hi == 1.0 - 2.0**-53


def test_instance_recipe():
    n, s, p = 40, 6, 8
    A, B, C = wl.philox_instance(5, n, s, p)
    ZA = wl.philox_normal_tensor(5, 0, n, n, p)
    ZB = wl.philox_normal_tensor(5, 1, s, s, p)
    fa, fb = 2.0 / np.sqrt(n * p), 2.0 / np.sqrt(s * p)
    assert np.array_equal(A[:, :, 1:], ZA[:, :, 1:] * fa)
    assert np.array_equal(A[:, :, 0], ZA[:, :, 0] * fa + 4.0 * np.eye(n))
    assert np.array_equal(B[:, :, 0], ZB[:, :, 0] * fb - 4.0 * np.eye(s))
    assert np.array_equal(C, wl.philox_normal_tensor(5, 2, n, s, p))
    # different tensors and seeds give different streams
    assert not np.allclose(ZA[:, :s, :], wl.philox_normal_tensor(5, 2, n, s, p))
    assert not np.allclose(C, wl.philox_instance(6, n, s, p)[2])


def test_moments():
    Z = wl.philox_normal_tensor(1, 0, 300, 200, 5).ravel()
    assert abs(Z.mean()) < 5.0 / np.sqrt(Z.size)
    assert abs(Z.var() - 1.0) < 0.01
    assert abs((Z**4).mean() - 3.0) < 0.05
    # the cos and sin halves of a Box-Muller pair are uncorrelated
    T = wl.philox_normal_tensor(1, 0, 300, 200, 4).reshape(-1, 4, order="F")
    assert abs(np.mean(T[:, 0] * T[:, 1])) < 0.01
