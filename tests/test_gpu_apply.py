"""GPU parity of tsylv_apply (Y = A*X - X*B through the half-spectrum Fourier
planes) against the oracle's circulant sums, element by element.

Tolerance: every entry of M(X) is a sum of (n + s) p products of inputs of
size <= amax * xmax; the DFT, the slice products and the inverse DFT add
rounding of the same order, so |Y - Y_oracle| <= 64 eps (n + s) p amax xmax
is a safe FP64 bound (the observed error is orders of magnitude below it)."""

import numpy as np
import pytest

from oracle import tproduct as tp
from gpu_util import ctx, dev, host, say, workload

EPS = np.finfo(np.float64).eps

SHAPES = [(8, 6, 4), (1, 1, 1), (5, 3, 1), (7, 2, 2), (9, 4, 3), (2, 5, 2), (33, 1, 6),
          (70, 5, 5), (64, 64, 8), (130, 70, 7), (65, 17, 9), (100, 3, 64), (40, 4, 65)]


def bound(A, B, X):
    n, s, p = X.shape
    amax = max(np.abs(A).max(), np.abs(B).max())
    return 64 * EPS * (n + s) * p * amax * np.abs(X).max()


@pytest.mark.gpu
@pytest.mark.parametrize("n,s,p", SHAPES)
def test_apply_matches_oracle(n, s, p):
    say("apply", n, s, p)
    rng = np.random.default_rng(n * 1000 + s * 10 + p)
    A = np.asfortranarray(rng.standard_normal((n, n, p)))
    B = np.asfortranarray(rng.standard_normal((s, s, p)))
    X = np.asfortranarray(rng.standard_normal((n, s, p)))
    c = ctx()
    Y = host(c.apply(dev(A), dev(B), dev(X)))
    ref = tp.sylv_op(A, B, X)
    err = np.abs(Y - ref).max()
    assert err <= bound(A, B, X), (err, bound(A, B, X))


@pytest.mark.gpu
def test_apply_full_size_sampled():
    """n = 4096, s = 64, p = 32 convection-diffusion operator, the launch
    configuration of the benchmark; 64 random entries (and the first/last
    rows and slices) checked against the oracle's per-entry circulant sums."""
    say("apply full size 4096/64/32")
    A, B, C = workload("cd_4096")
    n, s, p = C.shape
    c = ctx()
    Ad = dev(A)
    Y = host(c.apply(Ad, dev(B), dev(C)))
    rng = np.random.default_rng(7)
    idx = [(int(rng.integers(n)), int(rng.integers(s)), int(rng.integers(p))) for _ in range(64)]
    idx += [(0, 0, 0), (n - 1, s - 1, p - 1), (n - 1, 0, p // 2), (0, s - 1, 1)]
    ref = tp.sylv_op_entries(A, B, C, idx)
    got = np.array([Y[i, j, k] for i, j, k in idx])
    err = np.abs(got - ref).max()
    assert err <= bound(A, B, C), (err, bound(A, B, C))
