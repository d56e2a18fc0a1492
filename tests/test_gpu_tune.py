"""GPU tests of the apply's tile variants and the autotuner.

* Every tile variant of every precision, forced through the tuning table,
  gives tsylv_apply's result within the bars of the plain apply tests (FP64:
  64 eps (n + s) p amax xmax element-wise against the oracle's circulant
  sums; FP32 / BF16: relative 4 u sqrt(n + s) / 4 u), on ragged shapes that
  leave partial tiles in rows, columns and the k loop, odd and even p.
* tsylv_autotune returns a valid variant and positive times, records the
  choice, and solves that use it still match the oracle.
* The table survives a save / load round trip; a malformed file is rejected
  and merges nothing.
"""

import os

import numpy as np
import pytest

from oracle import kron, tproduct as tp
from paper_2405_09233_amd import tsylv, workloads
from gpu_util import ctx, dev, host, say, rel

EPS = np.finfo(np.float64).eps
U = {tsylv.FP32: 2.0 ** -24, tsylv.BF16: 2.0 ** -8}


def _operands(n, s, p, seed):
    rng = np.random.default_rng(seed)
    A = np.asfortranarray(rng.standard_normal((n, n, p)))
    B = np.asfortranarray(rng.standard_normal((s, s, p)))
    X = np.asfortranarray(rng.standard_normal((n, s, p)))
    return A, B, X


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [tsylv.FP64, tsylv.FP32, tsylv.BF16])
@pytest.mark.parametrize("n,s,p", [(70, 37, 5), (130, 20, 4), (33, 70, 1)])
def test_every_variant_matches_oracle(prec, n, s, p):
    c = ctx()
    A, B, X = _operands(n, s, p, seed=n + s + p)
    ref = tp.sylv_op(A, B, X)
    Ad, Bd, Xd = dev(A), dev(B), dev(X)
    try:
        for v in range(tsylv.apply_variants(prec)):
            say("variant", prec, v, n, s, p)
            c.tune_set(n, s, p, prec, v)
            Y = host(c.apply(Ad, Bd, Xd, prec=prec))
            if prec == tsylv.FP64:
                bound = 64 * EPS * (n + s) * p * max(np.abs(A).max(), np.abs(B).max()) \
                    * np.abs(X).max()
                assert np.abs(Y - ref).max() <= bound, (v, np.abs(Y - ref).max(), bound)
            else:
                u = U[prec]
                allowed = 4 * u * (np.sqrt(n + s) if prec == tsylv.FP32 else 1.0)
                assert rel(Y, ref) <= allowed, (v, rel(Y, ref), allowed)
    finally:
        c.tune_set(n, s, p, prec, -1)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [tsylv.FP64, tsylv.FP32, tsylv.BF16])
def test_autotune_choice_is_recorded_and_used(prec):
    n, s, p = 300, 24, 6
    c = ctx()
    say("autotune", prec, n, s, p)
    best, ms = c.autotune(n, s, p, prec=prec, reps=3)
    try:
        assert 0 <= best < tsylv.apply_variants(prec)
        assert len(ms) == tsylv.apply_variants(prec) and min(ms) > 0
        # the fastest, or the default tiles within 2 % of it
        assert ms[best] == min(ms) or ms[best] <= 1.02 * min(ms)
        assert c.tune_get(n, s, p, prec) == best
        # a solve of that shape runs with the tuned tiles and still converges
        A, B, C = workloads.dense_shifted(n, s, p, seed=9)
        if prec == tsylv.FP64:
            X, info = c.gmres(dev(A), dev(B), dev(C), m=30, tol=1e-10)
        else:
            X, info = c.gmres(dev(A), dev(B), dev(C), refine=1, prec=prec, inner_m=16, tol=1e-10)
        assert info.status == 0, info.as_dict()
        assert info.relres_true <= 1e-10
    finally:
        c.tune_set(n, s, p, prec, -1)


@pytest.mark.gpu
@pytest.mark.parametrize("variant", [3, 5])
def test_tuned_variant_solve_matches_kronecker(variant):
    n, s, p = 12, 5, 4
    c = ctx()
    say("tuned solve", variant)
    A, B, C = workloads.dense_shifted(n, s, p, seed=21)
    c.tune_set(n, s, p, tsylv.FP64, variant)
    try:
        X, info = c.gmres(dev(A), dev(B), dev(C), m=60, tol=1e-12)
        assert info.status == 0, info.as_dict()
        assert rel(host(X), kron.kron_solve(A, B, C)) <= 1e-9
    finally:
        c.tune_set(n, s, p, tsylv.FP64, -1)


@pytest.mark.gpu
def test_tune_file_round_trip(tmp_path):
    c = ctx()
    entries = [(tsylv.FP64, 4096, 64, 32, 2), (tsylv.BF16, 8192, 128, 64, 1), (tsylv.FP32, 7, 3, 2, 4)]
    for prec, n, s, p, v in entries:
        c.tune_set(n, s, p, prec, v)
    path = str(tmp_path / "tune.txt")
    c.tune_save(path)
    with open(path) as f:
        text = f.read()
    assert text.splitlines()[0] == "tsylv-tune 1"
    other = tsylv.Context(1 << 28, device=0)
    try:
        other.tune_load(path)
        for prec, n, s, p, v in entries:
            assert other.tune_get(n, s, p, prec) == v
        bad = str(tmp_path / "bad.txt")
        with open(bad, "w") as f:
            f.write("tsylv-tune 1\n0 10 2 3 1\n1 10 2 3 99\n")  # variant 99 does not exist
        with pytest.raises(tsylv.TsylvError):
            other.tune_load(bad)
        assert other.tune_get(10, 2, 3, tsylv.FP64) == -1  # nothing merged
        with pytest.raises(tsylv.TsylvError):
            other.tune_load(str(tmp_path / "missing.txt"))
        with pytest.raises(tsylv.TsylvError):
            other.tune_set(5, 5, 5, tsylv.FP64, tsylv.apply_variants(tsylv.FP64))
    finally:
        other.close()
        for prec, n, s, p, _ in entries:
            c.tune_set(n, s, p, prec, -1)
    assert os.path.exists(path)
