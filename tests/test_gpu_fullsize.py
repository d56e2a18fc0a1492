"""GPU parity at the full benchmark sizes, in the launch plans the benchmark
and the solves use.

* Every tile variant of the FP64, FP32 and BF16 apply at n = 4096, s = 64,
  p = 32 and at n = 8192, s = 128, p = 64 (convection-diffusion operators):
  68 sampled entries of Y = M(X) against the oracle's per-entry circulant
  sums.  Two bars for FP32 / BF16 (FP64 keeps the plain apply bound):
    - element-wise, a rigorous bound.  Slice k's product is formed from
      operands rounded to unit roundoff u (each part of a complex entry
      separately) and accumulated in FP32 over K = n + s terms with up to
      four real products per complex entry, so its error is at most
      (2 u + 4 gamma_{K+2}) (|Ahat_k| |Vhat_k| + |Vhat_k| |Bhat_k|) entry by
      entry, gamma_K = K 2^-24.  Since |Ahat_k| <= sum_t |A_t| entry-wise
      (likewise V, B) and the inverse DFT averages the p slices, entry
      (i, j, t) of Y is off by at most that factor times
      T(i, j) = sum_l Asum(i, l) Xsum(l, j) + sum_l Xsum(i, l) Bsum(l, j),
      Asum = sum_t |A_t|; the test allows twice that, plus the FP64 bound of
      the transforms;
    - normwise over the sample, the bar of the small-size tests: relative
      error <= 4 u (BF16) or 4 u sqrt(n + s) (FP32).
* A solution known exactly: X* random, C = M(X*) by the oracle's circulant
  sums, at n = 4096, s = 64, p = 32; the FP64 path (to relres 1e-11) must
  return X* within 1e-8, the FP32- and BF16-refined paths (to 1e-10) within
  1e-7 -- the solution bars of the FP64 and refined paths.
* n = 8192, s = 128, p = 64 (the mixed-precision configuration): refinement
  around FP32 / BF16 tGMRES(40) inner cycles to relres 1e-8 (true residual,
  48 sampled residual entries from the oracle), and, solved to 1e-10, the
  refined solution against the FP64 tGMRES(40) solution within 1e-7.  An
  oracle solve at this size is out of reach (one apply by circulant sums is
  7e13 flops); the FP64 path stands in, pinned to the oracle by the test
  above and by the small-size solution tests.
"""

import numpy as np
import pytest

from oracle import tproduct as tp
from paper_2405_09233_amd import tsylv
from gpu_util import ctx, dev, host, say, rel, workload

EPS = np.finfo(np.float64).eps
U = {tsylv.FP32: 2.0 ** -24, tsylv.BF16: 2.0 ** -8}
ARENA_GB = {"cd_4096": 24, "cd_8192": 96}


def _sample(n, s, p, seed):
    rng = np.random.default_rng(seed)
    idx = [(int(rng.integers(n)), int(rng.integers(s)), int(rng.integers(p))) for _ in range(64)]
    return idx + [(0, 0, 0), (n - 1, s - 1, p - 1), (n - 1, 0, p // 2), (0, s - 1, 1)]


def _abs_sums(A, B, X, idx):
    """T(i, j) of the module docstring for every sampled (i, j, t)."""
    Xsum = np.abs(X).sum(axis=2)
    Bsum = np.abs(B).sum(axis=2)
    rows = {}
    out = np.empty(len(idx))
    for e, (i, j, _) in enumerate(idx):
        if i not in rows:
            rows[i] = np.abs(A[i, :, :]).sum(axis=1)
        out[e] = rows[i] @ Xsum[:, j] + Xsum[i, :] @ Bsum[:, j]
    return out


_REF = {}


def _reference(name):
    """(A, B, X, idx, oracle entries, T) of a full-size workload, X = C."""
    if name not in _REF:
        A, B, C = workload(name)
        n, s, p = C.shape
        idx = _sample(n, s, p, seed=7)
        say("oracle entries", name)
        ref = tp.sylv_op_entries(A, B, C, idx)
        _REF[name] = (A, B, C, idx, ref, _abs_sums(A, B, C, idx))
    return _REF[name]


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [tsylv.FP64, tsylv.FP32, tsylv.BF16])
@pytest.mark.parametrize("name", ["cd_4096", "cd_8192"])
def test_apply_full_size_every_variant(name, prec):
    A, B, X, idx, ref, T = _reference(name)
    n, s, p = X.shape
    c = ctx(arena_gb=ARENA_GB[name])
    Ad, Bd, Xd = dev(A), dev(B), dev(X)
    fp64_bound = 64 * EPS * (n + s) * p * max(np.abs(A).max(), np.abs(B).max()) \
        * np.abs(X).max()
    try:
        for v in range(tsylv.apply_variants(prec)):
            say("full-size apply", name, "prec", prec, "variant", v)
            c.tune_set(n, s, p, prec, v)
            Y = c.apply(Ad, Bd, Xd, prec=prec)
            Yh = host(Y)
            del Y
            got = np.array([Yh[i, j, k] for i, j, k in idx])
            err = np.abs(got - ref)
            if prec == tsylv.FP64:
                assert err.max() <= fp64_bound, (v, err.max(), fp64_bound)
                continue
            u = U[prec]
            K = n + s
            elem = 2 * (2 * u + 4 * (K + 2) * 2.0 ** -24) * T + fp64_bound
            assert np.all(err <= elem), (v, int(np.argmax(err / elem)), (err / elem).max())
            normwise = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            allowed = 4 * u * (np.sqrt(K) if prec == tsylv.FP32 else 1.0)
            say("  normwise sample error %.3e (bar %.3e)" % (normwise, allowed))
            assert normwise <= allowed, (v, normwise, allowed)
    finally:
        c.tune_set(n, s, p, prec, -1)
        del Ad, Bd, Xd


_MANUFACTURED = {}


def _manufactured():
    """X* ~ N(0, 1) and C = M(X*) by the oracle at n = 4096, s = 64, p = 32."""
    if "data" not in _MANUFACTURED:
        A, B, _ = workload("cd_4096")
        n, s, p = A.shape[0], B.shape[0], A.shape[2]
        rng = np.random.default_rng(31)
        Xs = rng.standard_normal(n * s * p).reshape((n, s, p), order="F")
        say("oracle M(X*) at 4096/64/32")
        C = np.asfortranarray(tp.sylv_op(A, B, Xs))
        _MANUFACTURED["data"] = (A, B, C, Xs)
    return _MANUFACTURED["data"]


@pytest.mark.gpu
@pytest.mark.parametrize("path", ["fp64", "fp32", "bf16"])
def test_full_size_manufactured_solution_cd4096(path):
    A, B, C, Xs = _manufactured()
    c = ctx()
    say("manufactured solution", path)
    if path == "fp64":
        X, info = c.gmres(dev(A), dev(B), dev(C), m=30, tol=1e-11, max_cycles=3000)
        bar = 1e-8
    else:
        prec = tsylv.FP32 if path == "fp32" else tsylv.BF16
        X, info = c.gmres(dev(A), dev(B), dev(C), refine=1, prec=prec,
                          inner_m=32 if path == "fp32" else 28, inner_tol=1e-4, tol=1e-10,
                          max_outer=500)
        bar = 1e-7
    err = rel(host(X), Xs)
    say("  steps", info.steps, "outer", info.outer, "relres %.2e" % info.relres_true,
        "error vs X* %.3e" % err)
    assert info.status == 0, info.as_dict()
    assert err <= bar, (err, bar)


_FP64_8192 = {}


def _fp64_solution_8192(c, Ad, Bd, Cd):
    if "X" not in _FP64_8192:
        say("FP64 tGMRES(40) at 8192/128/64 to 1e-10")
        X, info = c.gmres(Ad, Bd, Cd, m=40, tol=1e-10, max_cycles=3000)
        say("  steps", info.steps, "cycles", info.cycles, "relres %.2e" % info.relres_true,
            "%.1f s" % info.seconds)
        assert info.status == 0, info.as_dict()
        _FP64_8192["X"] = host(X)
    return _FP64_8192["X"]


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [tsylv.BF16, tsylv.FP32])
def test_full_size_refined_cd8192(prec):
    """n = 8192 (128 x 64 grid), s = 128, p = 64: FP64 refinement around
    tGMRES(40) cycles with BF16 / FP32 slice products, inner tol 1e-4, to
    true relres 1e-8 -- the mixed-precision configuration at full size.
    Checked by the true residual recomputed by the FP64 tsylv_apply (pinned
    element-wise above), 48 sampled residual entries C - M(X) from the
    oracle's per-entry circulant sums, and, with both solved to 1e-10, the
    distance to the FP64 solution."""
    A, B, C = workload("cd_8192")
    c = ctx(arena_gb=ARENA_GB["cd_8192"])
    say("full size refined", prec, "8192/128/64")
    Ad, Bd, Cd = dev(A), dev(B), dev(C)
    X, info = c.gmres(Ad, Bd, Cd, refine=1, prec=prec, inner_m=40, inner_tol=1e-4, tol=1e-8,
                      max_outer=300)
    say("  outer", info.outer, "steps", info.steps, "relres", info.relres_true, "s",
        info.seconds)
    assert info.status == 0, info.as_dict()
    assert info.relres_true <= 1e-8
    MX = host(c.apply(Ad, Bd, X))
    R = C - MX
    assert np.linalg.norm(R) / np.linalg.norm(C) <= 1.05e-8
    Xh = host(X)
    rng = np.random.default_rng(5)
    n, s, p = C.shape
    idx = [(int(rng.integers(n)), int(rng.integers(s)), int(rng.integers(p))) for _ in range(48)]
    Ro = np.array([C[i, j, k] for i, j, k in idx]) - tp.sylv_op_entries(A, B, Xh, idx)
    Rg = np.array([R[i, j, k] for i, j, k in idx])
    scale = np.abs(A).max() * np.abs(Xh).max() * (n + s) * p * 64 * EPS
    assert np.abs(Ro - Rg).max() <= scale
    del MX, R
    # solution parity with the FP64 path, both to 1e-10
    X10, i10 = c.gmres(Ad, Bd, Cd, refine=1, prec=prec, inner_m=40, inner_tol=1e-4, tol=1e-10,
                       max_outer=500)
    assert i10.status == 0, i10.as_dict()
    X64 = _fp64_solution_8192(c, Ad, Bd, Cd)
    err = rel(host(X10), X64)
    say("  refined (1e-10) vs FP64 (1e-10): %.3e; at 1e-8: %.3e" % (err, rel(Xh, X64)))
    assert err <= 1e-7, err
    del Ad, Bd, Cd, X, X10
