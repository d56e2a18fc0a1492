"""Small instances solved whole in one workgroup (tGMRES / tFOM, Algorithm 3).

Plain FP64 tGMRES and tFOM of instances whose n s p, operator planes and
two basis vectors fit one workgroup's LDS run as a single launch
(kernels_tiny.hip); TSYLV_KRYLOV_TINY=0 sends them through the multi-launch
driver instead.  Bars:
  * unrestarted solves of the 8 x 8 x 4 dense instance: the Kronecker
    solution to 1e-10 (the same bar as the multi-launch path);
  * one cycle with no early exit: the oracle's iterate to 1e-10 (the
    minimiser / Galerkin solution over the same Krylov space), including a
    restart length whose basis spills from LDS to global memory;
  * converged restarted solves: the multi-launch path's solution to 1e-9,
    step counts within one cycle of each other;
  * a happy breakdown (the Krylov space exhausts the n s p unknowns before
    m steps) gives the exact solution;
  * the residual-estimate history has one entry per step and decreases
    within each tGMRES cycle;
  * tsylv_gmres_batch solves such instances in one launch, one workgroup
    each: every result bitwise the single solve's (the same kernel), alone
    or in a batch, next to instances that take the lockstep executor.
"""

import time

import numpy as np
import pytest

from oracle import kron
from oracle import krylov as kr
from paper_2405_09233_amd import workloads, tsylv
from gpu_util import ctx, dev, host, say, rel


def solve(method, A, B, C, **kw):
    c = ctx()
    fn = c.gmres if method == "gmres" else c.fom
    X, info = fn(dev(A), dev(B), dev(C), **kw)
    return host(X), info


@pytest.mark.gpu
@pytest.mark.parametrize("method", ["gmres", "fom"])
def test_tiny_unrestarted_matches_kronecker_and_multi_launch(method, monkeypatch):
    say("tiny unrestarted 8x8x4", method)
    A, B, C = workloads.tiny_dense(0)
    X, info = solve(method, A, B, C, m=C.size, tol=1e-12, max_cycles=2)
    assert info.status == 0, info.as_dict()
    assert info.relres_true <= 1e-12
    Xk = kron.kron_solve(A, B, C)
    assert rel(X, Xk) <= 1e-10
    monkeypatch.setenv("TSYLV_KRYLOV_TINY", "0")
    X2, info2 = solve(method, A, B, C, m=C.size, tol=1e-12, max_cycles=2)
    assert info2.status == 0
    assert abs(info.steps - info2.steps) <= 1
    assert info.cycles == info2.cycles
    assert rel(X, X2) <= 1e-10


@pytest.mark.gpu
@pytest.mark.parametrize("method", ["gmres", "fom"])
@pytest.mark.parametrize("n,s,p,m", [(8, 6, 4, 12), (12, 5, 3, 9), (9, 4, 1, 6),
                                     (10, 3, 2, 8), (16, 5, 6, 14),
                                     (40, 6, 5, 30)])  # 9 of 31 basis slots in LDS
def test_one_cycle_matches_oracle(method, n, s, p, m):
    say("tiny one cycle", method, n, s, p, m)
    A, B, C = workloads.dense_shifted(n, s, p, seed=7 * n + p)
    X, info = solve(method, A, B, C, m=m, tol=1e-300, max_cycles=1)
    assert info.status == 1 and info.cycles == 1 and info.steps == m, info.as_dict()
    Xo, io = kr.tkrylov_solve(A, B, C, method=method, m=m, tol=1e-300, max_cycles=1,
                              early_exit=False)
    assert rel(X, Xo) <= 1e-10
    assert info.relres_true == pytest.approx(io["relres_true"], rel=1e-8)


@pytest.mark.gpu
@pytest.mark.parametrize("method", ["gmres", "fom"])
@pytest.mark.parametrize("n,s,p,m", [(20, 4, 3, 5), (12, 7, 5, 6), (30, 3, 4, 10)])
def test_restarted_matches_multi_launch(method, n, s, p, m, monkeypatch):
    say("tiny restarted vs multi-launch", method, n, s, p, m)
    A, B, C = workloads.dense_shifted(n, s, p, seed=11 * s + n)
    X, info = solve(method, A, B, C, m=m, tol=1e-11, max_cycles=300)
    assert info.status == 0, info.as_dict()
    assert info.relres_true <= 1e-11
    monkeypatch.setenv("TSYLV_KRYLOV_TINY", "0")
    X2, info2 = solve(method, A, B, C, m=m, tol=1e-11, max_cycles=300)
    assert info2.status == 0
    assert rel(X, X2) <= 1e-9
    assert abs(info.steps - info2.steps) <= m
    Xk = kron.kron_solve(A, B, C)
    assert rel(X, Xk) <= 1e-8


@pytest.mark.gpu
@pytest.mark.parametrize("method", ["gmres", "fom"])
def test_happy_breakdown_gives_exact_solution(method):
    # n s p = 12 unknowns: the Krylov space is exhausted within 12 steps
    say("tiny breakdown", method)
    A, B, C = workloads.dense_shifted(3, 2, 2, seed=4)
    X, info = solve(method, A, B, C, m=20, tol=1e-14, max_cycles=3)
    assert info.status == 0, info.as_dict()
    assert info.steps <= 12 and info.cycles == 1
    assert rel(X, kron.kron_solve(A, B, C)) <= 1e-11


@pytest.mark.gpu
def test_history_and_zero_rhs():
    say("tiny history / zero rhs")
    A, B, C = workloads.dense_shifted(10, 4, 3, seed=2)
    hist = (tsylv.ctypes.c_double * 64)()
    o = tsylv.default_opts(tsylv.GMRES, m=6, tol=1e-11, max_cycles=100)
    o.res_hist = tsylv.ctypes.cast(hist, tsylv.ctypes.POINTER(tsylv.ctypes.c_double))
    o.res_hist_cap = 64
    X, info = ctx().gmres(dev(A), dev(B), dev(C), opts=o)
    assert info.status == 0
    h = np.array(hist[:info.res_hist_len])
    assert info.res_hist_len == min(info.steps, 64)
    for c0 in range(0, len(h), 6):
        assert np.all(np.diff(h[c0:c0 + 6]) <= 1e-14)
    if info.steps <= 64:
        assert h[len(h) - 1] == pytest.approx(info.relres_est, rel=1e-12)
    Xz, iz = solve("gmres", A, B, np.zeros_like(C))
    assert iz.status == 0 and iz.cycles == 0 and np.all(Xz == 0) and iz.relres_true == 0.0


@pytest.mark.gpu
def test_tiny_latency_below_multi_launch(monkeypatch):
    """The single-launch solve of the 8 x 8 x 4 instance (29 Arnoldi steps)
    is several times faster than the multi-launch driver's."""
    A, B, C = workloads.tiny_dense(0)
    c = ctx()
    Ad, Bd, Cd = dev(A), dev(B), dev(C)

    def p50(reps=30):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            c.gmres(Ad, Bd, Cd, m=C.size, tol=1e-12, max_cycles=2)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    p50()
    t_tiny = p50()
    monkeypatch.setenv("TSYLV_KRYLOV_TINY", "0")
    p50(5)
    t_multi = p50()
    say("8x8x4 unrestarted tGMRES p50: one workgroup %.1f us, multi-launch %.1f us"
        % (t_tiny * 1e6, t_multi * 1e6))
    assert t_tiny < 0.5 * t_multi


def _items(shapes, seed0):
    import torch
    data, items = [], []
    for k, (n, s, p) in enumerate(shapes):
        A, B, C = workloads.dense_shifted(n, s, p, seed=seed0 + k)
        Cd = dev(C)
        data.append((A, B, C))
        items.append((dev(A), dev(B), Cd, torch.zeros_like(Cd)))
    return data, items


@pytest.mark.gpu
def test_batch_of_small_instances_in_one_launch():
    import torch
    # ragged sizes, p odd and even, and one whose basis spills to global memory
    shapes = [(8, 6, 4), (12, 5, 3), (9, 4, 1), (10, 3, 2), (16, 5, 6), (40, 6, 5), (20, 7, 4)]
    say("tiny batch", shapes)
    c = ctx()
    data, items = _items(shapes, 1200)
    infos = c.gmres_batch(items, m=30, tol=1e-11, max_cycles=100)
    for k, ((A, B, C), (Ad, Bd, Cd, X), info) in enumerate(zip(data, items, infos)):
        assert info.status == 0, (k, info.as_dict())
        assert info.relres_true <= 1e-11
        assert rel(host(X), kron.kron_solve(A, B, C)) <= 1e-8
        Xs, i1 = c.gmres(Ad, Bd, Cd, m=30, tol=1e-11, max_cycles=100)
        assert torch.equal(X, Xs), k
        assert (i1.steps, i1.cycles, i1.relres_true) == (info.steps, info.cycles,
                                                         info.relres_true)
    # alone as a batch of one
    Ad, Bd, Cd, X = items[5]
    Xa = torch.zeros_like(Cd)
    ia = c.gmres_batch([(Ad, Bd, Cd, Xa)], m=30, tol=1e-11, max_cycles=100)[0]
    assert torch.equal(Xa, X) and ia.steps == infos[5].steps


@pytest.mark.gpu
def test_batch_mixes_single_workgroup_and_lockstep(monkeypatch):
    import torch
    shapes = [(8, 6, 4), (200, 16, 8), (14, 9, 3), (128, 12, 5)]
    say("tiny + lockstep batch", shapes)
    c = ctx()
    data, items = _items(shapes, 1300)
    infos = c.gmres_batch(items, m=20, tol=1e-11, max_cycles=200)
    assert all(i.status == 0 for i in infos), [i.as_dict() for i in infos]
    for (A, B, C), (Ad, Bd, Cd, X), info in zip(data, items, infos):
        assert info.relres_true <= 1e-11
        Xs, _ = c.gmres(Ad, Bd, Cd, m=20, tol=1e-11, max_cycles=200)
        assert rel(host(X), host(Xs)) <= 1e-8
    for k in (0, 2):  # the small ones: bitwise their single solves
        Ad, Bd, Cd, X = items[k]
        Xs, _ = c.gmres(Ad, Bd, Cd, m=20, tol=1e-11, max_cycles=200)
        assert torch.equal(X, Xs), k
    # per-instance stopping and X0, as in the lockstep executor
    for it in items:
        it[3].zero_()
    i2 = c.gmres_batch(items, m=2, tol=1e-12, max_cycles=1, raise_on_error=False)
    assert all(i.status == 1 and i.cycles == 1 and i.steps == 2 for i in i2)
    o = tsylv.default_opts(tsylv.GMRES, m=30, tol=1e-11, max_cycles=100)
    o.x0_given = 1
    i3 = c.gmres_batch(items, opts=o)
    assert all(i.status == 0 for i in i3)
    for (A, B, C), (_, _, _, X) in zip(data, items):
        if A.shape[0] <= 16:
            assert rel(host(X), kron.kron_solve(A, B, C)) <= 1e-8
