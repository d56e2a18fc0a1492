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
    within each tGMRES cycle.
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
