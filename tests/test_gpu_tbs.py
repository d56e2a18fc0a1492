"""GPU parity of tsylv_tbs, the t-Bartels-Stewart direct solve (section 4,
Algorithms 4 and 5), against the oracle.

Bars (FP64): the direct solution within 1e-9 (relative) of the oracle's
t-Bartels-Stewart / Kronecker solution and a true relative residual below
1e-11 on well-separated spectra -- a backward-stable direct method leaves
O(eps kappa); a slice whose spectra of Ahat and Bhat meet is reported as
TSYLV_ESINGULAR; sizes past 64 are rejected.
"""

import time

import numpy as np
import pytest

from oracle import kron, tbs
from paper_2405_09233_amd import workloads, tsylv
from gpu_util import ctx, dev, host, say, rel


def gpu_tbs(A, B, C, **kw):
    X, info = ctx().tbs(dev(A), dev(B), dev(C), raise_on_error=False, **kw)
    return host(X), info


@pytest.mark.gpu
def test_tiny_dense_matches_kronecker():
    say("tbs tiny dense 8x8x4")
    A, B, C = workloads.tiny_dense(seed=0)
    X, info = gpu_tbs(A, B, C)
    assert info.status == 0, info.as_dict()
    assert info.relres_true <= 1e-13
    assert rel(X, kron.kron_solve(A, B, C)) <= 1e-12


@pytest.mark.gpu
@pytest.mark.parametrize("n,s,p", [(1, 1, 1), (1, 5, 3), (7, 1, 4), (13, 9, 1), (20, 11, 2),
                                   (33, 17, 5), (64, 64, 3), (64, 3, 8), (5, 64, 6), (40, 40, 16),
                                   (48, 30, 33)])
def test_matches_oracle(n, s, p):
    say("tbs vs oracle", n, s, p)
    A, B, C = workloads.dense_shifted(n, s, p, seed=7 * n + 3 * s + p)
    X, info = gpu_tbs(A, B, C)
    assert info.status == 0, info.as_dict()
    assert info.relres_true <= 1e-11
    assert info.steps == 0 and info.cycles == 0
    assert rel(X, tbs.t_bartels_stewart(A, B, C)) <= 1e-9


@pytest.mark.gpu
def test_nonnormal_convection_diffusion_slices():
    """Strongly non-normal slices (convection-diffusion on a 6 x 8 grid, n =
    48) make the QR iteration work for its deflations."""
    say("tbs convection-diffusion 48 x 12 x 4")
    A, B, C = workloads.convection_diffusion(6, 8, 12, 4, seed=2)
    X, info = gpu_tbs(A, B, C)
    assert info.status == 0, info.as_dict()
    assert rel(X, tbs.t_bartels_stewart(A, B, C)) <= 1e-9


@pytest.mark.gpu
def test_shared_eigenvalue_is_singular():
    say("tbs singular")
    n, s, p = 6, 4, 3
    A = np.zeros((n, n, p), order="F")
    B = np.zeros((s, s, p), order="F")
    A[:, :, 0] = 2.0 * np.eye(n) + np.triu(np.ones((n, n)), 1)
    B[:, :, 0] = 2.0 * np.eye(s)
    C = np.asfortranarray(np.ones((n, s, p)))
    X, info = gpu_tbs(A, B, C)
    assert info.status == -4, info.as_dict()  # TSYLV_ESINGULAR


@pytest.mark.gpu
def test_size_limit():
    A, B, C = workloads.dense_shifted(65, 4, 2, seed=1)
    with pytest.raises(tsylv.TsylvError):
        ctx().tbs(dev(A), dev(B), dev(C))
    A, B, C = workloads.dense_shifted(8, 65, 2, seed=1)
    with pytest.raises(tsylv.TsylvError):
        ctx().tbs(dev(A), dev(B), dev(C))


@pytest.mark.gpu
def test_served_tbs_equals_synchronous():
    """TBS requests through the serving loop, mixed with tGMRES requests:
    each result is bitwise the synchronous one."""
    import torch
    say("tbs served")
    c = ctx()
    cases = [(8, 6, 4), (30, 12, 5), (64, 16, 2)]
    jobs = []
    for i, (n, s, p) in enumerate(cases):
        A, B, C = workloads.dense_shifted(n, s, p, seed=100 + i)
        Ad, Bd, Cd = dev(A), dev(B), dev(C)
        Xs, _ = c.tbs(Ad, Bd, Cd)
        Xa = torch.zeros_like(Cd)
        Xg = torch.zeros_like(Cd)
        ta = c.submit(Ad, Bd, Cd, Xa, method=tsylv.TBS)
        tg = c.submit(Ad, Bd, Cd, Xg, method=tsylv.GMRES, m=20, tol=1e-10)
        # the device inputs stay referenced until their requests are final
        jobs.append((Xs, Xa, ta, tg, (Ad, Bd, Cd, Xg)))
    deadline = time.time() + 60.0
    for Xs, Xa, ta, tg, _ in jobs:
        for t in (ta, tg):
            while True:
                st, info = c.poll(t)
                if st != 2:  # TSYLV_PENDING
                    break
                assert time.time() < deadline, "serving loop did not finish"
                time.sleep(0.001)
            assert st == 0, info.as_dict()
        assert np.array_equal(host(Xa), host(Xs))
