"""GPU parity of tsylv_tba (TBAS(m), Algorithm 8) against the oracle.

Bars (FP64):
  * one restart cycle: the Galerkin solution over the block Krylov space of
    A and R0 is unique, so the GPU iterate (block CGS2, shifted CholQR3, per-slice
    Bartels-Stewart) equals the oracle's (block MGS, tubal MGS, spatial
    t-Bartels-Stewart) to ~1e-9 relative, and so do the true residual and
    the residual estimate of the proposition of section 5.2;
  * converged solutions within 1e-8 of the Kronecker / t-BS solution;
  * a right-hand side with a non-invertible tube makes Normalization break
    down in both (oracle: Breakdown, GPU: TSYLV_EBREAKDOWN).
"""

import numpy as np
import pytest

from oracle import krylov as kr
from oracle import kron, tbs
from paper_2405_09233_amd import workloads, tsylv
from gpu_util import ctx, dev, host, say, rel


def gpu_tba(A, B, C, **kw):
    X, info = ctx().tba(dev(A), dev(B), dev(C), raise_on_error=False, **kw)
    return host(X), info


@pytest.mark.gpu
@pytest.mark.parametrize("n,s,p,m", [(24, 3, 3, 3), (20, 2, 4, 4), (18, 1, 2, 5), (30, 4, 1, 3),
                                     (16, 2, 5, 2), (40, 5, 6, 3)])
def test_one_cycle_matches_oracle(n, s, p, m):
    say("tba one cycle", n, s, p, m)
    A, B, C = workloads.dense_shifted(n, s, p, seed=n * 3 + p)
    X, info = gpu_tba(A, B, C, m=m, tol=1e-300, max_cycles=1)
    assert info.status == 1 and info.cycles == 1, info.as_dict()
    Xo, io = kr.tbas(A, B, C, m=m, tol=1e-300, max_cycles=1)
    assert rel(X, Xo) <= 1e-9
    assert info.relres_true == pytest.approx(io["relres_true"], rel=1e-7)
    assert info.relres_est == pytest.approx(io["est_hist"][0], rel=1e-6, abs=1e-14)


@pytest.mark.gpu
@pytest.mark.parametrize("n,s,p,m", [(24, 3, 3, 3), (30, 2, 2, 4), (21, 1, 4, 6), (36, 4, 5, 2)])
def test_converged_vs_exact(n, s, p, m):
    say("tba converged", n, s, p, m)
    A, B, C = workloads.dense_shifted(n, s, p, seed=5 * n + s)
    X, info = gpu_tba(A, B, C, m=m, tol=1e-11, max_cycles=300)
    assert info.status == 0, info.as_dict()
    assert info.relres_true <= 1e-11
    Xk = kron.kron_solve(A, B, C) if n * s * p <= 700 else tbs.t_bartels_stewart(A, B, C)
    assert rel(X, Xk) <= 1e-8
    Xo, io = kr.tbas(A, B, C, m=m, tol=1e-11, max_cycles=300)
    assert abs(info.cycles - io["cycles"]) <= 1


@pytest.mark.gpu
def test_convection_diffusion_vs_tbs():
    say("tba cd 8x8, s=4, p=4")
    A, B, C = workloads.convection_diffusion(8, 8, 4, 4, seed=2)
    X, info = gpu_tba(A, B, C, m=6, tol=1e-11, max_cycles=200)
    assert info.status == 0, info.as_dict()
    assert rel(X, tbs.t_bartels_stewart(A, B, C)) <= 1e-8


@pytest.mark.gpu
def test_restart_length_clamped_to_space():
    # (m + 1) s > n: the block Krylov space of a slice cannot exceed C^n
    say("tba clamp")
    A, B, C = workloads.dense_shifted(12, 4, 3, seed=4)
    X, info = gpu_tba(A, B, C, m=10, tol=1e-11, max_cycles=200)
    assert info.status == 0, info.as_dict()
    assert rel(X, kron.kron_solve(A, B, C)) <= 1e-8


@pytest.mark.gpu
def test_normalization_breakdown():
    say("tba breakdown")
    A, B, C = workloads.dense_shifted(10, 2, 4, seed=8)
    C = C.copy()
    C[:, 0, :] = C[:, 0, :1]       # tube of column 0 constant: zero Fourier coefficients k > 0
    with pytest.raises(kr.Breakdown):
        kr.tbas(A, B, C, m=2, tol=1e-10, max_cycles=5)
    X, info = gpu_tba(A, B, C, m=2, tol=1e-10, max_cycles=5)
    assert info.status == -3


@pytest.mark.gpu
def test_invalid_sizes():
    A, B, C = workloads.dense_shifted(5, 3, 2, seed=1)   # n < 2 s
    X, info = gpu_tba(A, B, C, m=2)
    assert info.status == -1


@pytest.mark.gpu
@pytest.mark.parametrize("m", [4, 8])
def test_medium_convection_diffusion(m):
    """n = 1024 (32 x 32 grid), s = 16, p = 8 (the Gram products take the
    split-K path), TBAS(m) to 1e-9; checked by the true residual (recomputed
    by tsylv_apply) and against FP64 tGMRES."""
    say("tba medium 1024/16/8 m", m)
    A, B, C = workloads.convection_diffusion(32, 32, 16, 8, seed=0)
    c = ctx()
    Ad, Bd, Cd = dev(A), dev(B), dev(C)
    X, info = c.tba(Ad, Bd, Cd, m=m, tol=1e-9, max_cycles=400)
    say("cycles", info.cycles, "relres", info.relres_true, "s", info.seconds)
    assert info.status == 0, info.as_dict()
    R = C - host(c.apply(Ad, Bd, X))
    assert np.linalg.norm(R) / np.linalg.norm(C) <= 1.05e-9
    Xg, ig = c.gmres(Ad, Bd, Cd, m=30, tol=1e-11)
    assert ig.status == 0
    assert rel(host(X), host(Xg)) <= 1e-6


@pytest.mark.gpu
def test_medium_dense_vs_tbs():
    """n = 512, s = 16, p = 4 dense operator: converged TBAS(4) against the
    oracle's t-Bartels-Stewart solution."""
    say("tba dense 512/16/4")
    A, B, C = workloads.dense_shifted(512, 16, 4, seed=3)
    X, info = gpu_tba(A, B, C, m=4, tol=1e-11, max_cycles=100)
    assert info.status == 0, info.as_dict()
    assert rel(X, tbs.t_bartels_stewart(A, B, C)) <= 1e-8


@pytest.mark.gpu
@pytest.mark.parametrize("n,s,p,m", [(24, 3, 3, 3), (40, 5, 6, 3), (200, 16, 4, 4), (260, 64, 3, 3),
                                     (140, 65, 2, 1), (96, 1, 5, 7), (300, 40, 2, 3),
                                     (200, 20, 3, 5)])
def test_device_and_host_projected_solves_agree(n, s, p, m, monkeypatch):
    """The projected equation of a TBAS cycle solved on the device (Bhat_k
    diagonalised, p_h s shifted block-Hessenberg systems) and on the host
    (Bartels-Stewart with the Schur form of Bhat_k): the same cycle iterate.
    s = 40 and 20 leave padding in the device kernels' 16-wide blocks; s = 65
    exceeds the device kernel's block limit and takes the host path in both
    runs."""
    say("tba projected device vs host", n, s, p, m)
    A, B, C = workloads.dense_shifted(n, s, p, seed=n + s)
    Xd, idv = gpu_tba(A, B, C, m=m, tol=1e-300, max_cycles=1)
    monkeypatch.setenv("TSYLV_TBA_HOST_PROJECTED", "1")
    Xh, ihs = gpu_tba(A, B, C, m=m, tol=1e-300, max_cycles=1)
    assert idv.status == 1 and ihs.status == 1, (idv.as_dict(), ihs.as_dict())
    assert rel(Xd, Xh) <= 1e-10
    assert idv.relres_est == pytest.approx(ihs.relres_est, rel=1e-8, abs=1e-15)
    assert idv.relres_true == pytest.approx(ihs.relres_true, rel=1e-8)


@pytest.mark.gpu
def test_ex3_ordering_matches_the_oracle():
    """The paper's convection-diffusion experiment family (section 6; n =
    1000, s = 3, p = 2, mu = 1e-3 -- the paper does not give mu), against the
    oracle's counts in tests/golden/ex3_counts.json (written by
    make_ex3_counts.py from the oracle alone): TBAS(10) follows the
    oracle's TBAS(10) cycle by cycle over the first 100 cycles (the
    residual estimate of the proposition of section 5.2, within 1e-6
    relative to cycle 50 and 1e-3 to cycle 100, while the residual grows to
    about 2e3) and then reaches 1e-6 (the count itself is decided at the
    rounding level: the oracle's moves between 312 and 467 cycles under
    one-ulp changes of C, so it is not compared), tGMRES(10) stalls where
    the oracle's does (same residual after the same number of cycles), and
    tFOM(10) does worse than tGMRES(10) (the oracle's diverges or meets a
    singular projected system) -- the ordering TBAS < tGMRES < tFOM of the
    experiment's table, whose counts are not reproducible (mu and the rand
    stream are missing)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "ex3_counts.json")) as f:
        gold = json.load(f)
    say("ex3 1000/3/2 vs oracle counts")
    A, B, C = workloads.ex3(1000, 3, 2, mu=1e-3)
    c = ctx()
    Ad, Bd, Cd = dev(A), dev(B), dev(C)
    import ctypes
    hist = (ctypes.c_double * 1000)()
    o = tsylv.default_opts(tsylv.TBA, m=10, tol=1e-6, max_cycles=1000)
    o.res_hist = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
    o.res_hist_cap = 1000
    X, it = c.tba(Ad, Bd, Cd, opts=o)
    say("  TBAS cycles", it.cycles, "oracle", gold["tbas"]["cycles"], "perturbed oracle",
        gold["tbas"]["perturbed"]["cycles"])
    assert it.status == 0 and it.relres_true <= 1e-6, it.as_dict()
    assert gold["tbas"]["converged"] and all(gold["tbas"]["perturbed"]["converged"])
    ref = np.array(gold["tbas"]["est_hist_first"])
    got = np.array(hist[:min(it.res_hist_len, len(ref))])
    assert len(got) == len(ref), (len(got), len(ref))
    dev_ = np.abs(got / ref - 1.0)
    say("  estimate history vs oracle: max rel diff to cycle 50 %.2e, to 100 %.2e"
        % (dev_[:50].max(), dev_.max()))
    assert dev_[:50].max() <= 1e-6 and dev_.max() <= 1e-3
    R = C - host(c.apply(Ad, Bd, X))
    assert np.linalg.norm(R) / np.linalg.norm(C) <= 1.05e-6
    ng = gold["tgmres"]["cycles"]
    _, ig = c.gmres(Ad, Bd, Cd, m=10, tol=1e-6, max_cycles=ng, raise_on_error=False)
    say("  tGMRES relres after", ng, "cycles", ig.relres_true, "oracle",
        gold["tgmres"]["relres_true"])
    assert not gold["tgmres"]["converged"] and ig.status == 1
    assert ig.relres_true == pytest.approx(gold["tgmres"]["relres_true"], rel=1e-2)
    assert ng < it.cycles or ig.relres_true > 0.5  # stalled, far from TBAS's 1e-6
    nf = 20
    _, iff = c.fom(Ad, Bd, Cd, m=10, tol=1e-6, max_cycles=nf, raise_on_error=False)
    say("  tFOM status", iff.status, "relres", iff.relres_true, "oracle", gold["tfom"])
    if "singular" in gold["tfom"]:
        assert iff.status == -4 or iff.relres_true > ig.relres_true
    else:
        assert not gold["tfom"]["converged"]
        assert iff.status < 0 or iff.relres_true > ig.relres_true