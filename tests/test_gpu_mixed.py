"""GPU parity of the mixed-precision path: FP32 and BF16 slice products
(through tsylv_apply's precision argument) and FP64 iterative refinement with
FP32 / BF16 inner tGMRES cycles (tsylv_gmres with refine = 1).

Bars:
  * apply in precision u (u = 2^-24 for FP32, 2^-8 for BF16 inputs with FP32
    accumulation): the operands of every slice product are rounded once
    (relative error <= u each) and the products accumulated in FP32 over
    K = n + s terms.  For random data the normwise relative error of Y is
    then about u (input rounding) plus 2^-24 sqrt(K) (accumulation); the test
    allows 4 u sqrt(K) for FP32 and 4 u for BF16, and elementwise the FP64
    bound with eps replaced by u.
  * refined solves: true FP64 relative residual <= tol, and the solution within
    1e-7 (relative) of the oracle's exact solution, the bar the refined mixed
    path is held to.
"""

import numpy as np
import pytest

from oracle import tproduct as tp
from oracle import kron, tbs
from paper_2405_09233_amd import workloads, tsylv
from gpu_util import ctx, dev, host, say, rel, workload

U32 = 2.0 ** -24
UBF = 2.0 ** -8


@pytest.mark.gpu
@pytest.mark.parametrize("prec,u", [(tsylv.FP32, U32), (tsylv.BF16, UBF)])
@pytest.mark.parametrize("n,s,p", [(8, 6, 4), (70, 5, 5), (130, 70, 7), (64, 20, 2), (33, 40, 1)])
def test_low_precision_apply(prec, u, n, s, p):
    say("apply prec", prec, n, s, p)
    rng = np.random.default_rng(n + 7 * s + p)
    A = np.asfortranarray(rng.standard_normal((n, n, p)))
    B = np.asfortranarray(rng.standard_normal((s, s, p)))
    X = np.asfortranarray(rng.standard_normal((n, s, p)))
    Y = host(ctx().apply(dev(A), dev(B), dev(X), prec=prec))
    ref = tp.sylv_op(A, B, X)
    allowed = 4 * u * (np.sqrt(n + s) if prec == tsylv.FP32 else 1.0)
    assert rel(Y, ref) <= allowed, (rel(Y, ref), allowed)
    bound = 64 * u * (n + s) * p * max(np.abs(A).max(), np.abs(B).max()) * np.abs(X).max()
    assert np.abs(Y - ref).max() <= bound


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [tsylv.FP32, tsylv.BF16])
@pytest.mark.parametrize("n,s,p", [(40, 6, 4), (64, 8, 3), (25, 3, 1), (30, 5, 6)])
def test_refined_solve_dense(prec, n, s, p):
    say("refined dense", prec, n, s, p)
    A, B, C = workloads.dense_shifted(n, s, p, seed=11 * n + p)
    X, info = ctx().gmres(dev(A), dev(B), dev(C), refine=1, prec=prec, inner_m=10,
                          inner_tol=1e-4, tol=1e-10, max_outer=200)
    assert info.status == 0, info.as_dict()
    assert info.relres_true <= 1e-10 and info.outer >= 1
    Xk = kron.kron_solve(A, B, C) if n * s * p <= 900 else tbs.t_bartels_stewart(A, B, C)
    assert rel(host(X), Xk) <= 1e-7


@pytest.mark.gpu
@pytest.mark.parametrize("basis", ["bf16", "fp32"])
@pytest.mark.parametrize("n,s,p,method", [(40, 6, 4, "gmres"), (300, 70, 5, "gmres"),
                                          (256, 64, 2, "gmres"), (90, 20, 3, "fom")])
def test_bf16_refined_basis_storage(basis, n, s, p, method, monkeypatch):
    """BF16-refined solves with the inner Krylov basis stored as tiled BF16
    vectors (the default) and as FP32 vectors: both reach the FP64 residual
    target and the oracle's solution within the refined bar.  The sizes
    cover tiled padding in rows and columns, none at all (n = 256, s = 64),
    two column tiles (s = 70) and a real-only spectrum (p = 2 has two real
    slices)."""
    monkeypatch.setenv("TSYLV_BF16_BASIS", basis)
    say("bf16 refined basis", basis, n, s, p, method)
    A, B, C = workloads.dense_shifted(n, s, p, seed=5 * n + s + p)
    solve = getattr(ctx(), method)
    X, info = solve(dev(A), dev(B), dev(C), refine=1, prec=tsylv.BF16, inner_m=20,
                    inner_tol=1e-4, tol=1e-10, max_outer=300)
    assert info.status == 0, info.as_dict()
    assert info.relres_true <= 1e-10 and info.outer >= 1
    assert rel(host(X), tbs.t_bartels_stewart(A, B, C)) <= 1e-7


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [tsylv.FP32, tsylv.BF16])
@pytest.mark.parametrize("method", ["gmres", "fom"])
@pytest.mark.parametrize("n,s,p,inner_m", [(120, 10, 5, 16), (6, 2, 2, 30), (40, 6, 4, 1)])
def test_device_and_host_driven_inner_cycles_agree(prec, method, n, s, p, inner_m, monkeypatch):
    """Refinement's inner cycles enqueued in chunks, with the delayed-CGS2
    round arithmetic on the device (always, and the default: after a cycle
    that ran all its rounds), against the same cycles stepped from the host:
    all reach the target and agree.  (6, 2, 2) has a Krylov
    space of dimension nsp = 24 < inner_m, so its cycles end on the estimate
    or on a breakdown inside the cycle; inner_m = 1 is the shortest cycle."""
    say("device vs host inner cycles", prec, method, n, s, p, inner_m)
    A, B, C = workloads.dense_shifted(n, s, p, seed=13 * n + p)
    out = {}
    for mode in ("2", "1", "0"):  # always / after a full cycle (default) / never
        monkeypatch.setenv("TSYLV_KRYLOV_DEVICE_CYCLE", mode)
        X, info = getattr(ctx(), method)(dev(A), dev(B), dev(C), refine=1, prec=prec,
                                         inner_m=inner_m, inner_tol=1e-4, tol=1e-10,
                                         max_outer=400)
        assert info.status == 0, (mode, info.as_dict())
        assert info.relres_true <= 1e-10
        out[mode] = (host(X), info.steps)
    assert rel(out["2"][0], out["0"][0]) <= 1e-8
    assert rel(out["1"][0], out["0"][0]) <= 1e-8
    Xk = tbs.t_bartels_stewart(A, B, C)
    assert rel(out["2"][0], Xk) <= 1e-7


@pytest.mark.gpu
def test_refined_fom_fp32():
    say("refined tFOM fp32")
    A, B, C = workloads.dense_shifted(36, 4, 4, seed=2)
    X, info = ctx().fom(dev(A), dev(B), dev(C), refine=1, prec=tsylv.FP32, inner_m=8,
                        tol=1e-10, max_outer=300)
    assert info.status == 0, info.as_dict()
    assert rel(host(X), kron.kron_solve(A, B, C)) <= 1e-7


@pytest.mark.gpu
def test_refined_convection_diffusion_fp32_vs_fp64():
    say("refined cd 8x8 fp32")
    A, B, C = workloads.convection_diffusion(8, 8, 8, 4, seed=3)
    c = ctx()
    X32, i32 = c.gmres(dev(A), dev(B), dev(C), refine=1, prec=tsylv.FP32, inner_m=20, tol=1e-10)
    X64, i64 = c.gmres(dev(A), dev(B), dev(C), m=20, tol=1e-10)
    assert i32.status == 0 and i64.status == 0
    Xt = tbs.t_bartels_stewart(A, B, C)
    assert rel(host(X32), Xt) <= 1e-7
    assert rel(host(X64), Xt) <= 1e-8


@pytest.mark.gpu
def test_refine_option_validation():
    A, B, C = workloads.dense_shifted(8, 3, 2, seed=1)
    c = ctx()
    with pytest.raises(tsylv.TsylvError):
        c.gmres(dev(A), dev(B), dev(C), refine=1, prec=tsylv.FP64)
    with pytest.raises(tsylv.TsylvError):
        c.gmres(dev(A), dev(B), dev(C), refine=0, prec=tsylv.FP32)


@pytest.mark.gpu
def test_full_size_refined_fp32_cd4096():
    """n = 4096, s = 64, p = 32 convection-diffusion, FP64 refinement around
    FP32 tGMRES(40) cycles, to true relres 1e-8 (benchmark configuration)."""
    say("full size refined fp32 4096/64/32")
    A, B, C = workload("cd_4096")
    c = ctx()
    Ad, Bd, Cd = dev(A), dev(B), dev(C)
    X, info = c.gmres(Ad, Bd, Cd, refine=1, prec=tsylv.FP32, inner_m=40, tol=1e-8)
    say("outer", info.outer, "steps", info.steps, "relres", info.relres_true, "s", info.seconds)
    assert info.status == 0, info.as_dict()
    R = host(Cd) - host(c.apply(Ad, Bd, X))
    assert np.linalg.norm(R) / np.linalg.norm(C) <= 1.05e-8
    # Solution parity with the FP64 path (itself pinned to the oracle): both
    # solved to 1e-10 so the kappa * relres error bound stays below 1e-7.
    X10, i10 = c.gmres(Ad, Bd, Cd, refine=1, prec=tsylv.FP32, inner_m=40, tol=1e-10)
    X64, i64 = c.gmres(Ad, Bd, Cd, m=30, tol=1e-10)
    assert i10.status == 0 and i64.status == 0
    assert rel(host(X10), host(X64)) <= 1e-7
