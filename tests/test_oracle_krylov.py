"""Pins of the oracle's Kronecker solve, tArnoldi, tGMRES, tFOM, Tubal-QR,
TBA and TBAS against facts independent of the oracle: numpy/scipy library
routines on the equivalent linear system (lstsq, QR of Krylov matrices,
scipy's GMRES, solve_sylvester per Fourier slice via numpy's FFT), the
propositions of sections 3 and 5, and hand-computed values."""

import json
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg

from oracle import tproduct as tp
from oracle import krylov as kr
from oracle import kron
from paper_2405_09233_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_problem(n=5, s=3, p=3, seed=0):
    return workloads.dense_shifted(n, s, p, seed=seed)


def fft_slice_solution(A, B, C):
    """Per Fourier slice, scipy's Sylvester solver (a library routine):
    Ahat_k X - X Bhat_k = Chat_k, back with numpy's inverse FFT."""
    Ah, Bh, Ch = (np.fft.fft(T, axis=2) for T in (A, B, C))
    Xh = np.zeros(Ch.shape, dtype=complex)
    for k in range(A.shape[2]):
        Xh[:, :, k] = scipy.linalg.solve_sylvester(Ah[:, :, k], -Bh[:, :, k], Ch[:, :, k])
    return np.real(np.fft.ifft(Xh, axis=2))


# ---------------------------------------------------------------- Kronecker

@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 8])
def test_kron_operator_matches_M(p):
    A, B, C = small_problem(4, 3, p, seed=p)
    X = np.random.default_rng(1).standard_normal(C.shape)
    K = kron.kron_matrix(A, B)
    lhs = K @ tp.bcirc(X).reshape(-1, order="F")
    rhs = tp.bcirc(tp.sylv_op(A, B, X)).reshape(-1, order="F")
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 8])
def test_kron_solve_vs_fft_sylvester(p):
    A, B, C = small_problem(4, 3, p, seed=10 + p)
    X, Z = kron.kron_solve(A, B, C, return_Z=True)
    np.testing.assert_allclose(Z, tp.bcirc(X), atol=1e-11)       # block circulant
    np.testing.assert_allclose(X, fft_slice_solution(A, B, C), atol=1e-11)
    assert tp.fnorm(C - tp.sylv_op(A, B, X)) <= 1e-12 * tp.fnorm(C)


def test_kron_tiny_dense_workload():
    A, B, C = workloads.tiny_dense(0)
    X = kron.kron_solve(A, B, C)
    np.testing.assert_allclose(X, fft_slice_solution(A, B, C), atol=1e-12)


def test_golden_tube_sylvester():
    with open(os.path.join(GOLDEN, "sylvester_hand.json")) as f:
        g = json.load(f)
    for c in g["sylvester_tubes"]:
        A = np.array(c["a"], float).reshape(1, 1, -1)
        B = np.array(c["b"], float).reshape(1, 1, -1)
        C = np.array(c["c"], float).reshape(1, 1, -1)
        np.testing.assert_allclose(kron.kron_solve(A, B, C).ravel(), c["x"], atol=1e-15)
        X, info = kr.tgmres(A, B, C, m=2, tol=1e-14, max_cycles=3)
        np.testing.assert_allclose(X.ravel(), c["x"], atol=1e-14)
        X, info = kr.tfom(A, B, C, m=2, tol=1e-14, max_cycles=3)
        np.testing.assert_allclose(X.ravel(), c["x"], atol=1e-14)
    for c in g["normalization_tubes"]:
        W = np.array(c["w"], float).reshape(1, 1, -1)
        U, a = kr.normalization(W)
        np.testing.assert_allclose(a, c["a"], atol=1e-14)
        np.testing.assert_allclose(U.ravel(), c["u"], atol=1e-14)


# ---------------------------------------------------------------- tArnoldi

def test_tarnoldi_relations_and_krylov_qr():
    A, B, C = small_problem(5, 3, 4, seed=3)
    Mop = lambda V: tp.sylv_op(A, B, V)
    m = 5
    Vs, H, Ws, k = kr.tarnoldi(Mop, C, m)
    assert k == m and len(Vs) == m + 1
    G = tp.tdiamond(Vs, Vs)
    np.testing.assert_allclose(G, np.eye(m + 1), atol=1e-12)          # V^T <> V = I
    for j in range(m):                                                 # W_m = V_{m+1} (*) Htilde
        np.testing.assert_allclose(Ws[j], kr.combine(Vs, H[:, j]), atol=1e-10)
    np.testing.assert_allclose(np.tril(H, -2), 0, atol=0)              # Hessenberg
    np.testing.assert_allclose(tp.tdiamond(Vs[:m], Ws), H[:m, :], atol=1e-10)
    # Independent: the basis is the Q factor (positive diagonal) of the
    # Krylov matrix [r, Mr, ..., M^m r] on the vectorised system.
    Mx = kron.sylv_matrix(A, B)
    r = C.reshape(-1, order="F")
    K = np.zeros((r.size, m + 1))
    K[:, 0] = r
    for j in range(1, m + 1):
        K[:, j] = Mx @ K[:, j - 1]
    Q, R = np.linalg.qr(K)
    Q = Q * np.sign(np.diag(R))
    for j in range(m + 1):
        np.testing.assert_allclose(Vs[j].reshape(-1, order="F"), Q[:, j], atol=1e-8)


def test_tarnoldi_happy_breakdown():
    # With B = 0 and A = 3 I (identity tensor plus 2 I on slice 1), M(X) = 3 X:
    # every C spans an invariant subspace, so tArnoldi stops after one step
    # with h_{2,1} = 0 and tGMRES returns C / 3 exactly.
    p = 3
    A = tp.identity(4, p).copy()
    A[:, :, 0] += 2.0 * np.eye(4)
    B = np.zeros((2, 2, p))
    C = np.random.default_rng(0).standard_normal((4, 2, p))
    Mop = lambda V: tp.sylv_op(A, B, V)
    Vs, H, Ws, k = kr.tarnoldi(Mop, C, 4)
    assert k == 1 and H.shape == (2, 1) and H[1, 0] == 0.0
    X, info = kr.tgmres(A, B, C, m=4, tol=1e-14)
    np.testing.assert_allclose(X, C / 3.0, atol=1e-14)


# ---------------------------------------------------------------- tGMRES

def test_tgmres_unrestarted_reaches_kron_solution():
    A, B, C = workloads.tiny_dense(0)
    N = C.size
    X, info = kr.tgmres(A, B, C, m=N, tol=1e-12, max_cycles=1)
    Xk = kron.kron_solve(A, B, C)
    assert info["converged"] and info["cycles"] == 1
    assert np.linalg.norm(X - Xk) <= 1e-10 * np.linalg.norm(Xk)
    est = np.array(info["est_hist"])
    assert np.all(np.diff(est) <= 1e-15)                   # monotone within the cycle


def test_tgmres_gamma_equals_true_residual_and_lstsq():
    A, B, C = small_problem(5, 3, 3, seed=7)
    Mop = lambda V: tp.sylv_op(A, B, V)
    beta = tp.fnorm(C)
    Vs, H, Ws, k = kr.tarnoldi(Mop, C, 8)
    Wmat = np.stack([w.reshape(-1) for w in Ws], axis=1)
    for j in range(1, k + 1):
        y, gam = kr.givens_ls(H[:j + 1, :j], beta)
        Xj = kr.combine(Vs, y)
        true = tp.fnorm(C - Mop(Xj))
        assert gam == pytest.approx(true, rel=1e-9, abs=1e-13)
        # lstsq on the explicit images M(V_i) (library routine)
        yl, *_ = np.linalg.lstsq(Wmat[:, :j], C.reshape(-1), rcond=None)
        np.testing.assert_allclose(y, yl, rtol=1e-8, atol=1e-10)


def test_tgmres_one_cycle_equals_scipy_gmres():
    A, B, C = small_problem(6, 4, 3, seed=21)
    m = 6
    X, info = kr.tgmres(A, B, C, m=m, tol=1e-30, max_cycles=1, early_exit=False)
    Mx = kron.sylv_matrix(A, B)
    b = C.reshape(-1, order="F")
    x, _ = scipy.sparse.linalg.gmres(Mx, b, x0=np.zeros_like(b), rtol=1e-30, atol=0,
                                     restart=m, maxiter=1)
    np.testing.assert_allclose(X.reshape(-1, order="F"), x, rtol=1e-9, atol=1e-11)


def test_tgmres_restarted_monotone_and_converges():
    A, B, C = small_problem(6, 4, 4, seed=5)
    X, info = kr.tgmres(A, B, C, m=4, tol=1e-11, max_cycles=200)
    assert info["converged"]
    th = np.array(info["true_hist"])
    assert np.all(np.diff(th) <= 1e-14)
    Xk = kron.kron_solve(A, B, C)
    assert np.linalg.norm(X - Xk) <= 1e-9 * np.linalg.norm(Xk)


# ---------------------------------------------------------------- tFOM

def test_tfom_residual_formula_and_galerkin():
    A, B, C = small_problem(5, 3, 4, seed=9)
    Mop = lambda V: tp.sylv_op(A, B, V)
    beta = tp.fnorm(C)
    m = 6
    Vs, H, Ws, k = kr.tarnoldi(Mop, C, m)
    y = kr.fom_solve(H[:m, :m], beta)
    X = kr.combine(Vs, y)
    R = C - Mop(X)
    assert tp.fnorm(R) == pytest.approx(H[m, m - 1] * abs(y[-1]), rel=1e-8)
    np.testing.assert_allclose(tp.tdiamond(Vs[:m], [R]).ravel(), 0, atol=1e-10 * beta)
    # Independent Galerkin solution on the vectorised system
    Mx = kron.sylv_matrix(A, B)
    Vm = np.stack([v.reshape(-1, order="F") for v in Vs[:m]], axis=1)
    yg = np.linalg.solve(Vm.T @ Mx @ Vm, Vm.T @ C.reshape(-1, order="F"))
    np.testing.assert_allclose(y, yg, rtol=1e-8, atol=1e-10)


def test_tfom_converges_to_kron():
    A, B, C = small_problem(6, 4, 3, seed=8)
    X, info = kr.tfom(A, B, C, m=5, tol=1e-11, max_cycles=300)
    assert info["converged"]
    Xk = kron.kron_solve(A, B, C)
    assert np.linalg.norm(X - Xk) <= 1e-9 * np.linalg.norm(Xk)


# ---------------------------------------------------------------- Tubal-QR / TBA

@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_tubal_qr(p):
    Amat = np.random.default_rng(p).standard_normal((6, 3, p))
    Q, R = kr.tubal_qr(Amat)
    np.testing.assert_allclose(tp.tprod(Q, R), Amat, atol=1e-12)
    np.testing.assert_allclose(tp.tprod(tp.ttrans(Q), Q), tp.identity(3, p), atol=1e-12)
    for k in range(p):
        np.testing.assert_allclose(np.tril(R[:, :, k], -1), 0, atol=0)
    # Independent: in every Fourier slice, numpy's QR with the phases of the
    # diagonal of R made real positive.
    Ah, Qh = np.fft.fft(Amat, axis=2), np.fft.fft(Q, axis=2)
    Rh = np.fft.fft(R, axis=2)
    for k in range(p):
        q, r = np.linalg.qr(Ah[:, :, k])
        ph = np.diag(r) / np.abs(np.diag(r))
        q = q * ph
        r = np.conj(ph)[:, None] * r
        np.testing.assert_allclose(Qh[:, :, k], q, atol=1e-11)
        np.testing.assert_allclose(Rh[:, :, k], r, atol=1e-11)
        assert np.all(np.abs(np.imag(np.diag(Rh[:, :, k]))) < 1e-12)
        assert np.all(np.real(np.diag(Rh[:, :, k])) > 0)


def test_normalization_breakdown():
    W = np.zeros((3, 1, 2))
    W[:, 0, 0] = 1.0
    W[:, 0, 1] = 1.0           # Fourier slice k=1 is zero: a not invertible
    with pytest.raises(kr.Breakdown):
        kr.normalization(W)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_tba_relations_and_block_krylov(p):
    n, s, m = 12, 2, 3
    rng = np.random.default_rng(40 + p)
    A = rng.standard_normal((n, n, p))
    V = rng.standard_normal((n, s, p))
    Vb, Hbig, H0 = kr.tba(A, V, m)
    Vm = kr.block_cat(Vb[:m])
    Vm1 = kr.block_cat(Vb)
    Hm = Hbig[:m * s]
    AV = tp.tprod(A, Vm)
    np.testing.assert_allclose(AV, tp.tprod(Vm1, Hbig), atol=1e-10)                   # for1
    np.testing.assert_allclose(tp.tprod(tp.ttrans(Vm), AV), Hm, atol=1e-10)          # for2
    np.testing.assert_allclose(tp.tprod(tp.ttrans(Vm1), AV), Hbig, atol=1e-10)       # for3
    np.testing.assert_allclose(tp.tprod(tp.ttrans(Vm1), Vm1), tp.identity((m + 1) * s, p),
                               atol=1e-10)                                            # for4
    np.testing.assert_allclose(tp.tprod(Vb[0], H0), V, atol=1e-12)
    # Independent: per Fourier slice the basis is the Q factor (positive real
    # diagonal) of the block Krylov matrix [V, A V, ..., A^m V] (numpy QR).
    Ah, Vh, Bh = np.fft.fft(A, axis=2), np.fft.fft(V, axis=2), np.fft.fft(Vm1, axis=2)
    for k in range(p):
        blocks = [Vh[:, :, k]]
        for j in range(m):
            blocks.append(Ah[:, :, k] @ blocks[-1])
        q, r = np.linalg.qr(np.concatenate(blocks, axis=1))
        ph = np.diag(r) / np.abs(np.diag(r))
        np.testing.assert_allclose(Bh[:, :, k], q * ph, atol=1e-8)


def test_tbas_galerkin_estimate_and_solution():
    A, B, C = small_problem(8, 2, 3, seed=33)
    m = 2
    X1, info1 = kr.tbas(A, B, C, m=m, tol=1e-30, max_cycles=1)
    R = C - tp.sylv_op(A, B, X1)
    Vb, Hbig, H0 = kr.tba(A, C, m)
    Vm = kr.block_cat(Vb[:m])
    np.testing.assert_allclose(tp.tprod(tp.ttrans(Vm), R), 0, atol=1e-10)           # Galerkin
    assert info1["est_hist"][0] == pytest.approx(tp.fnorm(R) / tp.fnorm(C), rel=1e-7)
    X, info = kr.tbas(A, B, C, m=3, tol=1e-11, max_cycles=100)
    assert info["converged"]
    Xk = kron.kron_solve(A, B, C)
    assert np.linalg.norm(X - Xk) <= 1e-9 * np.linalg.norm(Xk)
