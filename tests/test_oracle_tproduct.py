"""Pins of the oracle's T-product algebra against facts that do not come from
the oracle itself: the definition fold(bcirc(A) unfold(B)), numpy's FFT,
the block-diagonalisation eq. (5), the algebraic laws of Def. 2.2 and hand
computed values (tests/golden)."""

import json
import os

import numpy as np
import pytest

from oracle import tproduct as tp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 8])
def test_tprod_matches_bcirc_definition(p):
    A = rand((4, 3, p), 1)
    B = rand((3, 5, p), 2)
    ref = tp.fold(tp.bcirc(A) @ tp.unfold(B), 4, 5, p)
    np.testing.assert_allclose(tp.tprod(A, B), ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 7, 8])
def test_tprod_matches_fft_algorithm(p):
    # Algorithm 1 with numpy's FFT (a library primitive, independent of the
    # oracle's circulant sums): facewise products in the Fourier domain.
    A = rand((5, 4, p), 3)
    B = rand((4, 2, p), 4)
    Ah = np.fft.fft(A, axis=2)
    Bh = np.fft.fft(B, axis=2)
    Ch = np.einsum("ijk,jlk->ilk", Ah, Bh)
    ref = np.real(np.fft.ifft(Ch, axis=2))
    np.testing.assert_allclose(tp.tprod(A, B), ref, rtol=0, atol=1e-12)


def test_p1_is_matmul():
    A = rand((4, 3, 1), 5)
    B = rand((3, 6, 1), 6)
    np.testing.assert_allclose(tp.tprod(A, B)[:, :, 0], A[:, :, 0] @ B[:, :, 0], atol=1e-14)


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_dft_block_diagonalises_bcirc(p):
    # eq. (5) with the normalisation read as (F (x) I) bcirc(A) (F^{-1} (x) I);
    # F from numpy's FFT of the identity, Ahat from numpy's FFT.
    n1, n2 = 3, 2
    A = rand((n1, n2, p), 7)
    F = np.fft.fft(np.eye(p), axis=0)
    lhs = np.kron(F, np.eye(n1)) @ tp.bcirc(A) @ np.kron(np.linalg.inv(F), np.eye(n2))
    Ah = np.fft.fft(A, axis=2)
    rhs = np.zeros((n1 * p, n2 * p), dtype=complex)
    for k in range(p):
        rhs[k * n1:(k + 1) * n1, k * n2:(k + 1) * n2] = Ah[:, :, k]
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)
    np.testing.assert_allclose(tp.block_diag_of_dft(A), rhs, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6, 8])
def test_explicit_dft_matches_numpy(p):
    A = rand((3, 4, p), 8)
    np.testing.assert_allclose(tp.mode3_dft(A), np.fft.fft(A, axis=2), atol=1e-12)
    np.testing.assert_allclose(np.real(tp.mode3_idft(tp.mode3_dft(A))), A, atol=1e-13)
    F = tp.dft_matrix(p)
    # exact values at multiples of pi/2
    for k in range(p):
        for j in range(p):
            if (4 * j * k) % p == 0:
                assert F[k, j] in (1, -1, 1j, -1j)


def test_bcirc_is_homomorphism():
    A = rand((3, 4, 5), 9)
    B = rand((4, 2, 5), 10)
    np.testing.assert_allclose(tp.bcirc(tp.tprod(A, B)), tp.bcirc(A) @ tp.bcirc(B), atol=1e-12)


def test_identity_associativity_transpose():
    p = 4
    A = rand((3, 4, p), 11)
    B = rand((4, 5, p), 12)
    C = rand((5, 2, p), 13)
    np.testing.assert_allclose(tp.tprod(tp.identity(3, p), A), A, atol=1e-14)
    np.testing.assert_allclose(tp.tprod(A, tp.identity(4, p)), A, atol=1e-14)
    np.testing.assert_allclose(tp.tprod(tp.tprod(A, B), C), tp.tprod(A, tp.tprod(B, C)), atol=1e-12)
    np.testing.assert_allclose(tp.ttrans(tp.tprod(A, B)),
                               tp.tprod(tp.ttrans(B), tp.ttrans(A)), atol=1e-12)
    # transpose = conjugate transpose of every Fourier slice
    np.testing.assert_allclose(np.fft.fft(tp.ttrans(A), axis=2),
                               np.conj(np.transpose(np.fft.fft(A, axis=2), (1, 0, 2))), atol=1e-12)


def test_inner_norm_and_parseval():
    A = rand((3, 4, 5), 14)
    B = rand((3, 4, 5), 15)
    assert tp.inner(A, B) == pytest.approx(float(np.dot(A.ravel(), B.ravel())), rel=1e-14)
    assert tp.fnorm(A) == pytest.approx(np.linalg.norm(A.ravel()), rel=1e-14)
    Ah, Bh = np.fft.fft(A, axis=2), np.fft.fft(B, axis=2)
    assert tp.inner(A, B) == pytest.approx(np.real(np.vdot(Ah, Bh)) / 5, rel=1e-12)


def test_tube_inverse():
    a = np.array([3.0, 1.0, -0.5, 0.25])
    x = tp.tube_inv(a)
    e = np.zeros(4)
    e[0] = 1
    np.testing.assert_allclose(tp.tube_prod(a, x), e, atol=1e-14)
    np.testing.assert_allclose(np.fft.fft(x), 1.0 / np.fft.fft(a), atol=1e-14)


def test_golden_hand_computed():
    with open(os.path.join(GOLDEN, "tproduct_hand.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        if c["kind"] == "tube_prod":
            np.testing.assert_allclose(tp.tube_prod(c["a"], c["b"]), c["expect"], atol=1e-14)
        elif c["kind"] == "tprod":
            A = np.array(c["A"], dtype=float)   # given as [slice][row][col]
            B = np.array(c["B"], dtype=float)
            A = np.transpose(A, (1, 2, 0))
            B = np.transpose(B, (1, 2, 0))
            expect = np.transpose(np.array(c["expect"], dtype=float), (1, 2, 0))
            np.testing.assert_allclose(tp.tprod(A, B), expect, atol=1e-13)
        elif c["kind"] == "ttrans":
            A = np.transpose(np.array(c["A"], dtype=float), (1, 2, 0))
            expect = np.transpose(np.array(c["expect"], dtype=float), (1, 2, 0))
            np.testing.assert_allclose(tp.ttrans(A), expect, atol=0)
        else:
            raise AssertionError(c["kind"])


def test_sylv_op_entries_match_full():
    A = rand((6, 6, 5), 20)
    B = rand((3, 3, 5), 21)
    X = rand((6, 3, 5), 22)
    full = tp.tprod(A, X) - tp.tprod(X, B)
    idx = [(i, c, k) for i in range(6) for c in range(3) for k in range(5)]
    np.testing.assert_allclose(tp.sylv_op_entries(A, B, X, idx),
                               [full[i, c, k] for i, c, k in idx], atol=1e-13)


def test_ex3_workload_structure():
    """The experiment family's slices: mu/h^2 tridiag(-1, 2, -1) + c/(4h) T
    with T's stencil (1, 3, -5, 1) summing to zero, so every row with a full
    stencil annihilates the constant vector; the slices are banded (one
    subdiagonal, two superdiagonals) and C lies in [0, 1)."""
    from paper_2405_09233_amd import workloads
    n, s, p = 20, 5, 3
    A, B, C = workloads.ex3(n, s, p, mu=0.3, seed=4)
    for T, size in [(A, n), (B, s)]:
        for i in range(p):
            M = T[:, :, i]
            assert np.allclose(np.tril(M, -2), 0) and np.allclose(np.triu(M, 3), 0)
            ones = M @ np.ones(size)
            assert np.allclose(ones[1:size - 2], 0, atol=1e-9 * np.abs(M).max())
    # slice i differs from slice 1 only by (a_i - a_1)/(4 h) T
    h1 = 1.0 / (n + 1)
    D = (A[:, :, 1] - A[:, :, 0]) * 4 * h1
    assert np.allclose(np.diag(D), 3) and np.allclose(np.diag(D, 1), -5)
    assert np.allclose(np.diag(D, 2), 1) and np.allclose(np.diag(D, -1), 1)
    assert C.min() >= 0 and C.max() < 1
