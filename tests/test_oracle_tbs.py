"""Pins of the oracle's t-Schur and t-Bartels-Stewart (section 4) against the
Kronecker solve, per-slice scipy Sylvester solves via numpy's FFT and the
properties of the t-Schur theorem."""

import numpy as np
import pytest
import scipy.linalg

from oracle import tproduct as tp
from oracle import tbs
from oracle import kron
from paper_2405_09233_amd import workloads


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_t_schur_properties(p):
    A = np.random.default_rng(p).standard_normal((4, 4, p))
    U, R = tbs.t_schur(A)
    np.testing.assert_allclose(tp.tprod(tp.tprod(U, R), tp.tconjtrans(U)), A, atol=1e-11)
    np.testing.assert_allclose(tp.tprod(tp.tconjtrans(U), U), tp.identity(4, p), atol=1e-11)
    for k in range(p):
        np.testing.assert_allclose(np.tril(R[:, :, k], -1), 0, atol=1e-12)


def test_t_schur_real_when_spectra_real():
    # symmetric slices: every Fourier slice Hermitian, DC/Nyquist real symmetric
    rng = np.random.default_rng(3)
    A = rng.standard_normal((4, 4, 4))
    A = 0.5 * (A + tp.ttrans(A))
    U, R = tbs.t_schur(A)
    assert np.max(np.abs(np.imag(U))) < 1e-12


@pytest.mark.parametrize("n,s,p", [(3, 2, 1), (4, 3, 2), (4, 3, 3), (5, 2, 4), (3, 3, 5)])
def test_t_bartels_stewart_vs_kron_and_fft(n, s, p):
    A, B, C = workloads.dense_shifted(n, s, p, seed=n * 10 + p)
    X = tbs.t_bartels_stewart(A, B, C)
    Xk = kron.kron_solve(A, B, C)
    np.testing.assert_allclose(X, Xk, atol=1e-11)
    Xc = tbs.t_bartels_stewart(A, B, C, return_complex=True)
    assert np.max(np.abs(np.imag(Xc))) < 1e-11
    Ah, Bh, Ch = (np.fft.fft(T, axis=2) for T in (A, B, C))
    for k in range(p):
        ref = scipy.linalg.solve_sylvester(Ah[:, :, k], -Bh[:, :, k], Ch[:, :, k])
        np.testing.assert_allclose(np.fft.fft(X, axis=2)[:, :, k], ref, atol=1e-10)


def test_t_bartels_stewart_tiny_dense_workload():
    A, B, C = workloads.tiny_dense(0)
    X = tbs.t_bartels_stewart(A, B, C)
    Xk = kron.kron_solve(A, B, C)
    assert np.linalg.norm(X - Xk) <= 1e-12 * np.linalg.norm(Xk)


def test_back_substitution_plain_triangular():
    # p = 1: tubes are scalars, so this is the scalar Bartels-Stewart back
    # substitution; compare with scipy on the same triangular system.
    rng = np.random.default_rng(0)
    RA = np.triu(rng.standard_normal((4, 4))) + 3 * np.eye(4)
    RB = np.triu(rng.standard_normal((3, 3))) - 3 * np.eye(3)
    C1 = rng.standard_normal((4, 3))
    Y = tbs.t_back_substitution(RA[:, :, None], RB[:, :, None], C1[:, :, None])[:, :, 0]
    np.testing.assert_allclose(Y, scipy.linalg.solve_sylvester(RA, -RB, C1), atol=1e-12)
