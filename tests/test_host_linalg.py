"""CPU tests of the host-side FP64 complex linear algebra used by the TBAS
driver (Cholesky of Tubal-QR Gram matrices, triangular inverse, complex Schur,
banded projected Sylvester solve), compiled with g++ from the library's own
source and checked against numpy/scipy."""

import os
import subprocess

import numpy as np
import pytest
import scipy.linalg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_09233_amd", "csrc")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    out = tmp_path_factory.mktemp("hl") / "host_linalg_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC,
                    os.path.join(ROOT, "tests", "native", "host_linalg_check.cpp"),
                    os.path.join(CSRC, "host_linalg.cpp"), "-o", str(out)], check=True)
    return str(out)


def run(exe, header, mats):
    lines = [header]
    for m in mats:
        for v in np.asarray(m, dtype=complex).ravel(order="F"):
            lines.append("%.17g %.17g" % (v.real, v.imag))
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       check=True)
    return r.stdout.split("\n")


def parse(lines, start, shape):
    n = shape[0] * shape[1]
    vals = [complex(*map(float, l.split())) for l in lines[start:start + n]]
    return np.array(vals).reshape(shape, order="F"), start + n


def crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("s", [1, 3, 8, 17])
def test_cholesky_upper(exe, s):
    rng = np.random.default_rng(s)
    W = crand(rng, 3 * s, s)
    G = W.conj().T @ W
    out = run(exe, "chol %d" % s, [G])
    assert out[0] == "1"
    R, _ = parse(out, 1, (s, s))
    np.testing.assert_allclose(R.conj().T @ R, G, atol=1e-10 * np.abs(G).max())
    assert np.allclose(np.tril(R, -1), 0)
    assert np.all(np.abs(np.imag(np.diag(R))) == 0) and np.all(np.real(np.diag(R)) > 0)
    # equals the R of numpy's QR with a positive diagonal
    q, r = np.linalg.qr(W)
    ph = np.diag(r) / np.abs(np.diag(r))
    np.testing.assert_allclose(R, np.conj(ph)[:, None] * r, atol=1e-9)


def test_cholesky_rank_deficient(exe):
    rng = np.random.default_rng(0)
    W = crand(rng, 6, 3)
    W[:, 2] = W[:, 0] + 2 * W[:, 1]
    out = run(exe, "chol 3", [W.conj().T @ W])
    assert out[0] == "0"


@pytest.mark.parametrize("s", [1, 4, 9])
def test_tri_inv(exe, s):
    rng = np.random.default_rng(10 + s)
    R = np.triu(crand(rng, s, s)) + 3 * np.eye(s)
    out = run(exe, "triinv %d" % s, [R])
    Ri, _ = parse(out, 0, (s, s))
    np.testing.assert_allclose(Ri @ R, np.eye(s), atol=1e-12)


@pytest.mark.parametrize("n,real", [(1, False), (2, True), (5, False), (12, True), (40, False),
                                    (64, True)])
def test_schur(exe, n, real):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) if real else crand(rng, n, n)
    out = run(exe, "schur %d" % n, [A])
    assert out[0] == "1"
    T, pos = parse(out, 1, (n, n))
    U, _ = parse(out, pos, (n, n))
    np.testing.assert_allclose(U.conj().T @ U, np.eye(n), atol=1e-12 * n)
    np.testing.assert_allclose(U @ T @ U.conj().T, A, atol=1e-11 * n * np.abs(A).max())
    assert np.allclose(np.tril(T, -1), 0)
    ev = np.linalg.eigvals(A)
    dist = np.abs(np.diag(T)[:, None] - ev[None, :]).min(axis=1)
    assert dist.max() <= 1e-9 * n * max(1.0, np.abs(ev).max())


@pytest.mark.parametrize("m,s", [(1, 1), (2, 3), (4, 2), (3, 5)])
def test_sylvester_banded(exe, m, s):
    rng = np.random.default_rng(m * 10 + s)
    ms = m * s
    H = crand(rng, ms, ms)
    for i in range(ms):               # block upper Hessenberg: lower bandwidth s
        H[i + s + 1:, i] = 0
    H += 6 * np.eye(ms)
    B = crand(rng, s, s) - 6 * np.eye(s)
    C1 = crand(rng, ms, s)
    out = run(exe, "sylv %d %d %d" % (ms, s, s), [H, B, C1])
    assert out[0] == "1"
    Y, _ = parse(out, 1, (ms, s))
    np.testing.assert_allclose(Y, scipy.linalg.solve_sylvester(H, -B, C1), atol=1e-10)


@pytest.mark.parametrize("n,real", [(1, False), (3, True), (8, False), (24, True), (64, False)])
def test_eig_from_schur(exe, n, real):
    """B = W diag(lam) W^{-1} (the diagonalisation the device projected solve
    of TBAS uses), against the definition and numpy's eigenvalues."""
    rng = np.random.default_rng(100 + n)
    B = rng.standard_normal((n, n)) / np.sqrt(n) if real else crand(rng, n, n) / np.sqrt(2 * n)
    B -= 4 * np.eye(n)
    out = run(exe, "eig %d" % n, [B])
    ok, kappa = out[0].split()
    assert ok == "1" and np.isfinite(float(kappa)) and float(kappa) >= 1.0
    lam, pos = parse(out, 1, (n, 1))
    W, pos = parse(out, pos, (n, n))
    Wi, _ = parse(out, pos, (n, n))
    lam = lam.ravel()
    np.testing.assert_allclose(Wi @ W, np.eye(n), atol=1e-11 * float(kappa))
    np.testing.assert_allclose(B @ W, W * lam[None, :], atol=1e-11 * n)
    np.testing.assert_allclose(np.linalg.norm(W, axis=0), 1.0, atol=1e-12)
    ev = np.linalg.eigvals(B)
    assert np.abs(lam[:, None] - ev[None, :]).min(axis=1).max() <= 1e-10
    assert np.abs(ev[:, None] - lam[None, :]).min(axis=1).max() <= 1e-10


def test_eig_from_schur_defective(exe):
    """A Jordan block has no eigenvector basis: infinite condition."""
    B = np.array([[2.0, 1.0], [0.0, 2.0]])
    out = run(exe, "eig 2", [B])
    ok, kappa = out[0].split()
    assert ok == "1" and not np.isfinite(float(kappa))
