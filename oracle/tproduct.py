"""T-product algebra, written from the definitions of section 2.

TEST INFRASTRUCTURE ONLY (see the package docstring): not used by the
product path.

Tensors are numpy arrays of shape (rows, cols, p); ``T[:, :, k]`` is the
frontal slice k+1 of the paper (0-based here).  No FFT is used anywhere in
this module: the T-product is the explicit sum over the circulant pattern
of bcirc, and the mode-3 DFT needed by the t-Schur decomposition is an
explicit O(p^2) sum with a DFT matrix built from its definition.
"""

import numpy as np


# --------------------------------------------------------------------------
# Section 2.1: bcirc, unfold, fold
# --------------------------------------------------------------------------

def bcirc(A):
    """Block-circulant matrix of A (section 2.1, definition of bcirc).

    Block row r, block column c holds frontal slice ((r - c) mod p): the
    first block column is slices 1..p top to bottom and every following
    block column is the previous one shifted down by one block.
    """
    n1, n2, p = A.shape
    out = np.zeros((n1 * p, n2 * p), dtype=A.dtype)
    for r in range(p):
        for c in range(p):
            out[r * n1:(r + 1) * n1, c * n2:(c + 1) * n2] = A[:, :, (r - c) % p]
    return out


def unfold(A):
    """Stack the frontal slices vertically (section 2.1, unfold)."""
    n1, n2, p = A.shape
    return np.concatenate([A[:, :, k] for k in range(p)], axis=0)


def fold(M, n1, n2, p):
    """Inverse of :func:`unfold` (section 2.1, fold)."""
    assert M.shape == (n1 * p, n2)
    out = np.zeros((n1, n2, p), dtype=M.dtype)
    for k in range(p):
        out[:, :, k] = M[k * n1:(k + 1) * n1, :]
    return out


# --------------------------------------------------------------------------
# Definition of the T-product and its consequences
# --------------------------------------------------------------------------

def tprod(A, B):
    """T-product A * B = fold(bcirc(A) unfold(B)) (section 2.1, Def. of
    the T-product), evaluated as the circulant sum it expands to:

        (A * B)[:, :, k] = sum_j A[:, :, (k - j) mod p] @ B[:, :, j].

    Block row k of bcirc(A) holds slice (k - j) mod p in block column j,
    and block j of unfold(B) is slice j, so this is that matrix product
    written block by block.  Cost O(n1 n2 m p^2).
    """
    n1, n2, p = A.shape
    n2b, m, pb = B.shape
    if n2 != n2b or p != pb:
        raise ValueError("tprod: shapes %s and %s do not chain" % (A.shape, B.shape))
    dt = np.result_type(A.dtype, B.dtype)
    out = np.zeros((n1, m, p), dtype=dt)
    for k in range(p):
        out[:, :, k] = tprod_slice(A, B, k)
    return out


def tprod_slice(A, B, k):
    """Frontal slice k of A * B: sum_j A[:, :, (k - j) mod p] @ B[:, :, j]
    (block row k of bcirc(A) times unfold(B))."""
    p = A.shape[2]
    acc = np.zeros((A.shape[0], B.shape[1]), dtype=np.result_type(A.dtype, B.dtype))
    for j in range(p):
        acc += A[:, :, (k - j) % p] @ B[:, :, j]
    return acc


def ttrans(A):
    """Tensor transpose (section 2.1, Def. 2.2 item 4): transpose every
    frontal slice, then reverse the order of slices 2..p."""
    n1, n2, p = A.shape
    out = np.zeros((n2, n1, p), dtype=A.dtype)
    out[:, :, 0] = A[:, :, 0].T
    for k in range(1, p):
        out[:, :, k] = A[:, :, p - k].T
    return out


def tconjtrans(A):
    """Conjugate analogue of :func:`ttrans` for complex tensors: the slices
    are conjugate-transposed, then slices 2..p reversed.  For real tensors it
    equals the transpose of Def. 2.2 item 4."""
    return np.conj(ttrans(A))


def identity(n, p, dtype=np.float64):
    """Identity tensor (Def. 2.2 item 1): first slice I, the others zero."""
    out = np.zeros((n, n, p), dtype=dtype)
    out[:, :, 0] = np.eye(n, dtype=dtype)
    return out


def inner(A, B):
    """Scalar inner product <A, B> = sum_ijk a_ijk b_ijk (section 2.1,
    definition of the scalar inner product)."""
    return float(np.sum(A * B))


def fnorm(A):
    """Frobenius norm sqrt(<A, A>) (same definition)."""
    return float(np.sqrt(np.sum(A * A)))


def sylv_op(A, B, X):
    """The Sylvester operator M(X) = A * X - X * B of eq. (2)."""
    return tprod(A, X) - tprod(X, B)


def tdiamond(Ablocks, Bblocks):
    """T-diamond product (section 2.1, definition of A^T <> B): the matrix of
    scalar inner products <A_i, B_j> between two lists of equally shaped
    blocks."""
    out = np.zeros((len(Ablocks), len(Bblocks)))
    for i, a in enumerate(Ablocks):
        for j, b in enumerate(Bblocks):
            out[i, j] = inner(a, b)
    return out


# --------------------------------------------------------------------------
# Tubes (1 x 1 x p): product, inverse, circulant
# --------------------------------------------------------------------------

def circ(a):
    """p x p circulant matrix of a tube a (bcirc of a 1 x 1 x p tensor)."""
    a = np.asarray(a).reshape(-1)
    p = a.size
    out = np.zeros((p, p), dtype=a.dtype)
    for r in range(p):
        for c in range(p):
            out[r, c] = a[(r - c) % p]
    return out


def tube_prod(a, b):
    """T-product of two tubes: the circular convolution
    (a * b)_k = sum_j a_{(k - j) mod p} b_j (Def. of the T-product with
    n1 = n2 = m = 1)."""
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return circ(a) @ b


def tube_inv(a):
    """Inverse tube (Def. 2.2 item 2): the tube x with a * x = e, e the
    first unit tube, found by a dense LU solve of circ(a) x = e."""
    a = np.asarray(a).reshape(-1)
    e = np.zeros(a.size, dtype=a.dtype)
    e[0] = 1.0
    return np.linalg.solve(circ(a), e)


# --------------------------------------------------------------------------
# Explicit mode-3 DFT (section 2.1, fft(A, [], 3) and eq. (5))
# --------------------------------------------------------------------------

def dft_matrix(p):
    """The p x p DFT matrix F with F[k, j] = exp(-2 pi i j k / p), the matrix
    that MATLAB's fft applies along a tube.  The angle is reduced as
    (j k) mod p before the exponential so the multiples of pi/2 come out as
    exact 1, -1, i, -i."""
    F = np.zeros((p, p), dtype=np.complex128)
    for k in range(p):
        for j in range(p):
            r = (j * k) % p
            if (4 * r) % p == 0:
                quarter = (4 * r) // p
                F[k, j] = [1.0, -1j, -1.0, 1j][quarter]
            else:
                F[k, j] = np.exp(-2j * np.pi * r / p)
    return F


def mode3_dft(A):
    """Ahat[:, :, k] = sum_j A[:, :, j] F[k, j] (section 2.1, fft along the
    third mode), by the explicit O(p^2) sum."""
    p = A.shape[2]
    F = dft_matrix(p)
    out = np.zeros(A.shape, dtype=np.complex128)
    for k in range(p):
        for j in range(p):
            out[:, :, k] += F[k, j] * A[:, :, j]
    return out


def mode3_idft(Ahat):
    """Inverse of :func:`mode3_dft`: A_j = (1/p) sum_k conj(F[k, j]) Ahat_k."""
    p = Ahat.shape[2]
    F = dft_matrix(p)
    out = np.zeros(Ahat.shape, dtype=np.complex128)
    for j in range(p):
        for k in range(p):
            out[:, :, j] += np.conj(F[k, j]) * Ahat[:, :, k]
    return out / p


def block_diag_of_dft(A):
    """The block-diagonal matrix Diag(Ahat) of eq. (4)."""
    n1, n2, p = A.shape
    Ah = mode3_dft(A)
    out = np.zeros((n1 * p, n2 * p), dtype=np.complex128)
    for k in range(p):
        out[k * n1:(k + 1) * n1, k * n2:(k + 1) * n2] = Ah[:, :, k]
    return out


def sylv_op_entries(A, B, X, idx):
    """Selected entries of M(X) = A*X - X*B (eq. (2)), each by its own
    circulant sum: for (i, c, k) in idx,

        M(X)[i, c, k] = sum_j A[i, :, (k-j) mod p] . X[:, c, j]
                        - sum_j X[i, :, (k-j) mod p] . B[:, c, j].

    Cost O((n + s) p) per entry, so it can spot-check operators far too
    large for :func:`sylv_op`."""
    p = A.shape[2]
    out = np.zeros(len(idx))
    for t, (i, c, k) in enumerate(idx):
        acc = 0.0
        for j in range(p):
            kj = (k - j) % p
            acc += float(A[i, :, kj] @ X[:, c, j])
            acc -= float(X[i, :, kj] @ B[:, c, j])
        out[t] = acc
    return out
