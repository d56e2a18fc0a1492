"""t-Schur decomposition and the t-Bartels-Stewart method (section 4).

TEST INFRASTRUCTURE ONLY (see the package docstring): not used by the
product path.

Sign convention: the equation solved is A*X - X*B = C, the operator of
eq. (2) and of section 5.2 (section 4 writes the same method for the
"+" form; the "-" form is the one the Krylov solvers use and the one the
projected equation of TBAS needs).
"""

import numpy as np
import scipy.linalg

from .tproduct import (tprod, tconjtrans, mode3_dft, mode3_idft, circ,
                       tube_inv)


def t_schur(A):
    """t-Schur decomposition A = U * R * U^H (Theorem and Algorithm 4 of
    section 4): Schur-decompose every Fourier slice, then return to the
    spatial domain with the inverse DFT.

    Reading: a complex Fourier slice has no real Schur form, so every slice
    k <= floor(p/2) gets a complex Schur decomposition (scipy's, a library
    primitive) and the slices k > p/2 take the conjugates of their mirror
    slices p - k, as the conjugate symmetry of the DFT of a real tensor
    requires.  R is then upper triangular in every slice (not only
    quasi-triangular).  When a real slice (k = 0, or k = p/2 for even p) has
    complex eigenvalues its Schur factors are complex, so U and R are
    complex tensors; the transpose of the paper then becomes the conjugate
    transpose, and U^H * U = I still holds.
    """
    n, n2, p = A.shape
    assert n == n2
    Ah = mode3_dft(A)
    Uh = np.zeros_like(Ah)
    Rh = np.zeros_like(Ah)
    for k in range(p // 2 + 1):
        T, Z = scipy.linalg.schur(Ah[:, :, k], output="complex")
        Uh[:, :, k] = Z
        Rh[:, :, k] = T
    for k in range(p // 2 + 1, p):
        Uh[:, :, k] = np.conj(Uh[:, :, p - k])
        Rh[:, :, k] = np.conj(Rh[:, :, p - k])
    return mode3_idft(Uh), mode3_idft(Rh)


def t_back_substitution(RA, RB, C1):
    """Solve the triangular tensor equation RA * Y - Y * RB = C1 (the
    triangular equation of section 4 and its remark): tubes play the role of
    scalars, lateral slices of vectors and the T-product of the matrix
    product.  Tubes commute, so entry (i, j) reads

        (ra_ii - rb_jj) * y_ij = c_ij + sum_{l<j} y_il * rb_lj
                                      - sum_{l>i} ra_il * y_lj,

    solved column by column (j ascending) and, inside a column, from the
    last row up.  Tube products are circular convolutions; the tube inverse
    is a dense solve with the circulant matrix (Def. 2.2 item 2).
    """
    n, s, p = C1.shape
    dt = np.result_type(RA.dtype, RB.dtype, C1.dtype, np.complex128)
    Y = np.zeros((n, s, p), dtype=dt)

    def tp(a, b):
        return circ(np.asarray(a, dtype=dt)) @ np.asarray(b, dtype=dt)

    for j in range(s):
        for i in range(n - 1, -1, -1):
            t = C1[i, j, :].astype(dt)
            for l in range(j):
                t = t + tp(Y[i, l, :], RB[l, j, :])
            for l in range(i + 1, n):
                t = t - tp(RA[i, l, :], Y[l, j, :])
            d = RA[i, i, :] - RB[j, j, :]
            Y[i, j, :] = tp(tube_inv(d.astype(dt)), t)
    return Y


def t_bartels_stewart(A, B, C, return_complex=False):
    """t-Bartels-Stewart method (Algorithm 5 of section 4) for
    A*X - X*B = C: t-Schur forms of A and B, C1 = U_A^H * C * U_B,
    t-back-substitution for Y, X = U_A * Y * U_B^H.

    The result is real in exact arithmetic; the imaginary part left by
    rounding is dropped unless ``return_complex``.
    """
    UA, RA = t_schur(A)
    UB, RB = t_schur(B)
    C1 = tprod(tprod(tconjtrans(UA), C.astype(np.complex128)), UB)
    Y = t_back_substitution(RA, RB, C1)
    X = tprod(tprod(UA, Y), tconjtrans(UB))
    if return_complex:
        return X
    return np.real(X)
