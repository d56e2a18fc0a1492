"""Brute-force Kronecker solve of the Sylvester tensor equation.

TEST INFRASTRUCTURE ONLY (see the package docstring): not used by the
product path.

bcirc is an algebra homomorphism (bcirc(A*B) = bcirc(A) bcirc(B), which
follows from the definition of the T-product in section 2.1), so
A*X - X*B = C is equivalent to the matrix Sylvester equation
bcirc(A) Z - Z bcirc(B) = bcirc(C) with Z = bcirc(X), i.e. to the linear
system

    (I_{sp} (x) bcirc(A) - bcirc(B)^T (x) I_{np}) vec(Z) = vec(bcirc(C)).

It is solved by a dense LU; X is folded back from the first block column
of Z.  Only for tiny inputs: the system has (n p)(s p) unknowns.
"""

import numpy as np

from .tproduct import bcirc, fold


def kron_matrix(A, B):
    """The (np sp) x (np sp) matrix I (x) bcirc(A) - bcirc(B)^T (x) I."""
    n, _, p = A.shape
    s = B.shape[0]
    bA = bcirc(A)
    bB = bcirc(B)
    return np.kron(np.eye(s * p), bA) - np.kron(bB.T, np.eye(n * p))


def kron_solve(A, B, C, return_Z=False):
    """Solve A*X - X*B = C by the Kronecker system above.  vec stacks
    columns (Fortran order).  With ``return_Z`` the full solution matrix Z
    (which must be block circulant) is returned as well."""
    n, _, p = A.shape
    s = B.shape[0]
    K = kron_matrix(A, B)
    rhs = bcirc(C).reshape(-1, order="F")
    z = np.linalg.solve(K, rhs)
    Z = z.reshape((n * p, s * p), order="F")
    X = fold(Z[:, :s], n, s, p)
    if return_Z:
        return X, Z
    return X


def sylv_matrix(A, B):
    """Explicit nsp x nsp matrix of M acting on vec(unfold(X)) (Fortran
    order), built column by column by applying the Kronecker form to
    bcirc of unit tensors.  Used to compare tGMRES with textbook GMRES on the
    same linear system."""
    n, _, p = A.shape
    s = B.shape[0]
    K = kron_matrix(A, B)
    N = n * s * p
    out = np.zeros((N, N))
    for col in range(N):
        E = np.zeros(N)
        E[col] = 1.0
        X = E.reshape((n, s, p), order="F")
        z = K @ bcirc(X).reshape(-1, order="F")
        Z = z.reshape((n * p, s * p), order="F")
        out[:, col] = fold(Z[:, :s], n, s, p).reshape(-1, order="F")
    return out
