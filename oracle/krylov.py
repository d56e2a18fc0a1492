"""tArnoldi, tFOM, tGMRES (section 3) and Tubal-QR, TBA, TBAS(m) (section 5).

TEST INFRASTRUCTURE ONLY (see the package docstring): not used by the
product path.

Everything here is spatial and FP64: M is applied with the circulant-sum
T-product of :mod:`oracle.tproduct`, inner products are the plain sums of
section 2.1, and tubes are handled with circulant matrices.  The algorithms
follow the paper's steps in its order; where a step is garbled the reading
taken is stated in the docstring.
"""

import numpy as np

from .tproduct import (tprod, ttrans, inner, fnorm, sylv_op, circ, tube_prod,
                       tube_inv)

EPS = np.finfo(np.float64).eps


class Breakdown(Exception):
    """A tube met by Normalization is not invertible (section 5.1: the tube
    returned by Normalization must be invertible)."""


class SingularProjected(Exception):
    """The projected problem of a cycle has no unique solution."""


# --------------------------------------------------------------------------
# One modified Gram-Schmidt process for the three orthogonalisations
# --------------------------------------------------------------------------

def _gram_schmidt(count, basis, candidate, coef, remove, finish):
    """Modified Gram-Schmidt over any space with an inner product.

    Starting from `basis` (a list, extended in place), for j = 0, 1, ...,
    count - 1: w = candidate(j, basis) is made orthogonal to the basis one
    element at a time, in the order of the basis (c_i = coef(b_i, w), then
    w = remove(w, b_i, c_i)), and finish(j, w, coefs) returns (unit, size,
    stop): the new basis element (None when there is none), the coefficient
    of w along it, and whether the process ends after column j.

    The scalar Arnoldi process of section 3.1 (basis seeded with the
    normalised start, candidate M of basis element j, real coefficients),
    the tubal QR of section 5.1 (empty start, candidate the next lateral
    slice, tube coefficients) and the tubal block Arnoldi process (seeded
    with the first block, candidate A times block j, s x s x p tubal
    coefficients) are this one process with different operations.

    Returns the list of columns (coefs, size), one per completed j.
    """
    columns = []
    for j in range(count):
        w = candidate(j, basis)
        coefs = []
        for b in list(basis):
            c = coef(b, w)
            w = remove(w, b, c)
            coefs.append(c)
        unit, size, stop = finish(j, w, coefs)
        columns.append((coefs, size))
        if unit is not None:
            basis.append(unit)
        if stop:
            break
    return columns


# --------------------------------------------------------------------------
# Algorithm 2: tArnoldi
# --------------------------------------------------------------------------

def tarnoldi(Mop, V, m, on_step=None):
    """Tensor tArnoldi (Algorithm 2): the Arnoldi process of M with modified
    Gram-Schmidt -- the Krylov basis V_1 = V / ||V||_F, V_2, ... and the
    Hessenberg matrix of the coefficients.

    Reading: the algorithm lists A as input but applies M; M is used.  A
    zero h_{j+1,j} is detected as h_{j+1,j} <= 16 eps ||M(V_j)||_F (happy
    breakdown: the process stops with j columns).

    ``on_step(j, H)`` (optional) is called after column j (0-based) of the
    Hessenberg matrix is complete and may return True to stop early.

    Returns (Vs, H, W, k): the basis V_1..V_{k+1} (V_{k+1} absent after a
    breakdown), the (k+1) x k Hessenberg matrix, the images M(V_j), and k,
    the number of completed steps.
    """
    Vs = [V / fnorm(V)]
    H = np.zeros((m + 1, m))
    Ws, wnorm0 = [], []

    def candidate(j, basis):
        W = Mop(basis[j])
        Ws.append(W.copy())
        wnorm0.append(fnorm(W))
        return W

    def finish(j, W, coefs):
        H[:j + 1, j] = coefs
        H[j + 1, j] = fnorm(W)
        unit, stop = None, False
        if H[j + 1, j] <= 16 * EPS * wnorm0[j]:
            H[j + 1, j] = 0.0
            stop = True
        else:
            unit = W / H[j + 1, j]
        if on_step is not None and on_step(j, H[:j + 2, :j + 1]):
            stop = True
        return unit, H[j + 1, j], stop

    k = len(_gram_schmidt(m, Vs, candidate, lambda b, W: inner(b, W),
                          lambda W, b, c: W - c * b, finish))
    if k < m:
        return Vs, H[:k + 1, :k], Ws, k
    return Vs, H, Ws, m


def combine(Vs, y):
    """The product V_m (*) y = sum_j y_j V_j of section 3.1."""
    out = np.zeros_like(Vs[0])
    for j, yj in enumerate(y):
        out = out + yj * Vs[j]
    return out


# --------------------------------------------------------------------------
# Small problems of Algorithm 3, step 4(b)
# --------------------------------------------------------------------------

def givens_ls(Ht, beta):
    """Least-squares problem of tGMRES (section 3.3): y minimising
    || beta e_1 - Htilde y ||_2, through the QR decomposition of the
    (k+1) x k upper Hessenberg Htilde by Givens rotations, as in the
    residual proposition of section 3.3: gamma = beta Q^T e_1, y solves the
    triangular system with the first k entries of gamma, and the residual
    norm is |gamma_{k+1}|.

    Returns (y, |gamma_{k+1}|).
    """
    k = Ht.shape[1]
    U = np.array(Ht, dtype=np.float64)
    g = np.zeros(k + 1)
    g[0] = beta
    for i in range(k):
        a, b = U[i, i], U[i + 1, i]
        r = np.hypot(a, b)
        if r == 0.0:
            c, s = 1.0, 0.0
        else:
            c, s = a / r, b / r
        rot = np.array([[c, s], [-s, c]])
        U[i:i + 2, i:] = rot @ U[i:i + 2, i:]
        g[i:i + 2] = rot @ g[i:i + 2]
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        if U[i, i] == 0.0:
            raise SingularProjected("tGMRES: singular triangular factor")
        y[i] = (g[i] - U[i, i + 1:k] @ y[i + 1:]) / U[i, i]
    return y, abs(g[k])


def fom_solve(H, beta):
    """Small system of tFOM (section 3.2): H_k y = beta e_1, solved by LU
    with partial pivoting.  Raises SingularProjected when H_k is singular."""
    k = H.shape[0]
    rhs = np.zeros(k)
    rhs[0] = beta
    try:
        y = np.linalg.solve(H, rhs)
    except np.linalg.LinAlgError as exc:
        raise SingularProjected(str(exc))
    if not np.all(np.isfinite(y)):
        raise SingularProjected("tFOM: non-finite solution")
    return y


# --------------------------------------------------------------------------
# Algorithm 3: restarted tFOM / tGMRES
# --------------------------------------------------------------------------

def tkrylov_solve(A, B, C, method="gmres", m=30, tol=1e-8, max_cycles=100,
                  X0=None, early_exit=True):
    """Algorithm 3 (tFOM and tGMRES) for M(X) = A*X - X*B = C.

    Readings of the garbled control flow of Algorithm 3:
      * Iter_max is the maximum number of restart cycles; the true residual
        R = C - M(X) is recomputed at the start of every cycle and decides
        convergence, as a relative residual ||R||_F / ||C||_F <= tol.
      * Within a cycle the Arnoldi process also stops as soon as the cheap
        residual estimate is below tol ||C||_F (|gamma_{j+1}| for tGMRES,
        h_{j+1,j} |y_j| for tFOM: the two residual propositions of
        section 3), so that the last cycle does not run m steps needlessly.
      * tFOM: a step whose H_j is singular gives no estimate; when H_k is
        singular at the end of a cycle the tGMRES solution of that cycle is
        used for the restart and ``info['fom_fallback']`` counts it.

    Returns (X, info) with info = dict(steps, cycles, relres_true,
    converged, est_hist, true_hist, fom_fallback).
    """
    n, s, p = C.shape
    X = np.zeros_like(C) if X0 is None else np.array(X0, dtype=np.float64)
    Mop = lambda V: sylv_op(A, B, V)
    cnorm = fnorm(C)
    info = dict(steps=0, cycles=0, relres_true=None, converged=False,
                est_hist=[], true_hist=[], fom_fallback=0)
    if cnorm == 0.0:
        info.update(relres_true=0.0, converged=True)
        return np.zeros_like(C), info
    for cycle in range(max_cycles + 1):
        R0 = C - Mop(X)
        beta = fnorm(R0)
        rel = beta / cnorm
        info["true_hist"].append(rel)
        info["relres_true"] = rel
        if rel <= tol:
            info["converged"] = True
            return X, info
        if cycle == max_cycles:
            break
        info["cycles"] += 1

        def on_step(j, Hj):
            k = j + 1
            if method == "gmres":
                _, est = givens_ls(Hj, beta)
            else:
                try:
                    y = fom_solve(Hj[:k, :k], beta)
                    est = Hj[k, k - 1] * abs(y[-1])
                except SingularProjected:
                    est = np.inf
            info["est_hist"].append(est / cnorm)
            return early_exit and est <= tol * cnorm

        Vs, Ht, _, k = tarnoldi(Mop, R0, m, on_step)
        info["steps"] += k
        if method == "gmres":
            y, _ = givens_ls(Ht, beta)
        else:
            try:
                y = fom_solve(Ht[:k, :k], beta)
            except SingularProjected:
                info["fom_fallback"] += 1
                y, _ = givens_ls(Ht, beta)
        X = X + combine(Vs, y)
    return X, info


def tgmres(A, B, C, **kw):
    """tGMRES(m) of Algorithm 3."""
    return tkrylov_solve(A, B, C, method="gmres", **kw)


def tfom(A, B, C, **kw):
    """tFOM(m) of Algorithm 3."""
    return tkrylov_solve(A, B, C, method="fom", **kw)


# --------------------------------------------------------------------------
# Section 5.1: Normalization, Tubal-QR, TBA
# --------------------------------------------------------------------------

def normalization(W, breakdown_tol=16 * EPS):
    """Normalization of a lateral slice W (n x 1 x p), section 5.1: write
    W = U * a with U^T * U = e and a an invertible tube.

    Reading: the paper defines this step only by citation and the tube a is
    not unique; the symmetric positive choice is taken.  With the symmetric
    tube g = W^T * W, circ(g) is a symmetric positive semidefinite p x p
    matrix (it is bcirc(W)^T bcirc(W)); a is the first column of its
    positive semidefinite square root (computed with a symmetric
    eigendecomposition), and U = W * a^{-1}.  The tube a is declared not
    invertible when an eigenvalue of circ(a) is <= breakdown_tol times the
    largest one (Breakdown is raised).
    """
    n, one, p = W.shape
    assert one == 1
    g = tprod(ttrans(W), W).reshape(p)
    G = circ(g)
    G = 0.5 * (G + G.T)
    lam, Q = np.linalg.eigh(G)
    lam = np.clip(lam, 0.0, None)
    sq = np.sqrt(lam)
    if sq.max() == 0.0 or sq.min() <= breakdown_tol * sq.max():
        raise Breakdown("Normalization: tube not invertible")
    a = (Q * sq) @ Q[0, :]          # first column of Q diag(sq) Q^T
    ainv = tube_inv(a)
    U = tprod(W, ainv.reshape(1, 1, p))
    return U, a


def tubal_qr(Amat):
    """Tubal-QR factorisation A = Q * R (Theorem and Algorithm 6 of
    section 5.1): modified Gram-Schmidt of the lateral slices A_1..A_s with
    tube-valued coefficients r_ij = Q_i^T * A_j, each remainder split by
    Normalization into Q_j and the tube r_jj.

    Reading of the garbled loops: the coefficients of slice j are taken
    against Q_1..Q_{j-1} in order, each removed before the next is formed.
    R[i, j, :] is the tube r_ij; R is upper triangular in every frontal
    slice.
    """
    n, s, p = Amat.shape
    R = np.zeros((s, s, p))

    def finish(j, W, coefs):
        for i, rij in enumerate(coefs):
            R[i, j, :] = rij.reshape(p)
        Qj, a = normalization(W)
        R[j, j, :] = a
        return Qj, a, False

    Qs = []
    _gram_schmidt(s, Qs, lambda j, basis: Amat[:, j:j + 1, :].copy(),
                  lambda Qi, W: tprod(ttrans(Qi), W), lambda W, Qi, r: W - tprod(Qi, r),
                  finish)
    Q = np.concatenate(Qs, axis=1) if Qs else np.zeros((n, 0, p))
    return Q, R


def tba(A, V, m):
    """Tubal Block Arnoldi (Algorithm 7 of section 5.1): the block Arnoldi
    process of A with tube-valued (s x s x p) coefficients H_ij = V_i^T * W
    removed block by block (modified Gram-Schmidt), each remainder split by
    Tubal-QR into the next block and H_{j+1,j}.

    Reading: W = A * V_j uses A, not M (B enters only the projected
    equation of TBAS).

    Returns (Vb, Hbig, H0): the blocks V_1..V_{m+1} (each n x s x p), the
    block Hessenberg tensor of size (m+1)s x ms x p, and H0 from
    Tubal-QR(V).
    """
    n, s, p = V.shape
    V1, H0 = tubal_qr(V)
    Hbig = np.zeros(((m + 1) * s, m * s, p))

    def finish(j, W, coefs):
        for i, Hij in enumerate(coefs):
            Hbig[i * s:(i + 1) * s, j * s:(j + 1) * s, :] = Hij
        Vn, Hn = tubal_qr(W)
        Hbig[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s, :] = Hn
        return Vn, Hn, False

    Vb = [V1]
    _gram_schmidt(m, Vb, lambda j, basis: tprod(A, basis[j]),
                  lambda Vi, W: tprod(ttrans(Vi), W), lambda W, Vi, H: W - tprod(Vi, H),
                  finish)
    return Vb, Hbig, H0


def block_cat(blocks):
    """Lateral concatenation of blocks (Def. 2.5, block tensor)."""
    return np.concatenate(blocks, axis=1)


# --------------------------------------------------------------------------
# Section 5.2: TBAS(m)
# --------------------------------------------------------------------------

def tbas(A, B, C, m=10, tol=1e-8, max_cycles=50, X0=None):
    """Restarted Tubal-Block-Arnoldi Sylvester solver TBAS(m) (Algorithm 8).

    Each cycle: R0 = C - M(X0); TBA(A, R0, m); solve the projected equation
    H_m * Y - Y * B = V_m^T * R0 with t-Bartels-Stewart (Algorithm 5);
    X = X0 + V_m * Y.  Readings as in :func:`tkrylov_solve` for the
    restart loop and the relative stopping test.  The residual estimate of
    the proposition of section 5.2, ||H_{m+1,m} * E_m * Y||_F, is recorded
    in ``info['est_hist']``.
    """
    from .tbs import t_bartels_stewart
    n, s, p = C.shape
    X = np.zeros_like(C) if X0 is None else np.array(X0, dtype=np.float64)
    cnorm = fnorm(C)
    info = dict(steps=0, cycles=0, relres_true=None, converged=False,
                est_hist=[], true_hist=[])
    if cnorm == 0.0:
        info.update(relres_true=0.0, converged=True)
        return np.zeros_like(C), info
    for cycle in range(max_cycles + 1):
        R0 = C - sylv_op(A, B, X)
        rel = fnorm(R0) / cnorm
        info["true_hist"].append(rel)
        info["relres_true"] = rel
        if rel <= tol:
            info["converged"] = True
            return X, info
        if cycle == max_cycles:
            break
        info["cycles"] += 1
        Vb, Hbig, H0 = tba(A, R0, m)
        info["steps"] += m
        Vm = block_cat(Vb[:m])                          # n x ms x p
        Hm = Hbig[:m * s, :, :]                          # ms x ms x p
        C1 = tprod(ttrans(Vm), R0)                       # ms x s x p
        Y = t_bartels_stewart(Hm, B, C1)
        X = X + tprod(Vm, Y)
        Hlast = Hbig[m * s:, (m - 1) * s:, :]            # s x s x p
        est = fnorm(tprod(Hlast, Y[(m - 1) * s:, :, :]))
        info["est_hist"].append(est / cnorm)
    return X, info
