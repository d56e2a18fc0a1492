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
# Algorithm 2: tArnoldi
# --------------------------------------------------------------------------

def tarnoldi(Mop, V, m, on_step=None):
    """Tensor tArnoldi (Algorithm 2) with modified Gram-Schmidt as printed.

    Reading: the algorithm lists A as input but applies M (step 3(a)); M is
    used.  A zero h_{j+1,j} is detected as h_{j+1,j} <= 16 eps ||M(V_j)||_F
    (happy breakdown: the process stops with j columns).

    ``on_step(j, H)`` (optional) is called after column j (0-based) of the
    Hessenberg matrix is complete and may return True to stop early.

    Returns (Vs, H, W, k): the basis V_1..V_{k+1} (V_{k+1} absent after a
    breakdown), the (k+1) x k Hessenberg matrix, the images M(V_j), and k,
    the number of completed steps.
    """
    beta = fnorm(V)
    Vs = [V / beta]
    H = np.zeros((m + 1, m))
    Ws = []
    for j in range(m):
        W = Mop(Vs[j])
        Ws.append(W.copy())
        wnorm0 = fnorm(W)
        for i in range(j + 1):
            H[i, j] = inner(Vs[i], W)
            W = W - H[i, j] * Vs[i]
        H[j + 1, j] = fnorm(W)
        stop = False
        if H[j + 1, j] <= 16 * EPS * wnorm0:
            H[j + 1, j] = 0.0
            stop = True
        else:
            Vs.append(W / H[j + 1, j])
        if on_step is not None and on_step(j, H[:j + 2, :j + 1]):
            stop = True
        if stop:
            return Vs, H[:j + 2, :j + 1], Ws, j + 1
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
    section 5.1) by tubal modified Gram-Schmidt.

    Reading of the garbled loops: for j = 1..s, W = A_j; for i = 1..j-1,
    r_ij = Q_i^T * W and W -= Q_i * r_ij; then [Q_j, r_jj] =
    Normalization(W).  R[i, j, :] is the tube r_ij; R is upper triangular
    in every frontal slice.
    """
    n, s, p = Amat.shape
    Q = np.zeros((n, s, p))
    R = np.zeros((s, s, p))
    for j in range(s):
        W = Amat[:, j:j + 1, :].copy()
        for i in range(j):
            Qi = Q[:, i:i + 1, :]
            rij = tprod(ttrans(Qi), W)                  # 1 x 1 x p
            W = W - tprod(Qi, rij)
            R[i, j, :] = rij.reshape(p)
        Qj, a = normalization(W)
        Q[:, j:j + 1, :] = Qj
        R[j, j, :] = a
    return Q, R


def tba(A, V, m):
    """Tubal Block Arnoldi (Algorithm 7 of section 5.1).

    Reading: W = A * V_j uses A, not M (as printed; B enters only the
    projected equation of TBAS).  Block modified Gram-Schmidt with
    tube-valued coefficients H_ij = V_i^T * W, W -= V_i * H_ij, then
    [V_{j+1}, H_{j+1,j}] = Tubal-QR(W).

    Returns (Vb, Hbig, H0): the blocks V_1..V_{m+1} (each n x s x p), the
    block Hessenberg tensor of size (m+1)s x ms x p, and H0 from
    Tubal-QR(V).
    """
    n, s, p = V.shape
    V1, H0 = tubal_qr(V)
    Vb = [V1]
    Hbig = np.zeros(((m + 1) * s, m * s, p))
    for j in range(m):
        W = tprod(A, Vb[j])
        for i in range(j + 1):
            Hij = tprod(ttrans(Vb[i]), W)
            W = W - tprod(Vb[i], Hij)
            Hbig[i * s:(i + 1) * s, j * s:(j + 1) * s, :] = Hij
        Vn, Hn = tubal_qr(W)
        Vb.append(Vn)
        Hbig[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s, :] = Hn
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
