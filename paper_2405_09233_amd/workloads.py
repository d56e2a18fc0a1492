"""Seeded synthetic inputs for the T-product Sylvester equation A*X - X*B = C.

This module holds no arithmetic of the solvers: it only draws random
tensors and assembles the finite-difference matrices the workloads are made
of.  Both the GPU path (through the tests and the benchmark) and the FP64
oracle receive the arrays it returns.

Layout: every tensor is a float64 numpy array of shape (rows, cols, p) in
Fortran order, so that its memory is T[i + rows*j + rows*cols*k] -- the
frontal-slice-major layout the C-ABI takes.

Recipes
-------
* ``dense_shifted(n, s, p, seed)`` -- A slices i.i.d. N(0,1) scaled, +4 I on
  slice 1; B slices i.i.d. N(0,1) scaled, -4 I on slice 1; C i.i.d. N(0,1).
  Draw order A, B, C from ``numpy.random.default_rng(seed)`` with each
  tensor filled in Fortran order.  ``noise='literal'`` scales by 1/sqrt(n)
  (resp. 1/sqrt(s)); ``noise='pscaled'`` by 2/sqrt(n p) (resp. 2/sqrt(s p)),
  which keeps the spectra of the Fourier slices of A and B a fixed distance
  apart for every p (the literal recipe lets the slice spectra grow like
  sqrt(p) until they touch).  At p = 4 both are identical.
* ``convection_diffusion(nx, ny, s, p, seed)`` -- A slice 1 = the 5-point
  central-difference matrix of -mu Lap(u) + c . grad(u) on the unit square
  with Dirichlet boundary, an nx x ny interior grid (x fastest), h_x =
  1/(nx+1), h_y = 1/(ny+1), plus 8 I; A slices 2..p dense i.i.d.
  N(0, 1e-4); B slices i.i.d. N(0,1)/sqrt(s), -4 I on slice 1; C i.i.d.
  N(0, 1).  Draw order: A's noise slices, B, C.
* ``ex3(n, s, p, mu, seed)`` -- the convection-diffusion family of the
  paper's experiment (section 6): frontal slice i (i = 1..p) of A is
  mu/h1^2 tridiag(-1, 2, -1) + a_i/(4 h1) T, of B the same with s, h2 and b_i,
  where T is the banded matrix with 1 on the first subdiagonal, 3 on the
  diagonal, -5 on the first and 1 on the second superdiagonal; a_i = i,
  b_i = p + i, h1 = 1/(n+1), h2 = 1/(s+1).  C is uniform on [0, 1) (the
  experiment uses MATLAB's rand; its stream is not reproduced).  The paper
  does not give mu; it is a parameter here.
* ``philox_instance(seed, n, s, p)`` -- the dense p-scaled recipe drawn from
  a counter-based generator, so that the device can make the same instance
  in place (tsylv_generate, and serving requests that carry only a seed).
  Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC'11), key = (seed,
  tensor id) with A = 0, B = 1, C = 2.  Element (i, j, k) of a rows x cols x p
  tensor, e = i + rows j, uses the four words of the block at counter
  (e, floor(k / 4), 0, 0): uniforms u_r = ((w_r >> 12) + 1/2) 2^-52 (exact,
  in (0, 1)), and Box-Muller on (u0, u1) gives k % 4 = 0 (cos) and 1 (sin),
  on (u2, u3) k % 4 = 2 and 3: z = sqrt(-2 log u) cos(2 pi u') resp. sin.
  A = (2/sqrt(n p)) z + 4 I on slice 1, B = (2/sqrt(s p)) z - 4 I on slice 1
  (product rounded, then the shift added), C = z.
"""

import numpy as np


def _normal_tensor(rng, rows, cols, p):
    return rng.standard_normal(rows * cols * p).reshape((rows, cols, p), order="F")


def dense_shifted(n, s, p, seed=0, noise="pscaled", shift=4.0):
    """Dense random operator family with disjoint Fourier-slice spectra."""
    rng = np.random.default_rng(seed)
    if noise == "literal":
        fa, fb = 1.0 / np.sqrt(n), 1.0 / np.sqrt(s)
    elif noise == "pscaled":
        fa, fb = 2.0 / np.sqrt(n * p), 2.0 / np.sqrt(s * p)
    else:
        raise ValueError(noise)
    A = _normal_tensor(rng, n, n, p)
    A *= fa
    A[:, :, 0] += shift * np.eye(n)
    B = _normal_tensor(rng, s, s, p)
    B *= fb
    B[:, :, 0] -= shift * np.eye(s)
    C = _normal_tensor(rng, n, s, p)
    return np.asfortranarray(A), np.asfortranarray(B), np.asfortranarray(C)


def cd5_matrix(nx, ny, mu=1.0, c=(10.0, 10.0), hx=None, hy=None):
    """Dense 5-point matrix of -mu Lap(u) + c . grad(u), Dirichlet boundary,
    lexicographic numbering with x fastest.  Diagonal 2 mu/hx^2 + 2 mu/hy^2;
    x-neighbours -mu/hx^2 -/+ c_x/(2 hx) (west -, east +); likewise in y."""
    hx = 1.0 / (nx + 1) if hx is None else hx
    hy = 1.0 / (ny + 1) if hy is None else hy
    n = nx * ny
    M = np.zeros((n, n))
    d = 2 * mu / hx ** 2 + 2 * mu / hy ** 2
    w, e = -mu / hx ** 2 - c[0] / (2 * hx), -mu / hx ** 2 + c[0] / (2 * hx)
    so, no = -mu / hy ** 2 - c[1] / (2 * hy), -mu / hy ** 2 + c[1] / (2 * hy)
    for iy in range(ny):
        for ix in range(nx):
            r = ix + nx * iy
            M[r, r] = d
            if ix > 0:
                M[r, r - 1] = w
            if ix < nx - 1:
                M[r, r + 1] = e
            if iy > 0:
                M[r, r - nx] = so
            if iy < ny - 1:
                M[r, r + nx] = no
    return M


def convection_diffusion(nx, ny, s, p, seed=0, mu=1.0, c=(10.0, 10.0),
                         noise_std=1e-2, shift=8.0):
    """Convection-diffusion operator family (see the module docstring)."""
    rng = np.random.default_rng(seed)
    n = nx * ny
    A = np.empty((n, n, p), order="F")
    A[:, :, 0] = cd5_matrix(nx, ny, mu, c) + shift * np.eye(n)
    if p > 1:
        noise = rng.standard_normal(n * n * (p - 1)).reshape((n, n, p - 1), order="F")
        noise *= noise_std
        A[:, :, 1:] = noise
        del noise
    B = _normal_tensor(rng, s, s, p)
    B *= 1.0 / np.sqrt(s)
    B[:, :, 0] -= 4.0 * np.eye(s)
    C = _normal_tensor(rng, n, s, p)
    return A, np.asfortranarray(B), np.asfortranarray(C)


# Named workloads ---------------------------------------------------------

def tiny_dense(seed=0):
    """8 x 8 x 4 operator, 6 x 6 x 4 right factor, unrestarted tGMRES."""
    return dense_shifted(8, 6, 4, seed=seed, noise="literal")


def cd_4096(seed=0):
    """n = 4096 (64 x 64 grid, h = 1/65), s = 64, p = 32, dense FP64."""
    return convection_diffusion(64, 64, 64, 32, seed=seed)


def cd_8192(seed=0):
    """n = 8192 (128 x 64 grid), s = 128, p = 64 (34 GB of FP64 A)."""
    return convection_diffusion(128, 64, 128, 64, seed=seed)


def _ex3_slice(size, h, mu, coef):
    """mu/h^2 tridiag(-1, 2, -1) + coef/(4 h) T (T: 1 / 3 / -5 / 1 on the
    sub-, main, first and second super-diagonal)."""
    M = np.zeros((size, size))
    i = np.arange(size)
    M[i, i] = 2.0 * mu / h ** 2 + 3.0 * coef / (4.0 * h)
    M[i[1:], i[:-1]] = -mu / h ** 2 + 1.0 * coef / (4.0 * h)
    M[i[:-1], i[1:]] = -mu / h ** 2 - 5.0 * coef / (4.0 * h)
    M[i[:-2], i[2:]] = 1.0 * coef / (4.0 * h)
    return M


def ex3(n, s, p, mu=1.0, seed=0):
    """The paper's convection-diffusion experiment family (see the module
    docstring); Table 1 uses n in {1000, 2000}, s = 3, p = 2."""
    rng = np.random.default_rng(seed)
    h1, h2 = 1.0 / (n + 1), 1.0 / (s + 1)
    A = np.empty((n, n, p), order="F")
    B = np.empty((s, s, p), order="F")
    for i in range(1, p + 1):
        A[:, :, i - 1] = _ex3_slice(n, h1, mu, float(i))
        B[:, :, i - 1] = _ex3_slice(s, h2, mu, float(p + i))
    C = rng.random(n * s * p).reshape((n, s, p), order="F")
    return A, B, np.asfortranarray(C)


# ------------------------------------------------------------ counter-based

_PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)  # round multipliers
_PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)  # key schedule (Weyl)
_M32 = np.uint64(0xFFFFFFFF)


def _mulhilo64(a, m):
    """(high, low) 64-bit halves of the 128-bit product of uint64 array `a`
    and the constant `m`, from 32-bit partial products."""
    a0, a1 = a & _M32, a >> np.uint64(32)
    m0, m1 = np.uint64(m & 0xFFFFFFFF), np.uint64(m >> 32)
    p00, p01, p10, p11 = a0 * m0, a0 * m1, a1 * m0, a1 * m1
    mid = (p00 >> np.uint64(32)) + (p01 & _M32) + (p10 & _M32)
    hi = p11 + (p01 >> np.uint64(32)) + (p10 >> np.uint64(32)) + (mid >> np.uint64(32))
    lo = a * np.uint64(m)
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds=10):
    """Philox4x64-`rounds` on uint64 counter arrays (c0..c3) under the key
    (k0, k1); returns the four output word arrays."""
    c = [np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3)]
    k = [int(k0) & (2**64 - 1), int(k1) & (2**64 - 1)]
    with np.errstate(over="ignore"):
        for _ in range(rounds):
            hi0, lo0 = _mulhilo64(c[0], _PHILOX_M[0])
            hi1, lo1 = _mulhilo64(c[2], _PHILOX_M[1])
            c = [hi1 ^ c[1] ^ np.uint64(k[0]), lo1, hi0 ^ c[3] ^ np.uint64(k[1]), lo0]
            k = [(k[0] + _PHILOX_W[0]) & (2**64 - 1), (k[1] + _PHILOX_W[1]) & (2**64 - 1)]
    return c


def philox_normal_tensor(seed, tensor_id, rows, cols, p):
    """N(0,1) tensor (rows, cols, p), Fortran order, from the counter-based
    stream described in the module docstring."""
    E = rows * cols
    out = np.empty((E, p), order="F")
    e = np.arange(E, dtype=np.uint64)
    zero = np.zeros(E, dtype=np.uint64)
    for kb in range((p + 3) // 4):
        w = philox4x64(e, np.full(E, kb, dtype=np.uint64), zero, zero, seed, tensor_id)
        u = [((x >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0**-52 for x in w]
        for half in range(2):
            r = np.sqrt(-2.0 * np.log(u[2 * half]))
            t = 2.0 * np.pi * u[2 * half + 1]
            for trig, k in ((np.cos, 4 * kb + 2 * half), (np.sin, 4 * kb + 2 * half + 1)):
                if k < p:
                    out[:, k] = r * trig(t)
    return out.reshape((rows, cols, p), order="F")


def philox_instance(seed, n, s, p, shift=4.0):
    """The dense p-scaled instance of `seed` drawn from the counter-based
    stream (the instance tsylv_generate writes on the device)."""
    A = philox_normal_tensor(seed, 0, n, n, p) * (2.0 / np.sqrt(n * p))
    A[:, :, 0] += shift * np.eye(n)
    B = philox_normal_tensor(seed, 1, s, s, p) * (2.0 / np.sqrt(s * p))
    B[:, :, 0] -= shift * np.eye(s)
    C = philox_normal_tensor(seed, 2, n, s, p)
    return np.asfortranarray(A), np.asfortranarray(B), np.asfortranarray(C)
