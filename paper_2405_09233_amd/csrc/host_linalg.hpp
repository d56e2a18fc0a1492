// Small dense complex FP64 linear algebra on the host (no HIP): what the
// Tubal Block Arnoldi driver needs per Fourier slice -- Cholesky factors of
// Gram matrices (Tubal-QR), triangular inverses, a complex Schur
// decomposition and the projected Sylvester solve of TBAS(m).
// All matrices are column-major std::complex<double> arrays.
#pragma once

#include <complex>
#include <vector>

namespace tsylv {
namespace host {

using cplx = std::complex<double>;

// G = R^H R with R upper triangular and real positive diagonal; G (s x s,
// Hermitian, only its upper triangle is read) is overwritten by R (strict
// lower part zeroed).  Returns false if a pivot is not positive relative to
// the largest diagonal entry of G (rank deficiency).
bool cholesky_upper(cplx* G, int s, double rel_tol);

// Rinv = R^{-1} for an upper triangular R (s x s).
void tri_inv_upper(const cplx* R, cplx* Rinv, int s);

// C = A B (m x k times k x n).
void matmul(const cplx* A, const cplx* B, cplx* C, int m, int k, int n);

// Complex Schur decomposition A = U T U^H: A (n x n) is overwritten by the
// upper triangular T, U (n x n) receives the unitary factor.  Householder
// reduction to Hessenberg form, then single-shift QR iterations (Wilkinson
// shifts, deflation on negligible subdiagonals).  Returns false if the QR
// iteration does not converge.
bool schur(cplx* A, cplx* U, int n);

// Solves H Y - Y B = C1 for Y (ms x s), where H (ms x ms) has lower
// bandwidth `band` (block upper Hessenberg with s x s blocks: band = s) and B
// is s x s: Bartels-Stewart with the complex Schur form of B only,
//   B = U T U^H,  Z = Y U,  (H - t_jj I) z_j = (C1 U)_j + sum_{l<j} z_l t_lj,
// each shifted system by Gaussian elimination with partial pivoting inside
// the band.  Returns false if B's Schur form fails or a shifted system is
// singular (the spectra of H and B intersect).
bool sylvester_banded(const cplx* H, int ms, int band, const cplx* B, int s, const cplx* C1,
                      cplx* Y);

// Eigendecomposition B = W diag(lam) W^{-1} from B's complex Schur form
// B = U T U^H: the eigenvectors of the triangular T (back substitution, unit
// 2-norm columns) form an upper triangular Q, W = U Q, W^{-1} = Q^{-1} U^H.
// Returns the condition estimate ||Q||_F ||Q^{-1}||_F (infinite when two
// eigenvalues coincide to working precision); B is not needed, only T, U.
double eig_from_schur(const cplx* T, const cplx* U, int n, cplx* lam, cplx* W, cplx* Winv);

}  // namespace host
}  // namespace tsylv
