#include "host_linalg.hpp"

#include <algorithm>
#include <cmath>

namespace tsylv {
namespace host {

namespace {

constexpr double kEps = 2.220446049250313e-16;

inline cplx& at(cplx* A, int ld, int i, int j) { return A[i + (size_t)ld * j]; }
inline const cplx& at(const cplx* A, int ld, int i, int j) { return A[i + (size_t)ld * j]; }

// Givens rotation G = [c s; -conj(s) c] (c real) with G [a; b] = [r; 0].
inline void givens(cplx a, cplx b, double& c, cplx& s) {
  const double aa = std::abs(a), bb = std::abs(b);
  if (bb == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  if (aa == 0.0) {
    c = 0.0;
    s = std::conj(b) / bb;
    return;
  }
  const double r = std::hypot(aa, bb);
  c = aa / r;
  s = (a / aa) * std::conj(b) / r;
}

}  // namespace

bool cholesky_upper(cplx* G, int s, double rel_tol) {
  double dmax = 0.0;
  for (int i = 0; i < s; ++i) dmax = std::max(dmax, std::real(at(G, s, i, i)));
  if (!(dmax > 0.0)) return false;
  for (int j = 0; j < s; ++j) {
    // R(j, j)^2 = G(j, j) - sum_{k<j} |R(k, j)|^2
    double d = std::real(at(G, s, j, j));
    for (int k = 0; k < j; ++k) d -= std::norm(at(G, s, k, j));
    if (!(d > rel_tol * dmax)) return false;
    const double rjj = std::sqrt(d);
    at(G, s, j, j) = rjj;
    // R(j, l) = (G(j, l) - sum_{k<j} conj(R(k, j)) R(k, l)) / R(j, j), l > j
    for (int l = j + 1; l < s; ++l) {
      cplx t = at(G, s, j, l);
      for (int k = 0; k < j; ++k) t -= std::conj(at(G, s, k, j)) * at(G, s, k, l);
      at(G, s, j, l) = t / rjj;
    }
    for (int i = j + 1; i < s; ++i) at(G, s, i, j) = 0.0;
  }
  return true;
}

void tri_inv_upper(const cplx* R, cplx* Ri, int s) {
  for (int i = 0; i < s * s; ++i) Ri[i] = 0.0;
  for (int j = 0; j < s; ++j) {
    at(Ri, s, j, j) = 1.0 / at(R, s, j, j);
    for (int i = j - 1; i >= 0; --i) {
      cplx t = 0.0;
      for (int k = i + 1; k <= j; ++k) t += at(R, s, i, k) * at(Ri, s, k, j);
      at(Ri, s, i, j) = -t / at(R, s, i, i);
    }
  }
}

void matmul(const cplx* A, const cplx* B, cplx* C, int m, int k, int n) {
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < m; ++i) C[i + (size_t)m * j] = 0.0;
    for (int l = 0; l < k; ++l) {
      const cplx b = B[l + (size_t)k * j];
      if (b == cplx(0.0)) continue;
      for (int i = 0; i < m; ++i) C[i + (size_t)m * j] += A[i + (size_t)m * l] * b;
    }
  }
}

bool schur(cplx* A, cplx* U, int n) {
  for (int i = 0; i < n * n; ++i) U[i] = 0.0;
  for (int i = 0; i < n; ++i) at(U, n, i, i) = 1.0;
  // Householder reduction to upper Hessenberg form: A <- P A P, U <- U P.
  std::vector<cplx> v(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    double xn = 0.0;
    for (int i = k + 1; i < n; ++i) xn += std::norm(at(A, n, i, k));
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const cplx x0 = at(A, n, k + 1, k);
    const cplx ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cplx(1.0);
    const cplx alpha = -ph * xn;
    for (int i = k + 1; i < n; ++i) v[i] = at(A, n, i, k);
    v[k + 1] -= alpha;
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = k + 1; i < n; ++i) v[i] /= vn;
    // A <- (I - 2 v v^H) A   (rows k+1..n-1)
    for (int j = 0; j < n; ++j) {
      cplx t = 0.0;
      for (int i = k + 1; i < n; ++i) t += std::conj(v[i]) * at(A, n, i, j);
      t *= 2.0;
      for (int i = k + 1; i < n; ++i) at(A, n, i, j) -= v[i] * t;
    }
    // A <- A (I - 2 v v^H), U <- U (I - 2 v v^H)   (columns k+1..n-1)
    for (cplx* M : {A, U}) {
      for (int i = 0; i < n; ++i) {
        cplx t = 0.0;
        for (int j = k + 1; j < n; ++j) t += at(M, n, i, j) * v[j];
        t *= 2.0;
        for (int j = k + 1; j < n; ++j) at(M, n, i, j) -= t * std::conj(v[j]);
      }
    }
    for (int i = k + 2; i < n; ++i) at(A, n, i, k) = 0.0;
  }
  // Shifted QR iterations on the Hessenberg matrix.
  std::vector<double> cs(n);
  std::vector<cplx> sn(n);
  int hi = n - 1, iter = 0;
  const int max_iter = 100 * std::max(n, 1);
  int total = 0;
  while (hi > 0) {
    if (++total > max_iter) return false;
    int l = hi;
    while (l > 0) {
      const double sub = std::abs(at(A, n, l, l - 1));
      const double dia = std::abs(at(A, n, l - 1, l - 1)) + std::abs(at(A, n, l, l));
      if (sub <= kEps * (dia > 0.0 ? dia : 1.0)) {
        at(A, n, l, l - 1) = 0.0;
        break;
      }
      --l;
    }
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    ++iter;
    // Wilkinson shift: eigenvalue of the trailing 2 x 2 closer to A(hi, hi).
    const cplx a = at(A, n, hi - 1, hi - 1), b = at(A, n, hi - 1, hi);
    const cplx c = at(A, n, hi, hi - 1), d = at(A, n, hi, hi);
    const cplx tr = a + d, det = a * d - b * c;
    const cplx disc = std::sqrt(tr * tr / 4.0 - det);
    cplx mu1 = tr / 2.0 + disc, mu2 = tr / 2.0 - disc;
    cplx mu = (std::abs(mu1 - d) < std::abs(mu2 - d)) ? mu1 : mu2;
    if (iter % 11 == 10) mu = d + std::abs(c);  // exceptional shift
    // QR step on the active window [l, hi]: A - mu I = Q R, A <- R Q + mu I,
    // applied to the whole matrix so that A stays a similarity of the input.
    for (int k = l; k <= hi; ++k) at(A, n, k, k) -= mu;
    for (int k = l; k < hi; ++k) {
      givens(at(A, n, k, k), at(A, n, k + 1, k), cs[k], sn[k]);
      for (int j = k; j < n; ++j) {
        const cplx x = at(A, n, k, j), y = at(A, n, k + 1, j);
        at(A, n, k, j) = cs[k] * x + sn[k] * y;
        at(A, n, k + 1, j) = -std::conj(sn[k]) * x + cs[k] * y;
      }
    }
    for (int k = l; k < hi; ++k) {
      const int rmax = std::min(k + 2, hi + 1);
      for (int i = 0; i < rmax; ++i) {
        const cplx x = at(A, n, i, k), y = at(A, n, i, k + 1);
        at(A, n, i, k) = cs[k] * x + std::conj(sn[k]) * y;
        at(A, n, i, k + 1) = -sn[k] * x + cs[k] * y;
      }
      for (int i = 0; i < n; ++i) {
        const cplx x = at(U, n, i, k), y = at(U, n, i, k + 1);
        at(U, n, i, k) = cs[k] * x + std::conj(sn[k]) * y;
        at(U, n, i, k + 1) = -sn[k] * x + cs[k] * y;
      }
    }
    for (int k = l; k <= hi; ++k) at(A, n, k, k) += mu;
  }
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) at(A, n, i, j) = 0.0;
  return true;
}

bool sylvester_banded(const cplx* H, int ms, int band, const cplx* B, int s, const cplx* C1,
                      cplx* Y) {
  std::vector<cplx> T(B, B + (size_t)s * s), U((size_t)s * s);
  if (!schur(T.data(), U.data(), s)) return false;
  // D = C1 U, Z column by column, Y = Z U^H
  std::vector<cplx> D((size_t)ms * s), Z((size_t)ms * s, 0.0);
  matmul(C1, U.data(), D.data(), ms, s, s);
  std::vector<cplx> M((size_t)ms * ms), r(ms);
  double hmax = 0.0;
  for (size_t i = 0; i < (size_t)ms * ms; ++i) hmax = std::max(hmax, std::abs(H[i]));
  for (int j = 0; j < s; ++j) {
    const cplx t = at(T.data(), s, j, j);
    for (int i = 0; i < ms; ++i) {
      cplx v = at(D.data(), ms, i, j);
      for (int l = 0; l < j; ++l) v += at(Z.data(), ms, i, l) * at(T.data(), s, l, j);
      r[i] = v;
    }
    std::copy(H, H + (size_t)ms * ms, M.begin());
    for (int i = 0; i < ms; ++i) at(M.data(), ms, i, i) -= t;
    // Gaussian elimination with partial pivoting inside the lower band.
    for (int c = 0; c < ms; ++c) {
      const int last = std::min(ms - 1, c + band);
      int piv = c;
      double best = std::abs(at(M.data(), ms, c, c));
      for (int i = c + 1; i <= last; ++i) {
        const double a = std::abs(at(M.data(), ms, i, c));
        if (a > best) {
          best = a;
          piv = i;
        }
      }
      if (!(best > kEps * (hmax + std::abs(t)) * 1e-3)) return false;
      if (piv != c) {
        for (int jj = c; jj < ms; ++jj) std::swap(at(M.data(), ms, c, jj), at(M.data(), ms, piv, jj));
        std::swap(r[c], r[piv]);
      }
      const cplx inv = 1.0 / at(M.data(), ms, c, c);
      for (int i = c + 1; i <= last; ++i) {
        const cplx f = at(M.data(), ms, i, c) * inv;
        if (f == cplx(0.0)) continue;
        at(M.data(), ms, i, c) = 0.0;
        for (int jj = c + 1; jj < ms; ++jj) at(M.data(), ms, i, jj) -= f * at(M.data(), ms, c, jj);
        r[i] -= f * r[c];
      }
    }
    for (int i = ms - 1; i >= 0; --i) {
      cplx v = r[i];
      for (int jj = i + 1; jj < ms; ++jj) v -= at(M.data(), ms, i, jj) * at(Z.data(), ms, jj, j);
      at(Z.data(), ms, i, j) = v / at(M.data(), ms, i, i);
    }
  }
  // Y = Z U^H
  for (int j = 0; j < s; ++j)
    for (int i = 0; i < ms; ++i) {
      cplx v = 0.0;
      for (int l = 0; l < s; ++l) v += at(Z.data(), ms, i, l) * std::conj(at(U.data(), s, j, l));
      at(Y, ms, i, j) = v;
    }
  return true;
}

double eig_from_schur(const cplx* T, const cplx* U, int n, cplx* lam, cplx* W, cplx* Winv) {
  std::vector<cplx> Q((size_t)n * n, 0.0), Qi((size_t)n * n);
  double tmax = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) tmax = std::max(tmax, std::abs(at(T, n, i, j)));
  for (int j = 0; j < n; ++j) {
    lam[j] = at(T, n, j, j);
    at(Q.data(), n, j, j) = 1.0;
    for (int i = j - 1; i >= 0; --i) {
      cplx v = 0.0;
      for (int l = i + 1; l <= j; ++l) v += at(T, n, i, l) * at(Q.data(), n, l, j);
      const cplx d = at(T, n, i, i) - lam[j];
      if (!(std::abs(d) > kEps * tmax)) return INFINITY;  // (nearly) repeated eigenvalue
      at(Q.data(), n, i, j) = -v / d;
    }
    double nrm = 0.0;
    for (int i = 0; i <= j; ++i) nrm += std::norm(at(Q.data(), n, i, j));
    nrm = std::sqrt(nrm);
    for (int i = 0; i <= j; ++i) at(Q.data(), n, i, j) /= nrm;
  }
  tri_inv_upper(Q.data(), Qi.data(), n);
  double nq = 0.0, nqi = 0.0;
  for (size_t e = 0; e < (size_t)n * n; ++e) {
    nq += std::norm(Q[e]);
    nqi += std::norm(Qi[e]);
  }
  matmul(U, Q.data(), W, n, n, n);
  // Winv = Qi U^H
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      cplx v = 0.0;
      for (int l = 0; l < n; ++l) v += at(Qi.data(), n, i, l) * std::conj(at(U, n, j, l));
      at(Winv, n, i, j) = v;
    }
  const double kappa = std::sqrt(nq) * std::sqrt(nqi);
  return std::isfinite(kappa) ? kappa : INFINITY;
}

}  // namespace host
}  // namespace tsylv
