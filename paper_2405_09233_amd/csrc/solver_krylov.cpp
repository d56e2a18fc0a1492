// tGMRES(m) and tFOM(m): Algorithm 3 of section 3, on the GPU.
//
// Representation.  Every vector of the Krylov process (C, R, V_j, X) is kept
// in the orthonormal real Fourier representation: tube-wise, the half
// spectrum of the mode-3 DFT stored as p real planes, slice k scaled by
// sqrt(w_k / p) (w_k = 1 for the real DC/Nyquist slices, 2 otherwise).  That
// map is an orthogonal transformation of R^{nsp} (Parseval), so
//   * the inner product and Frobenius norm of section 2.1 are the plain dot
//     product and 2-norm of the stored reals, and
//   * M(X) = A*X - X*B acts slice by slice as Ahat_k V_k - V_k Bhat_k
//     (eq. (2) through Algorithm 1: the scaling commutes with the
//     slice-wise products),
// so tArnoldi (Algorithm 2) runs unchanged on the stored vectors and builds
// the same Hessenberg matrix as it would in the spatial domain.  The DFT is
// applied once to A, B, C (and X0) at the start and its inverse once to X at
// the end.
//
// Orthogonalisation: classical Gram-Schmidt with one full
// re-orthogonalisation (CGS2) instead of the printed modified Gram-Schmidt;
// both produce the same h_{ij} in exact arithmetic and CGS2 needs one
// reduction per pass instead of one per basis vector.
//
// Small problems stay on the host in FP64: progressive Givens QR of the
// Hessenberg matrix for tGMRES (residual proposition of section 3.3,
// ||R_j|| = |gamma_{j+1}|), LU with partial pivoting of H_j for tFOM
// (section 3.2, ||R_j|| = h_{j+1,j} |y_j|).
#include <chrono>
#include <cmath>
#include <vector>

#include "kernels.hpp"
#include "runtime.hpp"
#include "solvers.hpp"

namespace tsylv {

namespace {

constexpr double kEps = 2.220446049250313e-16;

struct KrylovPlan {
  int64_t n, s, p, N, ldv;
  int m;
  int nchunks, ldp;
  size_t bytes;
};

KrylovPlan plan_krylov(int64_t n, int64_t s, int64_t p, int m) {
  KrylovPlan P;
  P.n = n;
  P.s = s;
  P.p = p;
  P.N = n * s * p;
  P.ldv = round_up(P.N, 64);
  P.m = m;
  P.nchunks = kern::mdot_chunks(P.N);
  P.ldp = m + 2;
  size_t b = 0;
  b += Workspace::bytes_for(p * n * n, 8);       // Ah
  b += Workspace::bytes_for(p * s * s, 8);       // Bh
  b += 3 * Workspace::bytes_for(p * p, 8);       // transforms
  b += 2 * Workspace::bytes_for(P.N, 8);         // Zc, Zx
  b += Workspace::bytes_for((int64_t)(m + 1) * P.ldv, 8);  // basis
  b += Workspace::bytes_for((int64_t)P.nchunks * P.ldp, 8);  // partials
  b += 4 * Workspace::bytes_for(m + 2, 8);       // h1, h2, ww, y
  P.bytes = b;
  return P;
}

// Progressive Givens QR of the (j+1) x j Hessenberg matrix (tGMRES).
struct Givens {
  std::vector<double> c, s, g;
  std::vector<std::vector<double>> R;  // R[j] = column j (j+1 entries)
  explicit Givens(double beta) { g.push_back(beta); }
  // Adds column h[0..j+1] (j = current size) and returns |gamma_{j+2}|.
  double add(std::vector<double> h) {
    const size_t j = R.size();
    for (size_t i = 0; i < j; ++i) {
      double a = h[i], b = h[i + 1];
      h[i] = c[i] * a + s[i] * b;
      h[i + 1] = -s[i] * a + c[i] * b;
    }
    double a = h[j], b = h[j + 1];
    double r = std::hypot(a, b);
    double cj = 1.0, sj = 0.0;
    if (r != 0.0) {
      cj = a / r;
      sj = b / r;
    }
    c.push_back(cj);
    s.push_back(sj);
    h[j] = r;
    h.resize(j + 1);
    R.push_back(h);
    double gj = g[j];
    g[j] = cj * gj;
    g.push_back(-sj * gj);
    return std::fabs(g[j + 1]);
  }
  // Back substitution R y = g[0..k).
  std::vector<double> solve(size_t k) const {
    std::vector<double> y(k, 0.0);
    for (size_t ii = k; ii-- > 0;) {
      double t = g[ii];
      for (size_t l = ii + 1; l < k; ++l) t -= R[l][ii] * y[l];
      if (R[ii][ii] == 0.0) throw Error(TSYLV_ESINGULAR, "tGMRES: singular triangular factor");
      y[ii] = t / R[ii][ii];
    }
    return y;
  }
};

// LU with partial pivoting of the k x k upper-left block of H (column store),
// solving H y = beta e1.  Returns false if singular.
bool fom_solve(const std::vector<std::vector<double>>& Hcols, size_t k, double beta,
               std::vector<double>& y) {
  std::vector<double> M(k * k);
  for (size_t j = 0; j < k; ++j)
    for (size_t i = 0; i < k; ++i) M[i + k * j] = (i < Hcols[j].size()) ? Hcols[j][i] : 0.0;
  std::vector<double> b(k, 0.0);
  b[0] = beta;
  for (size_t col = 0; col < k; ++col) {
    size_t piv = col;
    double best = std::fabs(M[col + k * col]);
    for (size_t i = col + 1; i < k; ++i)
      if (std::fabs(M[i + k * col]) > best) {
        best = std::fabs(M[i + k * col]);
        piv = i;
      }
    if (best == 0.0) return false;
    if (piv != col) {
      for (size_t jj = 0; jj < k; ++jj) std::swap(M[col + k * jj], M[piv + k * jj]);
      std::swap(b[col], b[piv]);
    }
    for (size_t i = col + 1; i < k; ++i) {
      double f = M[i + k * col] / M[col + k * col];
      if (f == 0.0) continue;
      for (size_t jj = col; jj < k; ++jj) M[i + k * jj] -= f * M[col + k * jj];
      b[i] -= f * b[col];
    }
  }
  y.assign(k, 0.0);
  for (size_t ii = k; ii-- > 0;) {
    double t = b[ii];
    for (size_t jj = ii + 1; jj < k; ++jj) t -= M[ii + k * jj] * y[jj];
    y[ii] = t / M[ii + k * ii];
  }
  for (double v : y)
    if (!std::isfinite(v)) return false;
  return true;
}

}  // namespace

size_t krylov_workspace_bytes(int64_t n, int64_t s, int64_t p, int m) {
  return plan_krylov(n, s, p, m).bytes;
}

int krylov_solve(Ctx& ctx, int method, int64_t n, int64_t s, int64_t p, const double* A,
                 const double* B, const double* C, double* X, const tsylv_opts& o,
                 tsylv_info& info) {
  auto t0 = std::chrono::steady_clock::now();
  const int m = o.m;
  const KrylovPlan P = plan_krylov(n, s, p, m);
  hipStream_t st = ctx.stream;
  Workspace ws(ctx.arena, P.bytes);
  double* Ah = ws.take<double>(p * n * n);
  double* Bh = ws.take<double>(p * s * s);
  double* xf_op = ws.take<double>(p * p);
  double* xf_fwd = ws.take<double>(p * p);
  double* xf_inv = ws.take<double>(p * p);
  double* Zc = ws.take<double>(P.N);
  double* Zx = ws.take<double>(P.N);
  double* basis = ws.take<double>((int64_t)(m + 1) * P.ldv);
  double* part = ws.take<double>((int64_t)P.nchunks * P.ldp);
  double* d_h1 = ws.take<double>(m + 2);
  double* d_h2 = ws.take<double>(m + 2);
  double* d_ww = ws.take<double>(m + 2);
  double* d_y = ws.take<double>(m + 2);
  double* hbuf = ctx.host_buffer(4 * (size_t)(m + 2));
  double* h_h1 = hbuf;
  double* h_h2 = hbuf + (m + 2);
  double* h_ww = hbuf + 2 * (m + 2);
  double* h_y = hbuf + 3 * (m + 2);
  const int64_t N = P.N;
  auto V = [&](int j) { return basis + (int64_t)j * P.ldv; };

  // ||w||^2 of one vector, to the host.
  auto norm2 = [&](const double* w) {
    kern::mdot_partial(nullptr, 0, 0, w, N, part, P.ldp, 1, st);
    kern::reduce_partials(part, P.nchunks, P.ldp, 1, d_ww, st);
    TSYLV_HIP(hipMemcpyAsync(h_ww, d_ww, sizeof(double), hipMemcpyDeviceToHost, st));
    ctx.sync();
    return h_ww[0];
  };

  // Setup: Fourier planes of A, B (operator) and C, X0 (vectors), Algorithm 1 step 1.
  kern::build_xform(xf_op, (int)p, XF_OPERATOR, st);
  kern::build_xform(xf_fwd, (int)p, XF_FORWARD, st);
  kern::build_xform(xf_inv, (int)p, XF_INVERSE, st);
  {
    ProfScope ps(ctx, TSYLV_K_XFORM);
    kern::tube_xform_f64(A, Ah, xf_op, n * n, (int)p, st);
  }
  kern::tube_xform_f64(B, Bh, xf_op, s * s, (int)p, st);
  kern::tube_xform_f64(C, Zc, xf_fwd, n * s, (int)p, st);
  if (o.x0_given)
    kern::tube_xform_f64(X, Zx, xf_fwd, n * s, (int)p, st);
  else
    TSYLV_HIP(hipMemsetAsync(Zx, 0, N * sizeof(double), st));

  const double cnorm = std::sqrt(norm2(Zc));
  info.steps = info.cycles = 0;
  info.relres_est = 0.0;
  info.res_hist_len = 0;
  info.fom_fallback = 0;
  auto record = [&](double est) {
    info.relres_est = est;
    if (o.res_hist && info.res_hist_len < o.res_hist_cap) o.res_hist[info.res_hist_len++] = est;
  };

  int status = TSYLV_NOT_CONVERGED;
  if (cnorm == 0.0) {
    TSYLV_HIP(hipMemsetAsync(X, 0, N * sizeof(double), st));
    ctx.sync();
    info.relres_true = 0.0;
    info.status = TSYLV_OK;
    info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return TSYLV_OK;
  }

  for (int cycle = 0;; ++cycle) {
    // R0 = C - M(X0)  (Algorithm 3, step 3), into basis slot 0.
    if (cycle == 0 && !o.x0_given)
      TSYLV_HIP(hipMemcpyAsync(V(0), Zc, N * sizeof(double), hipMemcpyDeviceToDevice, st));
    else
      {
        ProfScope ps(ctx, TSYLV_K_APPLY);
        kern::apply_f64(Ah, Bh, Zx, V(0), Zc, -1.0, 1.0, n, s, (int)p, st);
      }
    const double beta = std::sqrt(norm2(V(0)));
    info.relres_true = beta / cnorm;
    if (info.relres_true <= o.tol) {
      status = TSYLV_OK;
      break;
    }
    if (cycle >= o.max_cycles) break;
    info.cycles++;
    kern::scale(V(0), V(0), 1.0 / beta, N, st);

    Givens giv(beta);
    std::vector<std::vector<double>> Hcols;
    std::vector<double> y_fom;
    size_t k = 0;
    bool fom_ok = false;
    for (int j = 0; j < m; ++j) {
      const int nv = j + 1;
      double* W = V(j + 1);
      // Algorithm 2 step 3(a): W = M(V_j)
      {
        ProfScope ps(ctx, TSYLV_K_APPLY);
        kern::apply_f64(Ah, Bh, V(j), W, nullptr, 1.0, 0.0, n, s, (int)p, st);
      }
      // step 3(b), CGS2: two passes of h = V^T W, W -= V h
      if (ctx.prof.on()) ctx.prof.begin(TSYLV_K_ORTHO, st);
      kern::mdot_partial(basis, P.ldv, nv, W, N, part, P.ldp, 1, st);
      kern::reduce_partials(part, P.nchunks, P.ldp, nv + 1, d_h1, st);
      kern::mupdate(basis, P.ldv, nv, d_h1, W, N, st);
      kern::mdot_partial(basis, P.ldv, nv, W, N, part, P.ldp, 0, st);
      kern::reduce_partials(part, P.nchunks, P.ldp, nv, d_h2, st);
      kern::mupdate(basis, P.ldv, nv, d_h2, W, N, st);
      // step 3(d): h_{j+1,j} = ||W||_F
      kern::mdot_partial(nullptr, 0, 0, W, N, part, P.ldp, 1, st);
      kern::reduce_partials(part, P.nchunks, P.ldp, 1, d_ww, st);
      if (ctx.prof.on()) ctx.prof.end(TSYLV_K_ORTHO, st);
      TSYLV_HIP(hipMemcpyAsync(h_h1, d_h1, (nv + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
      TSYLV_HIP(hipMemcpyAsync(h_h2, d_h2, nv * sizeof(double), hipMemcpyDeviceToHost, st));
      TSYLV_HIP(hipMemcpyAsync(h_ww, d_ww, sizeof(double), hipMemcpyDeviceToHost, st));
      ctx.sync();
      info.steps++;
      std::vector<double> h(nv + 1);
      for (int i = 0; i < nv; ++i) h[i] = h_h1[i] + h_h2[i];
      const double w0 = std::sqrt(h_h1[nv]);
      double hn = std::sqrt(h_ww[0]);
      bool breakdown = !(hn > 16.0 * kEps * w0);
      if (breakdown) hn = 0.0;
      h[nv] = hn;
      k = (size_t)nv;
      double est;
      if (method == TSYLV_METHOD_GMRES) {
        est = giv.add(h);
      } else {
        giv.add(h);  // keeps the tGMRES fallback available
        Hcols.push_back(h);
        fom_ok = fom_solve(Hcols, k, beta, y_fom);
        est = fom_ok ? hn * std::fabs(y_fom[k - 1]) : INFINITY;
      }
      record(est / cnorm);
      if (breakdown || est <= o.tol * cnorm) break;
      // step 3(e): V_{j+1} = W / h_{j+1,j}
      kern::scale(W, W, 1.0 / hn, N, st);
    }
    // Algorithm 3 step 4(b)-(c): small problem, X = X0 + V_k (*) y.
    std::vector<double> y;
    if (method == TSYLV_METHOD_GMRES) {
      y = giv.solve(k);
    } else if (fom_ok) {
      y = y_fom;
    } else {
      info.fom_fallback++;
      y = giv.solve(k);
    }
    for (size_t i = 0; i < k; ++i) h_y[i] = -y[i];
    TSYLV_HIP(hipMemcpyAsync(d_y, h_y, k * sizeof(double), hipMemcpyHostToDevice, st));
    kern::mupdate(basis, P.ldv, (int)k, d_y, Zx, N, st);
  }
  // Algorithm 1 step 3: back to the spatial domain.
  kern::tube_xform_f64(Zx, X, xf_inv, n * s, (int)p, st);
  ctx.sync();
  info.status = status;
  info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return status;
}

// Y = A*X - X*B through the Fourier planes (Algorithm 1).
size_t apply_workspace_bytes(int64_t n, int64_t s, int64_t p) {
  int64_t N = n * s * p;
  return Workspace::bytes_for(p * n * n, 8) + Workspace::bytes_for(p * s * s, 8) +
         3 * Workspace::bytes_for(p * p, 8) + 2 * Workspace::bytes_for(N, 8);
}

int apply_spatial(Ctx& ctx, int64_t n, int64_t s, int64_t p, const double* A, const double* B,
                  const double* X, double* Y) {
  hipStream_t st = ctx.stream;
  const int64_t N = n * s * p;
  Workspace ws(ctx.arena, apply_workspace_bytes(n, s, p));
  double* Ah = ws.take<double>(p * n * n);
  double* Bh = ws.take<double>(p * s * s);
  double* xf_op = ws.take<double>(p * p);
  double* xf_fwd = ws.take<double>(p * p);
  double* xf_inv = ws.take<double>(p * p);
  double* Zx = ws.take<double>(N);
  double* Zy = ws.take<double>(N);
  kern::build_xform(xf_op, (int)p, XF_OPERATOR, st);
  kern::build_xform(xf_fwd, (int)p, XF_FORWARD, st);
  kern::build_xform(xf_inv, (int)p, XF_INVERSE, st);
  kern::tube_xform_f64(A, Ah, xf_op, n * n, (int)p, st);
  kern::tube_xform_f64(B, Bh, xf_op, s * s, (int)p, st);
  kern::tube_xform_f64(X, Zx, xf_fwd, n * s, (int)p, st);
  kern::apply_f64(Ah, Bh, Zx, Zy, nullptr, 1.0, 0.0, n, s, (int)p, st);
  kern::tube_xform_f64(Zy, Y, xf_inv, n * s, (int)p, st);
  ctx.sync();
  return TSYLV_OK;
}

}  // namespace tsylv
