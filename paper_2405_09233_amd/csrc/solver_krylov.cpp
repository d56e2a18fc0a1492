// tGMRES(m) and tFOM(m) -- Algorithm 3 of section 3 -- on the GPU, and the
// mixed-precision iterative refinement built on them.
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
//
// Mixed precision (not in the paper): the restart loop of Algorithm 3 is
// kept in FP64 -- R = C - M(X) with the FP64 Fourier slices, X += d in FP64
// -- while each correction d is one tGMRES(inner_m) cycle on M d = R with
// FP32 basis vectors and the operator applied from FP32 or BF16 copies of
// the Fourier slices (FP32 accumulation); the Hessenberg least-squares
// problem stays FP64.  This is iterative refinement whose inner solver is
// one restart cycle, so it converges like restarted tGMRES as long as the
// low-precision operator error is small against each cycle's reduction.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <functional>
#include <vector>

#include "kernels.hpp"
#include "runtime.hpp"
#include "solvers.hpp"

namespace tsylv {

namespace {

constexpr double kEps = 2.220446049250313e-16;

// The operator M in Fourier planes, in FP64 and (optionally) one low
// precision copy used by the inner solves.
struct Operator {
  int64_t n = 0, s = 0, p = 0;
  const double* Ah64 = nullptr;
  const double* Bh64 = nullptr;
  const float* Ah32 = nullptr;
  const float* Bh32 = nullptr;
  const uint16_t* Ahb = nullptr;
  const uint16_t* Bhb = nullptr;
  int low = TSYLV_FP32;  // precision of the float-vector applies
};

void op_apply(Ctx& ctx, const Operator& op, const double* V, double* out, const double* Y,
              double alpha, double beta) {
  ProfScope ps(ctx, TSYLV_K_APPLY);
  kern::apply_f64(op.Ah64, op.Bh64, V, out, Y, alpha, beta, op.n, op.s, (int)op.p, ctx.stream);
}

void op_apply(Ctx& ctx, const Operator& op, const float* V, float* out, const float* Y,
              double alpha, double beta) {
  ProfScope ps(ctx, TSYLV_K_APPLY_LOW);
  if (op.low == TSYLV_BF16)
    kern::apply_bf16(op.Ahb, op.Bhb, V, out, Y, alpha, beta, op.n, op.s, (int)op.p, ctx.stream);
  else
    kern::apply_f32(op.Ah32, op.Bh32, V, out, Y, alpha, beta, op.n, op.s, (int)op.p, ctx.stream);
}

// Reduction buffers shared by the norm and dot kernels.
struct RedBuf {
  double* part = nullptr;
  int nchunks = 0, ldp = 0;
  double* d_ww = nullptr;
  double* h_ww = nullptr;
};

// ||v||^2 of one FP64 or FP32 vector, to the host.
template <typename TV>
double norm2(Ctx& ctx, const RedBuf& r, const TV* v, int64_t N) {
  kern::mdot_partial((const TV*)nullptr, 0, 0, v, N, r.part, r.ldp, 1, ctx.stream);
  kern::reduce_partials(r.part, r.nchunks, r.ldp, 1, r.d_ww, ctx.stream);
  TSYLV_HIP(hipMemcpyAsync(r.h_ww, r.d_ww, sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  ctx.sync();
  return r.h_ww[0];
}

// Device and pinned buffers of one Arnoldi cycle with basis type TV.
template <typename TV>
struct CycleWS {
  TV* basis = nullptr;
  int64_t ldv = 0;
  int m = 0;
  RedBuf red;
  double *d_h1 = nullptr, *d_h2 = nullptr, *d_y = nullptr;
  double *h_h1 = nullptr, *h_h2 = nullptr, *h_y = nullptr;
  TV* V(int j) const { return basis + (int64_t)j * ldv; }

  static size_t bytes(int64_t N, int m) {
    int64_t ldv = round_up(N, 64);
    int nch = kern::mdot_chunks(N);
    return Workspace::bytes_for((int64_t)(m + 1) * ldv, sizeof(TV)) +
           Workspace::bytes_for((int64_t)nch * (m + 2), 8) + 4 * Workspace::bytes_for(m + 2, 8);
  }
  // host: pinned staging of 4 (m + 2) doubles
  void carve(Workspace& ws, int64_t N, int m_, double* host) {
    m = m_;
    ldv = round_up(N, 64);
    basis = ws.take<TV>((int64_t)(m + 1) * ldv);
    red.nchunks = kern::mdot_chunks(N);
    red.ldp = m + 2;
    red.part = ws.take<double>((int64_t)red.nchunks * red.ldp);
    d_h1 = ws.take<double>(m + 2);
    d_h2 = ws.take<double>(m + 2);
    red.d_ww = ws.take<double>(m + 2);
    d_y = ws.take<double>(m + 2);
    h_h1 = host;
    h_h2 = host + (m + 2);
    red.h_ww = host + 2 * (m + 2);
    h_y = host + 3 * (m + 2);
  }
};

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

struct CycleOut {
  std::vector<double> y;  // coefficients of X += V_k (*) y
  size_t k = 0;           // steps taken
  double est = 0.0;       // last residual estimate (absolute)
  bool fom_fallback = false;
};

// One restart cycle of Algorithm 3 (steps 4(a)-(b)): up to m steps of
// tArnoldi on the normalised start vector in w.V(0), stopping early when the
// residual estimate drops to stop_abs or on a happy breakdown.
template <typename TV>
CycleOut arnoldi_cycle(Ctx& ctx, int method, const Operator& op, CycleWS<TV>& w, int64_t N,
                       double beta, double stop_abs, int m,
                       const std::function<void(double)>& record) {
  hipStream_t st = ctx.stream;
  const RedBuf& r = w.red;
  Givens giv(beta);
  std::vector<std::vector<double>> Hcols;
  std::vector<double> y_fom;
  bool fom_ok = false;
  CycleOut out;
  for (int j = 0; j < m; ++j) {
    const int nv = j + 1;
    TV* W = w.V(j + 1);
    // Algorithm 2 step 3(a): W = M(V_j)
    op_apply(ctx, op, (const TV*)w.V(j), W, (const TV*)nullptr, 1.0, 0.0);
    // step 3(b), CGS2: two passes of h = V^T W, W -= V h
    if (ctx.prof.on()) ctx.prof.begin(TSYLV_K_ORTHO, st);
    kern::mdot_partial((const TV*)w.basis, w.ldv, nv, (const TV*)W, N, r.part, r.ldp, 1, st);
    kern::reduce_partials(r.part, r.nchunks, r.ldp, nv + 1, w.d_h1, st);
    kern::mupdate((const TV*)w.basis, w.ldv, nv, w.d_h1, W, N, st);
    kern::mdot_partial((const TV*)w.basis, w.ldv, nv, (const TV*)W, N, r.part, r.ldp, 0, st);
    kern::reduce_partials(r.part, r.nchunks, r.ldp, nv, w.d_h2, st);
    kern::mupdate((const TV*)w.basis, w.ldv, nv, w.d_h2, W, N, st);
    // step 3(d): h_{j+1,j} = ||W||_F
    kern::mdot_partial((const TV*)nullptr, 0, 0, (const TV*)W, N, r.part, r.ldp, 1, st);
    kern::reduce_partials(r.part, r.nchunks, r.ldp, 1, r.d_ww, st);
    if (ctx.prof.on()) ctx.prof.end(TSYLV_K_ORTHO, st);
    TSYLV_HIP(hipMemcpyAsync(w.h_h1, w.d_h1, (nv + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    TSYLV_HIP(hipMemcpyAsync(w.h_h2, w.d_h2, nv * sizeof(double), hipMemcpyDeviceToHost, st));
    TSYLV_HIP(hipMemcpyAsync(r.h_ww, r.d_ww, sizeof(double), hipMemcpyDeviceToHost, st));
    ctx.sync();
    std::vector<double> h(nv + 1);
    for (int i = 0; i < nv; ++i) h[i] = w.h_h1[i] + w.h_h2[i];
    const double w0 = std::sqrt(w.h_h1[nv]);
    double hn = std::sqrt(r.h_ww[0]);
    const bool breakdown = !(hn > 16.0 * kEps * w0);
    if (breakdown) hn = 0.0;
    h[nv] = hn;
    out.k = (size_t)nv;
    double est;
    if (method == TSYLV_METHOD_GMRES) {
      est = giv.add(h);
    } else {
      giv.add(h);  // keeps the tGMRES fallback available
      Hcols.push_back(h);
      fom_ok = fom_solve(Hcols, out.k, beta, y_fom);
      est = fom_ok ? hn * std::fabs(y_fom[out.k - 1]) : INFINITY;
    }
    out.est = est;
    record(est);
    if (breakdown || est <= stop_abs) break;
    // step 3(e): V_{j+1} = W / h_{j+1,j}
    kern::scale((const TV*)W, W, 1.0 / hn, N, st);
  }
  // Algorithm 3 step 4(b): the small problem.
  if (method == TSYLV_METHOD_GMRES) {
    out.y = giv.solve(out.k);
  } else if (fom_ok) {
    out.y = y_fom;
  } else {
    out.fom_fallback = true;
    out.y = giv.solve(out.k);
  }
  return out;
}

// Adds V_k (*) y to X (Algorithm 3 step 4(c)); X is FP64, V of type TV.
template <typename TV>
void add_combination(Ctx& ctx, CycleWS<TV>& w, const CycleOut& c, double* X, int64_t N) {
  for (size_t i = 0; i < c.k; ++i) w.h_y[i] = -c.y[i];
  TSYLV_HIP(hipMemcpyAsync(w.d_y, w.h_y, c.k * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
  kern::mupdate((const TV*)w.basis, w.ldv, (int)c.k, w.d_y, X, N, ctx.stream);
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

size_t setup_bytes(int64_t n, int64_t s, int64_t p) {
  const int64_t N = n * s * p;
  return Workspace::bytes_for(p * n * n, 8) + Workspace::bytes_for(p * s * s, 8) +
         3 * Workspace::bytes_for(p * p, 8) + 2 * Workspace::bytes_for(N, 8);
}

// Algorithm 1 step 1 for the operator (unscaled DFT planes of A and B) and
// the orthonormal planes of C and X0.
Setup setup_fourier(Ctx& ctx, Workspace& ws, int64_t n, int64_t s, int64_t p, const double* A,
                    const double* B, const double* C, const double* X, bool x0_given) {
  hipStream_t st = ctx.stream;
  const int64_t N = n * s * p;
  Setup S;
  S.Ah = ws.take<double>(p * n * n);
  S.Bh = ws.take<double>(p * s * s);
  S.xf_op = ws.take<double>(p * p);
  S.xf_fwd = ws.take<double>(p * p);
  S.xf_inv = ws.take<double>(p * p);
  S.Zc = ws.take<double>(N);
  S.Zx = ws.take<double>(N);
  kern::build_xform(S.xf_op, (int)p, XF_OPERATOR, st);
  kern::build_xform(S.xf_fwd, (int)p, XF_FORWARD, st);
  kern::build_xform(S.xf_inv, (int)p, XF_INVERSE, st);
  {
    ProfScope ps(ctx, TSYLV_K_XFORM);
    kern::tube_xform_f64(A, S.Ah, S.xf_op, n * n, (int)p, st);
  }
  kern::tube_xform_f64(B, S.Bh, S.xf_op, s * s, (int)p, st);
  kern::tube_xform_f64(C, S.Zc, S.xf_fwd, n * s, (int)p, st);
  if (x0_given)
    kern::tube_xform_f64(X, S.Zx, S.xf_fwd, n * s, (int)p, st);
  else
    TSYLV_HIP(hipMemsetAsync(S.Zx, 0, N * sizeof(double), st));
  return S;
}

size_t krylov_workspace_bytes(int64_t n, int64_t s, int64_t p, const tsylv_opts& o) {
  const int64_t N = n * s * p;
  size_t b = setup_bytes(n, s, p);
  if (!o.refine) return b + CycleWS<double>::bytes(N, o.m);
  b += Workspace::bytes_for(N, 8);  // FP64 residual
  b += CycleWS<float>::bytes(N, o.inner_m);
  if (o.prec == TSYLV_BF16)
    b += Workspace::bytes_for(p * n * n, 2) + Workspace::bytes_for(p * s * s, 2);
  else
    b += Workspace::bytes_for(p * n * n, 4) + Workspace::bytes_for(p * s * s, 4);
  return b;
}

int krylov_solve(Ctx& ctx, int method, int64_t n, int64_t s, int64_t p, const double* A,
                 const double* B, const double* C, double* X, const tsylv_opts& o,
                 tsylv_info& info) {
  auto t0 = std::chrono::steady_clock::now();
  const bool refine = o.refine != 0;
  const int64_t N = n * s * p;
  hipStream_t st = ctx.stream;
  Workspace ws(ctx.arena, krylov_workspace_bytes(n, s, p, o));
  Setup S = setup_fourier(ctx, ws, n, s, p, A, B, C, X, o.x0_given != 0);
  Operator op;
  op.n = n;
  op.s = s;
  op.p = p;
  op.Ah64 = S.Ah;
  op.Bh64 = S.Bh;

  CycleWS<double> w64;
  CycleWS<float> w32;
  double* R64 = nullptr;
  const int m_cycle = refine ? o.inner_m : o.m;
  double* host = ctx.host_buffer(4 * (size_t)(m_cycle + 2));
  if (!refine) {
    w64.carve(ws, N, o.m, host);
  } else {
    R64 = ws.take<double>(N);
    w32.carve(ws, N, o.inner_m, host);
    op.low = o.prec == TSYLV_BF16 ? TSYLV_BF16 : TSYLV_FP32;
    if (op.low == TSYLV_BF16) {
      uint16_t* Ab = ws.take<uint16_t>(p * n * n);
      uint16_t* Bb = ws.take<uint16_t>(p * s * s);
      kern::convert_f64_bf16(S.Ah, Ab, p * n * n, st);
      kern::convert_f64_bf16(S.Bh, Bb, p * s * s, st);
      op.Ahb = Ab;
      op.Bhb = Bb;
    } else {
      float* Af = ws.take<float>(p * n * n);
      float* Bf = ws.take<float>(p * s * s);
      kern::convert_f64_f32(S.Ah, Af, p * n * n, st);
      kern::convert_f64_f32(S.Bh, Bf, p * s * s, st);
      op.Ah32 = Af;
      op.Bh32 = Bf;
    }
  }
  const RedBuf& red = refine ? w32.red : w64.red;

  // ||C||_F (Parseval: the planes of C are orthonormal coordinates)
  const double cnorm = std::sqrt(norm2<double>(ctx, red, S.Zc, N));
  info.steps = info.cycles = info.outer = 0;
  info.relres_est = 0.0;
  info.res_hist_len = 0;
  info.fom_fallback = 0;
  auto record = [&](double est_abs) {
    double est = est_abs / cnorm;
    info.relres_est = est;
    if (o.res_hist && info.res_hist_len < o.res_hist_cap) o.res_hist[info.res_hist_len++] = est;
  };

  if (cnorm == 0.0) {
    TSYLV_HIP(hipMemsetAsync(X, 0, N * sizeof(double), st));
    ctx.sync();
    info.relres_true = 0.0;
    info.status = TSYLV_OK;
    info.seconds = seconds_since(t0);
    return TSYLV_OK;
  }

  int status = TSYLV_NOT_CONVERGED;
  const int max_iter = refine ? o.max_outer : o.max_cycles;
  for (int it = 0;; ++it) {
    // R0 = C - M(X0)  (Algorithm 3, step 3), in FP64.
    double* R = refine ? R64 : w64.V(0);
    if (it == 0 && !o.x0_given)
      TSYLV_HIP(hipMemcpyAsync(R, S.Zc, N * sizeof(double), hipMemcpyDeviceToDevice, st));
    else
      op_apply(ctx, op, (const double*)S.Zx, R, (const double*)S.Zc, -1.0, 1.0);
    const double beta = std::sqrt(norm2<double>(ctx, red, R, N));
    info.relres_true = beta / cnorm;
    if (info.relres_true <= o.tol) {
      status = TSYLV_OK;
      break;
    }
    if (it >= max_iter) break;
    info.cycles++;
    if (!refine) {
      kern::scale((const double*)R, R, 1.0 / beta, N, st);
      CycleOut c = arnoldi_cycle<double>(ctx, method, op, w64, N, beta, o.tol * cnorm, o.m, record);
      info.steps += (int)c.k;
      info.fom_fallback += c.fom_fallback ? 1 : 0;
      add_combination(ctx, w64, c, S.Zx, N);
    } else {
      info.outer++;
      kern::scale((const double*)R, w32.V(0), 1.0 / beta, N, st);  // rounds to FP32
      const double stop = std::max(o.inner_tol * beta, 0.5 * o.tol * cnorm);
      CycleOut c = arnoldi_cycle<float>(ctx, method, op, w32, N, beta, stop, o.inner_m, record);
      info.steps += (int)c.k;
      info.fom_fallback += c.fom_fallback ? 1 : 0;
      add_combination(ctx, w32, c, S.Zx, N);
    }
  }
  // Algorithm 1 step 3: back to the spatial domain.
  {
    ProfScope ps(ctx, TSYLV_K_XFORM);
    kern::tube_xform_f64(S.Zx, X, S.xf_inv, n * s, (int)p, st);
  }
  ctx.sync();
  info.status = status;
  info.seconds = seconds_since(t0);
  return status;
}

// Y = A*X - X*B through the Fourier planes (Algorithm 1), with the slice
// products in the requested precision.
size_t apply_workspace_bytes(int64_t n, int64_t s, int64_t p) {
  int64_t N = n * s * p;
  return Workspace::bytes_for(p * n * n, 8) + Workspace::bytes_for(p * s * s, 8) +
         3 * Workspace::bytes_for(p * p, 8) + 2 * Workspace::bytes_for(N, 8) +
         Workspace::bytes_for(p * n * n, 4) + Workspace::bytes_for(p * s * s, 4) +
         2 * Workspace::bytes_for(N, 4);
}

int apply_spatial(Ctx& ctx, int64_t n, int64_t s, int64_t p, const double* A, const double* B,
                  const double* X, double* Y, int prec) {
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
  if (prec == TSYLV_FP64) {
    ProfScope ps(ctx, TSYLV_K_APPLY);
    kern::apply_f64(Ah, Bh, Zx, Zy, nullptr, 1.0, 0.0, n, s, (int)p, st);
  } else {
    float* Vf = ws.take<float>(N);
    float* Wf = ws.take<float>(N);
    kern::convert_f64_f32(Zx, Vf, N, st);
    if (prec == TSYLV_BF16) {
      uint16_t* Ab = reinterpret_cast<uint16_t*>(ws.take<float>(p * n * n));
      uint16_t* Bb = reinterpret_cast<uint16_t*>(ws.take<float>(p * s * s));
      kern::convert_f64_bf16(Ah, Ab, p * n * n, st);
      kern::convert_f64_bf16(Bh, Bb, p * s * s, st);
      ProfScope ps(ctx, TSYLV_K_APPLY_LOW);
      kern::apply_bf16(Ab, Bb, Vf, Wf, nullptr, 1.0, 0.0, n, s, (int)p, st);
    } else {
      float* Af = ws.take<float>(p * n * n);
      float* Bf = ws.take<float>(p * s * s);
      kern::convert_f64_f32(Ah, Af, p * n * n, st);
      kern::convert_f64_f32(Bh, Bf, p * s * s, st);
      ProfScope ps(ctx, TSYLV_K_APPLY_LOW);
      kern::apply_f32(Af, Bf, Vf, Wf, nullptr, 1.0, 0.0, n, s, (int)p, st);
    }
    kern::convert_f32_f64(Wf, Zy, N, st);
  }
  kern::tube_xform_f64(Zy, Y, xf_inv, n * s, (int)p, st);
  ctx.sync();
  return TSYLV_OK;
}

}  // namespace tsylv
