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
//
// The solve is a resumable state machine (krylov_task.hpp): SETUP (DFTs,
// ||C||), RESTART (X += V y of the last cycle, R = C - M(X), ||R||), STEP
// (one Arnoldi step), FINAL (inverse DFT).  Each phase enqueues its kernels
// and one small device-to-host copy; the host logic runs after the stream
// is synchronised.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "krylov_task.hpp"
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
  uint16_t* Vtb = nullptr;  // scratch: the BF16 apply's tiled copy of V
  int low = TSYLV_FP32;  // precision of the float-vector applies
  int var64 = -1, var_low = -1;  // tile variants (-1: the default for s)
};

// Reduction buffers shared by the norm and dot kernels.
struct RedBuf {
  double* part = nullptr;
  int nchunks = 0, ldp = 0;
  double* d_ww = nullptr;
  double* h_ww = nullptr;
};

// Device and pinned buffers of one Arnoldi cycle with basis type TV.
template <typename TV>
struct CycleWS {
  TV* basis = nullptr;
  int64_t len = 0;  // elements per vector (the tiled length for BF16 vectors)
  int64_t ldv = 0;
  int m = 0;
  RedBuf red;
  double *d_h1 = nullptr, *d_h2 = nullptr, *d_y = nullptr, *d_sigma = nullptr;
  double *h_h1 = nullptr, *h_h2 = nullptr, *h_y = nullptr, *h_sigma = nullptr;
  // device-driven cycles: the Hessenberg columns (ldh = m + 2 per column),
  // the pending first projection and [w2prev, breakdown round], with their
  // pinned copies (H and scal side by side so one copy returns both)
  double *d_H = nullptr, *d_h1p = nullptr, *d_scal = nullptr;
  double *h_H = nullptr, *h_scal = nullptr;
  TV* V(int j) const { return basis + (int64_t)j * ldv; }
  int ldh() const { return m + 2; }
  static int64_t hess_len(int m) { return (int64_t)(m + 2) * (m + 1) + 2; }

  // sigma (m + 2) followed by the update coefficients of the delayed sweeps
  static int64_t coef_len(int m) { return 3 * (int64_t)(m + 2) + 2; }
  static size_t bytes(int64_t N, int m, bool device_cycle = false) {
    int64_t ldv = round_up(N, 64);
    int nch = kern::mdot_chunks(N);
    return Workspace::bytes_for((int64_t)(m + 1) * ldv, sizeof(TV)) +
           Workspace::bytes_for((int64_t)nch * (2 * m + 4), 8) +
           Workspace::bytes_for(3 * (m + 2), 8) + Workspace::bytes_for(m + 2, 8) +
           Workspace::bytes_for(coef_len(m), 8) +
           (device_cycle ? Workspace::bytes_for(hess_len(m), 8) +
                               Workspace::bytes_for(m + 2, 8)
                         : 0);
  }
  // host: pinned staging of 7 (m + 2) + 2 doubles, plus hess_len(m) for a
  // device-driven cycle
  void carve(Workspace& ws, int64_t N, int m_, double* host, bool device_cycle = false) {
    m = m_;
    len = N;
    ldv = round_up(N, 64);
    basis = ws.take<TV>((int64_t)(m + 1) * ldv);
    red.nchunks = kern::mdot_chunks(N);  // >= ortho_chunks(N)
    red.ldp = 2 * m + 4;                 // up to 2 nv + 3 sums per chunk
    red.part = ws.take<double>((int64_t)red.nchunks * red.ldp);
    // h1, h2 and ||w||^2 side by side on both ends, so one copy returns them
    d_h1 = ws.take<double>(3 * (m + 2));
    d_h2 = d_h1 + (m + 2);
    red.d_ww = d_h1 + 2 * (m + 2);
    d_y = ws.take<double>(m + 2);
    d_sigma = ws.take<double>(coef_len(m));
    h_h1 = host;
    h_h2 = host + (m + 2);
    red.h_ww = host + 2 * (m + 2);
    h_y = host + 3 * (m + 2);
    h_sigma = host + 4 * (m + 2);
    if (device_cycle) {
      d_H = ws.take<double>(hess_len(m));
      d_scal = d_H + (int64_t)(m + 2) * (m + 1);
      d_h1p = ws.take<double>(m + 2);
      h_H = host + 7 * (m + 2) + 2;
      h_scal = h_H + (int64_t)(m + 2) * (m + 1);
    }
  }
};

// Progressive Givens QR of the (j+1) x j Hessenberg matrix (tGMRES).
struct Givens {
  std::vector<double> c, s, g;
  std::vector<std::vector<double>> R;  // R[j] = column j (j+1 entries)
  void reset(double beta) {
    c.clear();
    s.clear();
    R.clear();
    g.assign(1, beta);
  }
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

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// ---------------------------------------------------------------------------
// Fourier setup shared with the TBA driver
// ---------------------------------------------------------------------------

size_t setup_bytes(int64_t n, int64_t s, int64_t p) {
  const int64_t N = n * s * p;
  return Workspace::bytes_for(p * n * n, 8) + Workspace::bytes_for(p * s * s, 8) +
         3 * Workspace::bytes_for(p * p, 8) + 2 * Workspace::bytes_for(N, 8);
}

// Algorithm 1 step 1 for the operator (unscaled DFT planes of A and B) and
// the orthonormal planes of C and X0.
kern::GenTensor gen_instance(uint64_t seed, int which, int64_t n, int64_t s, int64_t p) {
  kern::GenTensor g;
  g.seed = seed;
  g.id = (uint64_t)which;
  if (which == 0) {
    g.rows = n;
    g.scale = 2.0 / std::sqrt((double)(n * p));
    g.shift = 4.0;
  } else if (which == 1) {
    g.rows = s;
    g.scale = 2.0 / std::sqrt((double)(s * p));
    g.shift = -4.0;
  } else {
    g.rows = n;
    g.scale = 1.0;
    g.shift = 0.0;
  }
  return g;
}

Setup setup_fourier(Ctx& ctx, hipStream_t st, bool profile, Workspace& ws, int64_t n, int64_t s,
                    int64_t p, const double* A, const double* B, const double* C, const double* X,
                    bool x0_given, const uint64_t* gen) {
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
  if (gen) {
    {
      ProfScope ps(ctx, TSYLV_K_XFORM, st, profile);
      kern::tube_xform_gen_f64(gen_instance(*gen, 0, n, s, p), S.Ah, S.xf_op, n * n, (int)p, st);
    }
    kern::tube_xform_gen_f64(gen_instance(*gen, 1, n, s, p), S.Bh, S.xf_op, s * s, (int)p, st);
    kern::tube_xform_gen_f64(gen_instance(*gen, 2, n, s, p), S.Zc, S.xf_fwd, n * s, (int)p, st);
  } else {
    {
      ProfScope ps(ctx, TSYLV_K_XFORM, st, profile);
      kern::tube_xform_f64(A, S.Ah, S.xf_op, n * n, (int)p, st);
    }
    kern::tube_xform_f64(B, S.Bh, S.xf_op, s * s, (int)p, st);
    kern::tube_xform_f64(C, S.Zc, S.xf_fwd, n * s, (int)p, st);
  }
  if (x0_given)
    kern::tube_xform_f64(X, S.Zx, S.xf_fwd, n * s, (int)p, st);
  else
    TSYLV_HIP(hipMemsetAsync(S.Zx, 0, N * sizeof(double), st));
  return S;
}

// The fused Gram-Schmidt kernels take the whole cycle's basis at once.
static bool fused_cycle(const tsylv_opts& o) {
  return (o.refine ? o.inner_m : o.m) + 1 <= kern::ortho_max_vectors(o.refine != 0);
}

// BF16-refined solves keep their inner basis as tiled BF16 vectors (the
// layout the BF16 apply reads), halving the Gram-Schmidt traffic; with the
// fused kernels only.  TSYLV_BF16_BASIS=fp32 keeps FP32 vectors instead.
static bool bf16_basis(const tsylv_opts& o) {
  if (!o.refine || o.prec != TSYLV_BF16 || !fused_cycle(o)) return false;
  const char* f = std::getenv("TSYLV_BF16_BASIS");
  return !(f && std::strcmp(f, "fp32") == 0);
}

// Delayed CGS2 (two sweeps per step) unless TSYLV_KRYLOV_CGS2=1 forces the
// three-sweep form.
static bool delayed_cgs2(const tsylv_opts& o) {
  const char* f = std::getenv("TSYLV_KRYLOV_CGS2");
  return fused_cycle(o) && !(f && f[0] == '1');
}

// Refinement's inner cycles may run device-driven (rounds enqueued in
// chunks, the round arithmetic on the device) with the delayed process:
// 1 (default) after a cycle that ran all its rounds, 2 always,
// 0 (TSYLV_KRYLOV_DEVICE_CYCLE=0) never.
static int device_cycle_mode(const tsylv_opts& o) {
  if (!o.refine || !delayed_cgs2(o)) return 0;
  const char* f = std::getenv("TSYLV_KRYLOV_DEVICE_CYCLE");
  if (f && f[0] == '0') return 0;
  if (f && f[0] == '2') return 2;
  return 1;
}
static bool device_cycle(const tsylv_opts& o) { return device_cycle_mode(o) != 0; }

// Plain FP64 tGMRES / tFOM of a small instance run whole in one workgroup
// (kern::tiny_krylov) unless TSYLV_KRYLOV_TINY=0.
static bool tiny_path(int method, int64_t n, int64_t s, int64_t p, const tsylv_opts& o) {
  if (o.refine || (method != TSYLV_METHOD_GMRES && method != TSYLV_METHOD_FOM)) return false;
  const char* f = std::getenv("TSYLV_KRYLOV_TINY");
  if (f && f[0] == '0') return false;
  return kern::tiny_krylov_fits(n, s, p, o.m);
}
static int64_t tiny_hist_len(const tsylv_opts& o) {
  if (!o.res_hist || o.res_hist_cap <= 0) return 0;
  return std::min<int64_t>(o.res_hist_cap, (int64_t)std::max(o.max_cycles, 0) * o.m);
}
static size_t tiny_bytes(int64_t N, const tsylv_opts& o) {
  return Workspace::bytes_for((int64_t)(o.m + 1) * N, 8) +
         Workspace::bytes_for((int64_t)o.m * o.m, 8) +
         Workspace::bytes_for(kern::kTinyRecord, 8) +
         Workspace::bytes_for(std::max<int64_t>(tiny_hist_len(o), 1), 8);
}

size_t krylov_workspace_bytes(int method, int64_t n, int64_t s, int64_t p, const tsylv_opts& o) {
  const int64_t N = n * s * p;
  size_t b = setup_bytes(n, s, p);
  if (method == TSYLV_METHOD_TBS)  // residual slot + reduction buffers, Schur scratch, flag
    return b + CycleWS<double>::bytes(N, 1) +
           Workspace::bytes_for(2 * kern::tbs_scratch_complex(n, s, (int)p), 8) +
           Workspace::bytes_for(1, sizeof(int));
  if (tiny_path(method, n, s, p, o)) return b + tiny_bytes(N, o);
  if (!o.refine) return b + CycleWS<double>::bytes(N, o.m);
  b += Workspace::bytes_for(N, 8);  // FP64 residual
  const bool dc = device_cycle(o);
  if (bf16_basis(o))
    return b +
           CycleWS<kern::bf16t>::bytes(kern::bf16_vtiled_elems(n, s, (int)p), o.inner_m, dc) +
           Workspace::bytes_for(kern::bf16_tiled_elems(n, (int)p), 2) +
           Workspace::bytes_for(p * s * s, 2);
  b += CycleWS<float>::bytes(N, o.inner_m, dc);
  if (o.prec == TSYLV_BF16)
    b += Workspace::bytes_for(kern::bf16_tiled_elems(n, (int)p), 2) +
         Workspace::bytes_for(p * s * s, 2) +
         Workspace::bytes_for(kern::bf16_vtiled_elems(n, s, (int)p), 2);
  else
    b += Workspace::bytes_for(p * n * n, 4) + Workspace::bytes_for(p * s * s, 4);
  return b;
}

// ---------------------------------------------------------------------------
// The resumable solve
// ---------------------------------------------------------------------------

struct KrylovState {
  // (method TBS completes in its SETUP phase: enqueue_direct)
  enum Phase { SETUP, RESTART, STEP, FINAL, DONE };

  Ctx& ctx;
  hipStream_t st;
  bool prof;
  int method;
  int64_t n, s, p, N;
  double* X;
  tsylv_opts o;
  bool refine;
  Workspace ws;
  Setup S;
  Operator op;
  CycleWS<double> w64;
  CycleWS<float> w32;
  CycleWS<kern::bf16t> w16;
  bool tiled = false;  // inner basis in tiled BF16 (w16) instead of FP32 (w32)
  bool devcyc = false;  // inner cycles enqueued in chunks (enqueue_chunk / complete_chunk)
  double* R64 = nullptr;
  RedBuf* red = nullptr;
  double* tbs_scratch = nullptr;  // method TBS: Schur factors and products per slice
  int* tbs_flag = nullptr;        // method TBS: 0, or 1 / 2 (Schur failure / singular)
  // small instances solved whole in one workgroup (tiny_path): basis slots
  // past its LDS, rotated Hessenberg columns, the result record and the
  // estimates; the record comes back through the pinned buffer
  bool tiny = false;
  double *tiny_basis = nullptr, *tiny_R = nullptr, *tiny_out = nullptr, *tiny_hist = nullptr;
  double* tiny_pinned = nullptr;

  Phase phase = SETUP;
  int status = TSYLV_NOT_CONVERGED;
  tsylv_info info{};
  std::chrono::steady_clock::time_point t0;
  double cnorm = 0.0, beta = 0.0;
  int iter = 0;               // restart cycles / refinement steps started
  int j = 0;                  // Arnoldi step inside the cycle
  double pending_scale = 0;   // 1 / h of the previous step (0: none; unfused path)
  bool scale_v0 = false;
  // Fused CGS2 (restart length within ortho_max_vectors): basis vectors kept
  // unnormalised, sigma_i = 1 / ||V_i|| carried to the apply (alpha) and the
  // Gram-Schmidt kernels, so no separate scaling sweep.
  bool fused = false;
  // Delayed reorthogonalisation (the default with the fused kernels): one
  // projection sweep and one update sweep per step, see enqueue_round.
  bool delayed = false;
  int dj = 0;                 // round of the delayed process
  bool final_round = false;   // the next round finalises the last column, no apply
  std::vector<double> h1p;    // first-pass coefficients of the pending column
  double w2prev = 0.0;        // ||M q_{dj-1}||^2, reference of the breakdown test
  int nv_upd = 0;             // update sweep: basis vectors it combines
  int corr_slot = -1;         // update sweep: slot it corrects (-1: none)
  int pending_update = 0;     // basis vectors to combine into X before the next residual
  Givens giv;
  std::vector<std::vector<double>> Hcols;
  std::vector<double> y_fom;
  bool fom_ok = false;

  KrylovState(Ctx& c, hipStream_t stream, bool profile, double* pinned, int meth, int64_t n_,
              int64_t s_, int64_t p_, const double* A, const double* B, const double* C,
              double* X_, const tsylv_opts& opts, const uint64_t* gen)
      : ctx(c), st(stream), prof(profile), method(meth), n(n_), s(s_), p(p_), N(n_ * s_ * p_),
        X(X_), o(opts), refine(opts.refine != 0),
        ws(c.arena, krylov_workspace_bytes(meth, n_, s_, p_, opts)) {
    t0 = std::chrono::steady_clock::now();
    info.status = TSYLV_PENDING;
    S = setup_fourier(ctx, st, prof, ws, n, s, p, A, B, C, X, o.x0_given != 0, gen);
    op.n = n;
    op.s = s;
    op.p = p;
    op.Ah64 = S.Ah;
    op.Bh64 = S.Bh;
    op.var64 = ctx.tune.get(TSYLV_FP64, n, s, p);
    fused = fused_cycle(o);
    tiled = bf16_basis(o);
    delayed = delayed_cgs2(o);
    devcyc = device_cycle(o);
    dcmode = device_cycle_mode(o);
    tiny = tiny_path(method, n, s, p, o);
    if (tiny) {
      tiny_basis = ws.take<double>((int64_t)(o.m + 1) * N);
      tiny_R = ws.take<double>((int64_t)o.m * o.m);
      tiny_out = ws.take<double>(kern::kTinyRecord);
      tiny_hist = ws.take<double>(std::max<int64_t>(tiny_hist_len(o), 1));
      tiny_pinned = pinned;
    } else if (method == TSYLV_METHOD_TBS) {
      w64.carve(ws, N, 1, pinned);
      red = &w64.red;
      tbs_scratch = ws.take<double>(2 * kern::tbs_scratch_complex(n, s, (int)p));
      tbs_flag = ws.take<int>(1);
    } else if (!refine) {
      w64.carve(ws, N, o.m, pinned);
      red = &w64.red;
    } else if (tiled) {
      R64 = ws.take<double>(N);
      const int64_t Nt = kern::bf16_vtiled_elems(n, s, (int)p);
      w16.carve(ws, Nt, o.inner_m, pinned, devcyc);
      red = &w16.red;
      // The tiled padding (rows >= n, columns >= s) must read as zero; the
      // kernels that write basis vectors keep it so.
      if (Nt != N)
        TSYLV_HIP(hipMemsetAsync(w16.basis, 0, (size_t)(o.inner_m + 1) * w16.ldv * 2, st));
      op.low = TSYLV_BF16;
      op.var_low = ctx.tune.get(TSYLV_BF16, n, s, p);
      uint16_t* Ab = ws.take<uint16_t>(kern::bf16_tiled_elems(n, (int)p));
      uint16_t* Bb = ws.take<uint16_t>(p * s * s);
      kern::tile_operator_bf16(S.Ah, Ab, n, (int)p, st);
      kern::convert_f64_bf16(S.Bh, Bb, p * s * s, st);
      op.Ahb = Ab;
      op.Bhb = Bb;
    } else {
      R64 = ws.take<double>(N);
      w32.carve(ws, N, o.inner_m, pinned, devcyc);
      red = &w32.red;
      op.low = o.prec == TSYLV_BF16 ? TSYLV_BF16 : TSYLV_FP32;
      op.var_low = ctx.tune.get(op.low, n, s, p);
      if (op.low == TSYLV_BF16) {
        uint16_t* Ab = ws.take<uint16_t>(kern::bf16_tiled_elems(n, (int)p));
        uint16_t* Bb = ws.take<uint16_t>(p * s * s);
        kern::tile_operator_bf16(S.Ah, Ab, n, (int)p, st);
        kern::convert_f64_bf16(S.Bh, Bb, p * s * s, st);
        op.Ahb = Ab;
        op.Bhb = Bb;
        op.Vtb = ws.take<uint16_t>(kern::bf16_vtiled_elems(n, s, (int)p));
      } else {
        float* Af = ws.take<float>(p * n * n);
        float* Bf = ws.take<float>(p * s * s);
        kern::convert_f64_f32(S.Ah, Af, p * n * n, st);
        kern::convert_f64_f32(S.Bh, Bf, p * s * s, st);
        op.Ah32 = Af;
        op.Bh32 = Bf;
      }
    }
  }

  void apply(const double* V, double* out, const double* Y, double alpha, double beta_) {
    ProfScope ps(ctx, TSYLV_K_APPLY, st, prof);
    kern::apply_f64(op.Ah64, op.Bh64, V, out, Y, alpha, beta_, n, s, (int)p, st, op.var64);
  }
  void apply(const float* V, float* out, const float* Y, double alpha, double beta_) {
    ProfScope ps(ctx, TSYLV_K_APPLY_LOW, st, prof);
    if (op.low == TSYLV_BF16)
      kern::apply_bf16(op.Ahb, op.Bhb, V, op.Vtb, out, Y, alpha, beta_, n, s, (int)p, st,
                       op.var_low);
    else
      kern::apply_f32(op.Ah32, op.Bh32, V, out, Y, alpha, beta_, n, s, (int)p, st, op.var_low);
  }

  void apply(const kern::bf16t* V, kern::bf16t* out, const kern::bf16t* Y, double alpha,
             double beta_) {
    ProfScope ps(ctx, TSYLV_K_APPLY_LOW, st, prof);
    if (Y || beta_ != 0.0) throw Error(TSYLV_EINVAL, "apply: tiled vectors take no Y");
    kern::apply_bf16_tiled(op.Ahb, op.Bhb, V, out, alpha, n, s, (int)p, st, op.var_low);
  }

  // ||v||^2 to red->h_ww[0] after the next synchronisation.
  void enqueue_norm2(const double* v) {
    kern::mdot_partial((const double*)nullptr, 0, 0, v, N, red->part, red->ldp, 1, st);
    // chunks of v's own length (a tiled basis has longer vectors than v)
    kern::reduce_partials(red->part, kern::mdot_chunks(N), red->ldp, 1, red->d_ww, st);
    TSYLV_HIP(hipMemcpyAsync(red->h_ww, red->d_ww, sizeof(double), hipMemcpyDeviceToHost, st));
  }

  // Algorithm 2 step 3 for the current j: W = M(V_j), CGS2, ||W||.
  template <typename TV>
  void enqueue_step(CycleWS<TV>& w) {
    const int nv = j + 1;
    TV* W = w.V(j + 1);
    const RedBuf& r = w.red;
    if (fused) {
      // W = M(sigma_j V_j); CGS2 against sigma_i V_i in three sweeps.
      const int64_t L = w.len;
      TSYLV_HIP(hipMemcpyAsync(w.d_sigma, w.h_sigma, nv * sizeof(double), hipMemcpyHostToDevice,
                               st));
      apply((const TV*)w.V(j), W, (const TV*)nullptr, w.h_sigma[j], 0.0);
      ProfScope ps(ctx, TSYLV_K_ORTHO, st, prof);
      const int och = kern::ortho_chunks(L);
      kern::ortho_dots((const TV*)w.basis, w.ldv, nv, w.d_sigma, (const TV*)W, L, r.part, r.ldp,
                       st);
      kern::reduce_partials(r.part, och, r.ldp, nv + 1, w.d_h1, st);
      kern::ortho_update((const TV*)w.basis, w.ldv, nv, w.d_h1, w.d_sigma, W, L, r.part, r.ldp, 0,
                         st);
      kern::reduce_partials(r.part, och, r.ldp, nv, w.d_h2, st);
      kern::ortho_update((const TV*)w.basis, w.ldv, nv, w.d_h2, w.d_sigma, W, L, r.part, r.ldp, 1,
                         st);
      kern::reduce_partials(r.part, och, r.ldp, 1, r.d_ww, st);
    } else if constexpr (std::is_same_v<TV, kern::bf16t>) {
      throw Error(TSYLV_EINVAL, "krylov: BF16 vectors need the fused kernels");
    } else {
      if (pending_scale != 0.0) {  // step 3(e) of the previous step: V_j = W / h_{j,j-1}
        kern::scale((const TV*)w.V(j), w.V(j), pending_scale, N, st);
        pending_scale = 0.0;
      }
      apply((const TV*)w.V(j), W, (const TV*)nullptr, 1.0, 0.0);
      ProfScope ps(ctx, TSYLV_K_ORTHO, st, prof);
      kern::mdot_partial((const TV*)w.basis, w.ldv, nv, (const TV*)W, N, r.part, r.ldp, 1, st);
      kern::reduce_partials(r.part, r.nchunks, r.ldp, nv + 1, w.d_h1, st);
      kern::mupdate((const TV*)w.basis, w.ldv, nv, w.d_h1, W, N, st);
      kern::mdot_partial((const TV*)w.basis, w.ldv, nv, (const TV*)W, N, r.part, r.ldp, 0, st);
      kern::reduce_partials(r.part, r.nchunks, r.ldp, nv, w.d_h2, st);
      kern::mupdate((const TV*)w.basis, w.ldv, nv, w.d_h2, W, N, st);
      kern::mdot_partial((const TV*)nullptr, 0, 0, (const TV*)W, N, r.part, r.ldp, 1, st);
      kern::reduce_partials(r.part, r.nchunks, r.ldp, 1, r.d_ww, st);
    }
    // h1 (nv + 1 values), h2 (nv) and ||w||^2 in one copy (same layout on host)
    TSYLV_HIP(hipMemcpyAsync(w.h_h1, w.d_h1, (2 * (w.m + 2) + 1) * sizeof(double),
                             hipMemcpyDeviceToHost, st));
  }

  // ---- delayed reorthogonalisation --------------------------------------
  // CGS2 with the second projection of each vector delayed to the next step
  // (the low-synchronisation DCGS2 scheme of Bielich et al., 2022), so that a
  // step reads the basis twice instead of three times.  Slot j holds u_j,
  // the once-projected new direction, until the next round corrects it.
  // Round j >= 1 enqueues
  //   * the update sweep of round j - 1: slot j - 1 <- v_{j-1} = u_{j-1} -
  //     Q a (its reprojection) and slot j <- u_j (the first projection of
  //     M q_{j-1}, expressed through W' = M u_{j-1} of that round);
  //   * W' = M u_j into slot j + 1;
  //   * one sweep for a = Q^T u_j, b = Q^T W', u_j . W', ||u_j||^2, ||W'||^2
  //     over the final vectors q_0..q_{j-1} (Q).
  // Completing it finalises column j - 1 of H: h_{0..j-1} += a and
  // h_{j,j-1} = nu = ||u_j - Q a|| (from the exact ||u_j||^2), so q_j =
  // (u_j - Q a) / nu; with M q_i = Q H e_i for the finished columns,
  // M q_j = (W' - Q g) / nu (g = H a), which gives the first projection of
  // the next column from the sweep's scalars alone.  The last round of a
  // cycle skips the apply (it only needs a and ||u_j||^2).  In exact
  // arithmetic the Hessenberg matrix equals CGS2's.
  template <typename TV>
  void enqueue_round(CycleWS<TV>& w) {
    const RedBuf& r = w.red;
    const int64_t L = w.len;
    const int och = kern::ortho_chunks(L);
    double* d_coef = w.d_sigma + (w.m + 2);
    if (dj == 0) {
      TSYLV_HIP(hipMemcpyAsync(w.d_sigma, w.h_sigma, sizeof(double), hipMemcpyHostToDevice, st));
      apply((const TV*)w.V(0), w.V(1), (const TV*)nullptr, w.h_sigma[0], 0.0);
      ProfScope ps(ctx, TSYLV_K_ORTHO, st, prof);
      kern::ortho_dots((const TV*)w.basis, w.ldv, 1, w.d_sigma, (const TV*)w.V(1), L, r.part,
                       r.ldp, st);
      kern::reduce_partials(r.part, och, r.ldp, 2, w.d_h1, st);
    } else {
      TSYLV_HIP(hipMemcpyAsync(w.d_sigma, w.h_sigma, (w.m + 2 + 2 * nv_upd + 2) * sizeof(double),
                               hipMemcpyHostToDevice, st));
      {
        ProfScope ps(ctx, TSYLV_K_ORTHO, st, prof);
        kern::ortho_update2((const TV*)w.basis, w.ldv, nv_upd, d_coef,
                            corr_slot >= 0 ? w.V(corr_slot) : (TV*)nullptr, w.V(dj), L, st);
      }
      if (final_round) {
        ProfScope ps(ctx, TSYLV_K_ORTHO, st, prof);
        kern::ortho_dots((const TV*)w.basis, w.ldv, dj, w.d_sigma, (const TV*)w.V(dj), L, r.part,
                         r.ldp, st);
        kern::reduce_partials(r.part, och, r.ldp, dj + 1, w.d_h1, st);
      } else {
        apply((const TV*)w.V(dj), w.V(dj + 1), (const TV*)nullptr, 1.0, 0.0);
        ProfScope ps(ctx, TSYLV_K_ORTHO, st, prof);
        kern::ortho_dots2((const TV*)w.basis, w.ldv, dj, w.d_sigma, (const TV*)w.V(dj),
                          (const TV*)w.V(dj + 1), L, r.part, r.ldp, st);
        kern::reduce_partials(r.part, och, r.ldp, 2 * dj + 3, w.d_h1, st);
      }
    }
    TSYLV_HIP(hipMemcpyAsync(w.h_h1, w.d_h1, (2 * (w.m + 2) + 1) * sizeof(double),
                             hipMemcpyDeviceToHost, st));
  }

  // Inner cycles of the delayed process enqueued in chunks of rounds:
  // dcgs2_round does each round's arithmetic on the device, so the host
  // synchronises once per chunk (4, then 8, then 16 ... rounds) and runs the
  // Givens / LU step over the columns the chunk finished (complete_chunk).
  // The columns, the basis and the coefficients are those of the
  // host-driven rounds; a cycle that meets its stopping test inside a chunk
  // is truncated at that column (the same solution as stopping there), so
  // at most one chunk of rounds is spent past the stop.
  // A cycle runs device-driven only when the previous one of the solve ended
  // by count: cycles that stop early on the estimate (small, easy systems)
  // stay host-driven, which stops them at the exact step.
  int dcmode = 0;           // device_cycle_mode of the options
  bool last_full = false;  // the previous cycle ran all its rounds
  bool dev_now = false;    // the current cycle is device-driven
  int cyc_next = 0;   // next round to enqueue
  int cyc_chunk = 4;  // rounds in the next chunk
  int cyc_cols = 0;   // columns the host has processed

  template <typename TV>
  void enqueue_chunk(CycleWS<TV>& w) {
    const RedBuf& r = w.red;
    const int64_t L = w.len;
    const int och = kern::ortho_chunks(L);
    const int M = o.inner_m, ldh = w.ldh();
    double* d_coef = w.d_sigma + (w.m + 2);
    const int last = std::min(M, cyc_next + cyc_chunk - 1);
    for (int rr = cyc_next; rr <= last; ++rr) {
      if (rr == 0) {
        TSYLV_HIP(hipMemcpyAsync(w.d_sigma, w.h_sigma, sizeof(double), hipMemcpyHostToDevice,
                                 st));
        apply((const TV*)w.V(0), w.V(1), (const TV*)nullptr, w.h_sigma[0], 0.0);
        ProfScope ps(ctx, TSYLV_K_ORTHO, st, prof);
        kern::ortho_dots((const TV*)w.basis, w.ldv, 1, w.d_sigma, (const TV*)w.V(1), L, r.part,
                         r.ldp, st);
        kern::reduce_partials(r.part, och, r.ldp, 2, w.d_h1, st);
        kern::dcgs2_round(w.d_h1, 0, false, ldh, w.d_H, w.d_h1p, w.d_sigma, d_coef, w.d_scal,
                          st);
        continue;
      }
      const bool fin = rr == M;
      {
        ProfScope ps(ctx, TSYLV_K_ORTHO, st, prof);
        kern::ortho_update2((const TV*)w.basis, w.ldv, rr == 1 ? 1 : rr - 1, d_coef,
                            rr == 1 ? (TV*)nullptr : w.V(rr - 1), w.V(rr), L, st);
      }
      if (!fin) apply((const TV*)w.V(rr), w.V(rr + 1), (const TV*)nullptr, 1.0, 0.0);
      ProfScope ps(ctx, TSYLV_K_ORTHO, st, prof);
      if (fin) {
        kern::ortho_dots((const TV*)w.basis, w.ldv, rr, w.d_sigma, (const TV*)w.V(rr), L, r.part,
                         r.ldp, st);
        kern::reduce_partials(r.part, och, r.ldp, rr + 1, w.d_h1, st);
      } else {
        kern::ortho_dots2((const TV*)w.basis, w.ldv, rr, w.d_sigma, (const TV*)w.V(rr),
                          (const TV*)w.V(rr + 1), L, r.part, r.ldp, st);
        kern::reduce_partials(r.part, och, r.ldp, 2 * rr + 3, w.d_h1, st);
      }
      kern::dcgs2_round(w.d_h1, rr, fin, ldh, w.d_H, w.d_h1p, w.d_sigma, d_coef, w.d_scal, st);
    }
    cyc_next = last + 1;
    cyc_chunk *= 2;
    // the finished columns and [w2prev, breakdown], and sigma, back to the host
    TSYLV_HIP(hipMemcpyAsync(w.h_H, w.d_H, CycleWS<TV>::hess_len(w.m) * sizeof(double),
                             hipMemcpyDeviceToHost, st));
    TSYLV_HIP(hipMemcpyAsync(w.h_sigma, w.d_sigma, (M + 1) * sizeof(double),
                             hipMemcpyDeviceToHost, st));
  }

  // Returns true when the cycle ends (its correction is then pending).
  template <typename TV>
  bool complete_chunk(CycleWS<TV>& w, double stop_abs) {
    const int M = o.inner_m, ldh = w.ldh();
    const int broken = (int)w.h_scal[1];         // round that met h = 0, or -1
    int done = std::min(cyc_next - 1, M);        // rounds 1..done finished columns 0..done-1
    bool end = cyc_next > M;
    if (broken >= 1 && broken <= done) {
      done = broken;
      end = true;
    }
    int J = done;
    bool est_stop = false;
    for (int i = cyc_cols; i < done; ++i) {
      std::vector<double> h(w.h_H + (int64_t)ldh * i, w.h_H + (int64_t)ldh * i + i + 2);
      info.steps++;
      Hcols.push_back(h);
      double est;
      if (method == TSYLV_METHOD_GMRES) {
        est = giv.add(h);
      } else {
        giv.add(h);
        fom_ok = fom_solve(Hcols, (size_t)(i + 1), beta, y_fom);
        est = fom_ok ? h[i + 1] * std::fabs(y_fom[i]) : INFINITY;
      }
      info.relres_est = est / cnorm;
      if (o.res_hist && info.res_hist_len < o.res_hist_cap)
        o.res_hist[info.res_hist_len++] = info.relres_est;
      if (est <= stop_abs) {
        J = i + 1;
        end = true;
        est_stop = true;
        break;
      }
    }
    const bool early = est_stop || (broken >= 1 && broken <= std::min(cyc_next - 1, M));
    cyc_cols = J;
    if (!end) return false;
    last_full = !early && J == M;
    std::vector<double> y;
    if (method == TSYLV_METHOD_GMRES) {
      y = giv.solve((size_t)J);
    } else if (fom_ok) {
      y = y_fom;
    } else {
      info.fom_fallback++;
      y = giv.solve((size_t)J);
    }
    for (int i = 0; i < J; ++i) w.h_y[i] = -y[i] * w.h_sigma[i];
    pending_update = J;
    return true;
  }

  // Decides whether the round after the current one is the cycle's last: by
  // count, or when the column it will finalise (first projection h1p, norm
  // estimated by Pythagoras) already meets the stopping test.
  void plan_next_round(double stop_abs) {
    const int mcyc = refine ? o.inner_m : o.m;
    const int next = dj + 1;
    final_round = next >= mcyc;
    if (final_round) return;
    double h2 = 0.0;
    for (double v : h1p) h2 += v * v;
    const double nu2 = w2prev - h2;
    if (!(nu2 > 256.0 * kEps * kEps * w2prev)) {
      final_round = true;  // (near) breakdown ahead
      return;
    }
    if (method == TSYLV_METHOD_GMRES) {
      Givens t = giv;
      std::vector<double> h(h1p);
      h.push_back(std::sqrt(nu2));
      if (t.add(h) <= stop_abs) final_round = true;
    }
  }

  template <typename TV>
  bool complete_round(CycleWS<TV>& w, double stop_abs) {
    const double* res = w.h_h1;
    const int mcyc = refine ? o.inner_m : o.m;
    double* coef = w.h_sigma + (w.m + 2);
    if (dj == 0) {
      // q_0 . W' and ||M q_0||^2; the update forms u_1 = W' - h q_0
      h1p.assign(1, res[0]);
      w2prev = res[1];
      nv_upd = 1;
      corr_slot = -1;
      coef[0] = 0.0;
      coef[1] = -res[0] * w.h_sigma[0];
      coef[2] = 1.0;
      coef[3] = 0.0;
      plan_next_round(stop_abs);
      dj = 1;
      return false;
    }
    const int j = dj;
    std::vector<double> a(res, res + j), b;
    double c = 0.0, d, e = 0.0;
    if (final_round) {
      d = res[j];
    } else {
      b.assign(res + j, res + 2 * j);
      c = res[2 * j];
      d = res[2 * j + 1];
      e = res[2 * j + 2];
    }
    double na2 = 0.0;
    for (double v : a) na2 += v * v;
    const double nu2 = d - na2;
    const bool breakdown = !(nu2 > 256.0 * kEps * kEps * w2prev);  // reading: h_{j+1,j} = 0
    const double nu = breakdown ? 0.0 : std::sqrt(nu2);
    std::vector<double> h(j + 1);
    for (int i = 0; i < j; ++i) h[i] = h1p[i] + a[i];
    h[j] = nu;
    info.steps++;
    Hcols.push_back(h);
    double est;
    if (method == TSYLV_METHOD_GMRES) {
      est = giv.add(h);
    } else {
      giv.add(h);  // keeps the tGMRES fallback available
      fom_ok = fom_solve(Hcols, (size_t)j, beta, y_fom);
      est = fom_ok ? nu * std::fabs(y_fom[j - 1]) : INFINITY;
    }
    info.relres_est = est / cnorm;
    if (o.res_hist && info.res_hist_len < o.res_hist_cap)
      o.res_hist[info.res_hist_len++] = info.relres_est;
    if (breakdown || est <= stop_abs || j >= mcyc || final_round) {
      last_full = !breakdown && !(est <= stop_abs) && j >= mcyc;
      std::vector<double> y;
      if (method == TSYLV_METHOD_GMRES) {
        y = giv.solve((size_t)j);
      } else if (fom_ok) {
        y = y_fom;
      } else {
        info.fom_fallback++;
        y = giv.solve((size_t)j);
      }
      for (int i = 0; i < j; ++i) w.h_y[i] = -y[i] * w.h_sigma[i];
      pending_update = j;
      return true;
    }
    // q_j = (u_j - Q a) / nu;  g = H a over the finished columns 0..j-1
    w.h_sigma[j] = 1.0 / nu;
    std::vector<double> g(j + 1, 0.0);
    for (int i = 0; i < j; ++i)
      for (int l = 0; l <= i + 1 && l <= j; ++l) g[l] += Hcols[i][l] * a[i];
    double ab = 0.0;
    for (int l = 0; l < j; ++l) ab += a[l] * b[l];
    const double qjw = (c - ab) / nu;  // q_j . W'
    std::vector<double> h1n(j + 1);
    for (int l = 0; l < j; ++l) h1n[l] = (b[l] - g[l]) / nu;
    h1n[j] = (qjw - g[j]) / nu;
    // ||M q_j||^2 = ||W' - Q g||^2 / nu^2
    double gw = 0.0, gg = 0.0;
    for (int l = 0; l < j; ++l) gw += g[l] * b[l];
    gw += g[j] * qjw;
    for (double v : g) gg += v * v;
    w2prev = std::max(0.0, (e - 2.0 * gw + gg) / (nu * nu));
    // update sweep: v_j = u_j - sum a_l q_l;  u_{j+1} = M q_j - sum h1n_l q_l
    //   = W' / nu - sum_{l<j} (g_l / nu + h1n_l) q_l - (g_j / nu + h1n_j) v_j / nu
    nv_upd = j;
    corr_slot = j;
    for (int l = 0; l < j; ++l) {
      coef[l] = a[l] * w.h_sigma[l];
      coef[j + l] = -(g[l] / nu + h1n[l]) * w.h_sigma[l];
    }
    coef[2 * j] = 1.0 / nu;
    coef[2 * j + 1] = -(g[j] / nu + h1n[j]) / nu;
    h1p = h1n;
    plan_next_round(stop_abs);
    dj = j + 1;
    return false;
  }

  // Consumes a step's h column; returns true when the cycle ends.
  template <typename TV>
  bool complete_step(CycleWS<TV>& w, double stop_abs) {
    const int nv = j + 1;
    std::vector<double> h(nv + 1);
    for (int i = 0; i < nv; ++i) h[i] = w.h_h1[i] + w.h_h2[i];
    const double w0 = std::sqrt(w.h_h1[nv]);
    double hn = std::sqrt(w.red.h_ww[0]);
    const bool breakdown = !(hn > 16.0 * kEps * w0);  // reading: h_{j+1,j} = 0
    if (breakdown) hn = 0.0;
    h[nv] = hn;
    info.steps++;
    double est;
    if (method == TSYLV_METHOD_GMRES) {
      est = giv.add(h);
    } else {
      giv.add(h);  // keeps the tGMRES fallback available
      Hcols.push_back(h);
      fom_ok = fom_solve(Hcols, (size_t)nv, beta, y_fom);
      est = fom_ok ? hn * std::fabs(y_fom[nv - 1]) : INFINITY;
    }
    info.relres_est = est / cnorm;
    if (o.res_hist && info.res_hist_len < o.res_hist_cap)
      o.res_hist[info.res_hist_len++] = info.relres_est;
    const int mcyc = refine ? o.inner_m : o.m;
    if (breakdown || est <= stop_abs || nv >= mcyc) {
      // Algorithm 3 step 4(b): the small problem; 4(c) is enqueued next.
      std::vector<double> y;
      if (method == TSYLV_METHOD_GMRES) {
        y = giv.solve((size_t)nv);
      } else if (fom_ok) {
        y = y_fom;
      } else {
        info.fom_fallback++;
        y = giv.solve((size_t)nv);
      }
      for (int i = 0; i < nv; ++i) w.h_y[i] = -y[i] * (fused ? w.h_sigma[i] : 1.0);
      pending_update = nv;
      return true;
    }
    if (fused)
      w.h_sigma[j + 1] = 1.0 / hn;  // V_{j+1} stays unnormalised (step 3(e) folded in)
    else
      pending_scale = 1.0 / hn;
    ++j;
    return false;
  }

  // Algorithm 3 step 4(c): X += V_k (*) y (X FP64, V of type TV).
  template <typename TV>
  void enqueue_update(CycleWS<TV>& w) {
    TSYLV_HIP(hipMemcpyAsync(w.d_y, w.h_y, pending_update * sizeof(double), hipMemcpyHostToDevice,
                             st));
    if constexpr (std::is_same_v<TV, kern::bf16t>)
      kern::untile_update_bf16(w.basis, w.ldv, pending_update, w.d_y, S.Zx, n, s, (int)p, st);
    else
      kern::mupdate((const TV*)w.basis, w.ldv, pending_update, w.d_y, S.Zx, N, st);
    pending_update = 0;
  }

  // Method TBS in one pass (one synchronisation): ||C||, Algorithm 5 on
  // every Fourier slice, R = C - M(X) and ||R|| in FP64, the inverse DFT of
  // X; the two norms and the flag come back together.
  void enqueue_direct() {
    const RedBuf& r = w64.red;
    const int nch = kern::mdot_chunks(N);
    kern::mdot_partial((const double*)nullptr, 0, 0, S.Zc, N, r.part, r.ldp, 1, st);
    kern::reduce_partials(r.part, nch, r.ldp, 1, w64.d_h1, st);
    TSYLV_HIP(hipMemsetAsync(tbs_flag, 0, sizeof(int), st));
    kern::tbs_solve(S.Ah, S.Bh, S.Zc, S.Zx, n, s, (int)p, tbs_scratch, tbs_flag, st);
    double* R = w64.V(0);
    apply((const double*)S.Zx, R, (const double*)S.Zc, -1.0, 1.0);
    kern::mdot_partial((const double*)nullptr, 0, 0, R, N, r.part, r.ldp, 1, st);
    kern::reduce_partials(r.part, nch, r.ldp, 1, w64.d_h1 + 1, st);
    {
      ProfScope ps(ctx, TSYLV_K_XFORM, st, prof);
      kern::tube_xform_f64(S.Zx, X, S.xf_inv, n * s, (int)p, st);
    }
    TSYLV_HIP(hipMemcpyAsync(w64.h_h1, w64.d_h1, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    TSYLV_HIP(hipMemcpyAsync(w64.h_y, tbs_flag, sizeof(int), hipMemcpyDeviceToHost, st));
  }

  void complete_direct() {
    int flag = 0;
    std::memcpy(&flag, w64.h_y, sizeof(int));
    cnorm = std::sqrt(w64.h_h1[0]);
    info.relres_true = cnorm > 0.0 ? std::sqrt(w64.h_h1[1]) / cnorm : 0.0;
    info.relres_est = info.relres_true;
    if (flag == 2)
      status = TSYLV_ESINGULAR;
    else if (flag == 1)
      status = TSYLV_EBREAKDOWN;
    else
      status = info.relres_true <= o.tol ? TSYLV_OK : TSYLV_NOT_CONVERGED;
  }

  // Small instances: Algorithm 3 whole in one launch, the inverse DFT of X
  // and the result record back in one copy.
  void enqueue_tiny() {
    kern::tiny_krylov(S.Ah, S.Bh, S.Zc, S.Zx, tiny_basis, tiny_R, tiny_hist,
                      (int)tiny_hist_len(o), tiny_out, (int)n, (int)s, (int)p, o.m,
                      std::max(o.max_cycles, 0), method == TSYLV_METHOD_FOM, o.x0_given != 0,
                      o.tol, st);
    {
      ProfScope ps(ctx, TSYLV_K_XFORM, st, prof);
      kern::tube_xform_f64(S.Zx, X, S.xf_inv, n * s, (int)p, st);
    }
    TSYLV_HIP(hipMemcpyAsync(tiny_pinned, tiny_out, kern::kTinyRecord * sizeof(double),
                             hipMemcpyDeviceToHost, st));
  }

  void complete_tiny() {
    const double* r = tiny_pinned;
    status = (int)r[0];
    info.steps = (int)r[1];
    info.cycles = (int)r[2];
    info.relres_true = r[3];
    info.relres_est = r[4];
    info.fom_fallback = (int)r[5];
    const int hl = (int)r[6];
    if (hl > 0 && o.res_hist) {
      TSYLV_HIP(hipMemcpyAsync(o.res_hist, tiny_hist, hl * sizeof(double),
                               hipMemcpyDeviceToHost, st));
      TSYLV_HIP(hipStreamSynchronize(st));
    }
    info.res_hist_len = hl;
  }

  void enqueue() {
    switch (phase) {
      case SETUP:
        if (tiny) {
          enqueue_tiny();
          break;
        }
        if (method == TSYLV_METHOD_TBS) {
          enqueue_direct();
          break;
        }
        enqueue_norm2(S.Zc);  // ||C||_F (Parseval)
        break;
      case RESTART: {
        if (pending_update) {
          if (tiled)
            enqueue_update(w16);
          else if (refine)
            enqueue_update(w32);
          else
            enqueue_update(w64);
        }
        // R0 = C - M(X0)  (Algorithm 3, step 3), in FP64.
        double* R = refine ? R64 : w64.V(0);
        if (iter == 0 && !o.x0_given)
          TSYLV_HIP(hipMemcpyAsync(R, S.Zc, N * sizeof(double), hipMemcpyDeviceToDevice, st));
        else
          apply((const double*)S.Zx, R, (const double*)S.Zc, -1.0, 1.0);
        enqueue_norm2(R);
        break;
      }
      case STEP:
        if (scale_v0) {
          if (tiled) {
            kern::tile_scale_bf16(R64, w16.V(0), 1.0 / beta, n, s, (int)p, st);
            w16.h_sigma[0] = 1.0;
          } else if (refine) {
            kern::scale((const double*)R64, w32.V(0), 1.0 / beta, N, st);  // rounds to FP32
            w32.h_sigma[0] = 1.0;
          } else if (fused) {
            w64.h_sigma[0] = 1.0 / beta;  // V_0 = R kept unnormalised
          } else {
            kern::scale((const double*)w64.V(0), w64.V(0), 1.0 / beta, N, st);
          }
          scale_v0 = false;
        }
        if (dev_now) {
          if (tiled)
            enqueue_chunk(w16);
          else
            enqueue_chunk(w32);
        } else if (delayed) {
          if (tiled)
            enqueue_round(w16);
          else if (refine)
            enqueue_round(w32);
          else
            enqueue_round(w64);
        } else if (tiled) {
          enqueue_step(w16);
        } else if (refine) {
          enqueue_step(w32);
        } else {
          enqueue_step(w64);
        }
        break;
      case FINAL: {
        // Algorithm 1 step 3: back to the spatial domain.
        ProfScope ps(ctx, TSYLV_K_XFORM, st, prof);
        if (cnorm == 0.0)
          TSYLV_HIP(hipMemsetAsync(X, 0, N * sizeof(double), st));
        else
          kern::tube_xform_f64(S.Zx, X, S.xf_inv, n * s, (int)p, st);
        break;
      }
      case DONE:
        break;
    }
  }

  void complete() {
    switch (phase) {
      case SETUP:
        if (tiny) {
          complete_tiny();
          phase = DONE;
          info.status = status;
          info.seconds = seconds_since(t0);
          break;
        }
        if (method == TSYLV_METHOD_TBS) {
          complete_direct();
          phase = DONE;
          info.status = status;
          info.seconds = seconds_since(t0);
          break;
        }
        cnorm = std::sqrt(red->h_ww[0]);
        if (cnorm == 0.0) {
          info.relres_true = 0.0;
          status = TSYLV_OK;
          phase = FINAL;
        } else {
          phase = RESTART;
        }
        break;

      case RESTART: {
        beta = std::sqrt(red->h_ww[0]);
        info.relres_true = beta / cnorm;
        const int max_iter = refine ? o.max_outer : o.max_cycles;
        if (info.relres_true <= o.tol) {
          status = TSYLV_OK;
          phase = FINAL;
        } else if (iter >= max_iter) {
          status = TSYLV_NOT_CONVERGED;
          phase = FINAL;
        } else {
          ++iter;
          info.cycles++;
          if (refine) info.outer++;
          giv.reset(beta);
          Hcols.clear();
          fom_ok = false;
          j = 0;
          dj = 0;
          final_round = false;
          cyc_next = 0;
          cyc_chunk = 4;
          cyc_cols = 0;
          dev_now = dcmode == 2 || (dcmode == 1 && last_full);
          pending_scale = 0.0;
          scale_v0 = true;
          phase = STEP;
        }
        break;
      }
      case STEP: {
        const double stop = refine ? std::max(o.inner_tol * beta, 0.5 * o.tol * cnorm)
                                   : o.tol * cnorm;
        bool end;
        if (dev_now)
          end = tiled ? complete_chunk(w16, stop) : complete_chunk(w32, stop);
        else if (tiled)
          end = delayed ? complete_round(w16, stop) : complete_step(w16, stop);
        else if (refine)
          end = delayed ? complete_round(w32, stop) : complete_step(w32, stop);
        else
          end = delayed ? complete_round(w64, stop) : complete_step(w64, stop);
        if (end) phase = RESTART;
        break;
      }
      case FINAL:
        phase = DONE;
        info.status = status;
        info.seconds = seconds_since(t0);
        break;
      case DONE:
        break;
    }
  }
};

KrylovTask::KrylovTask(Ctx& ctx, hipStream_t st, bool profile, double* pinned, int method,
                       int64_t n, int64_t s, int64_t p, const double* A, const double* B,
                       const double* C, double* X, const tsylv_opts& o, const uint64_t* gen)
    : s_(new KrylovState(ctx, st, profile, pinned, method, n, s, p, A, B, C, X, o, gen)) {}

KrylovTask::~KrylovTask() = default;

size_t KrylovTask::pinned_doubles(const tsylv_opts& o) {
  const int m = o.refine ? o.inner_m : o.m;
  return 7 * (size_t)(m + 2) + 2 + (device_cycle(o) ? (size_t)CycleWS<float>::hess_len(m) : 0);
}

void KrylovTask::enqueue() { s_->enqueue(); }
void KrylovTask::complete() { s_->complete(); }
bool KrylovTask::done() const { return s_->phase == KrylovState::DONE; }
int KrylovTask::status() const { return s_->status; }
const tsylv_info& KrylovTask::info() const { return s_->info; }
hipStream_t KrylovTask::stream() const { return s_->st; }

int krylov_solve(Ctx& ctx, int method, int64_t n, int64_t s, int64_t p, const double* A,
                 const double* B, const double* C, double* X, const tsylv_opts& o,
                 tsylv_info& info) {
  KrylovTask t(ctx, ctx.stream, true, ctx.host_buffer(KrylovTask::pinned_doubles(o)), method, n, s,
               p, A, B, C, X, o);
  while (!t.done()) {
    t.enqueue();
    ctx.sync();
    t.complete();
  }
  info = t.info();
  return t.status();
}

// ---------------------------------------------------------------------------
// Y = A*X - X*B through the Fourier planes (Algorithm 1), with the slice
// products in the requested precision.
// ---------------------------------------------------------------------------

size_t apply_workspace_bytes(int64_t n, int64_t s, int64_t p) {
  int64_t N = n * s * p;
  return Workspace::bytes_for(p * n * n, 8) + Workspace::bytes_for(p * s * s, 8) +
         3 * Workspace::bytes_for(p * p, 8) + 2 * Workspace::bytes_for(N, 8) +
         std::max(Workspace::bytes_for(p * n * n, 4),
                  Workspace::bytes_for(kern::bf16_tiled_elems(n, (int)p), 2)) +
         Workspace::bytes_for(p * s * s, 4) + 2 * Workspace::bytes_for(N, 4) +
         Workspace::bytes_for(kern::bf16_vtiled_elems(n, s, (int)p), 2);
}

namespace {

// Algorithm 1 for Y = A*X - X*B with the slice products in `prec`: every
// buffer taken from `ws` (an arena workspace or a caller's scratch); the
// slice-product launch is timed when `ctx` is given and profiling is on.
template <class WS>
void apply_core(WS& ws, hipStream_t st, Ctx* ctx, int64_t n, int64_t s, int64_t p,
                const double* A, const double* B, const double* X, double* Y, int prec,
                int variant) {
  const int64_t N = n * s * p;
  double* Ah = ws.template take<double>(p * n * n);
  double* Bh = ws.template take<double>(p * s * s);
  double* xf_op = ws.template take<double>(p * p);
  double* xf_fwd = ws.template take<double>(p * p);
  double* xf_inv = ws.template take<double>(p * p);
  double* Zx = ws.template take<double>(N);
  double* Zy = ws.template take<double>(N);
  kern::build_xform(xf_op, (int)p, XF_OPERATOR, st);
  kern::build_xform(xf_fwd, (int)p, XF_FORWARD, st);
  kern::build_xform(xf_inv, (int)p, XF_INVERSE, st);
  kern::tube_xform_f64(A, Ah, xf_op, n * n, (int)p, st);
  kern::tube_xform_f64(B, Bh, xf_op, s * s, (int)p, st);
  kern::tube_xform_f64(X, Zx, xf_fwd, n * s, (int)p, st);
  const int kid = prec == TSYLV_FP64 ? TSYLV_K_APPLY : TSYLV_K_APPLY_LOW;
  const bool prof = ctx && ctx->prof.on(kid);
  if (prec == TSYLV_FP64) {
    if (prof) ctx->prof.begin(kid, st);
    kern::apply_f64(Ah, Bh, Zx, Zy, nullptr, 1.0, 0.0, n, s, (int)p, st, variant);
    if (prof) ctx->prof.end(kid, st);
  } else {
    float* Vf = ws.template take<float>(N);
    float* Wf = ws.template take<float>(N);
    kern::convert_f64_f32(Zx, Vf, N, st);
    if (prec == TSYLV_BF16) {
      uint16_t* Ab = ws.template take<uint16_t>(kern::bf16_tiled_elems(n, (int)p));
      uint16_t* Bb = reinterpret_cast<uint16_t*>(ws.template take<float>(p * s * s));
      kern::tile_operator_bf16(Ah, Ab, n, (int)p, st);
      kern::convert_f64_bf16(Bh, Bb, p * s * s, st);
      uint16_t* Vt = ws.template take<uint16_t>(kern::bf16_vtiled_elems(n, s, (int)p));
      if (prof) ctx->prof.begin(kid, st);
      kern::apply_bf16(Ab, Bb, Vf, Vt, Wf, nullptr, 1.0, 0.0, n, s, (int)p, st, variant);
      if (prof) ctx->prof.end(kid, st);
    } else {
      float* Af = ws.template take<float>(p * n * n);
      float* Bf = ws.template take<float>(p * s * s);
      kern::convert_f64_f32(Ah, Af, p * n * n, st);
      kern::convert_f64_f32(Bh, Bf, p * s * s, st);
      if (prof) ctx->prof.begin(kid, st);
      kern::apply_f32(Af, Bf, Vf, Wf, nullptr, 1.0, 0.0, n, s, (int)p, st, variant);
      if (prof) ctx->prof.end(kid, st);
    }
    kern::convert_f32_f64(Wf, Zy, N, st);
  }
  kern::tube_xform_f64(Zy, Y, xf_inv, n * s, (int)p, st);
}

}  // namespace

int apply_spatial(Ctx& ctx, int64_t n, int64_t s, int64_t p, const double* A, const double* B,
                  const double* X, double* Y, int prec) {
  Workspace ws(ctx.arena, apply_workspace_bytes(n, s, p));
  apply_core(ws, ctx.stream, &ctx, n, s, p, A, B, X, Y, prec, ctx.tune.get(prec, n, s, p));
  ctx.sync();
  return TSYLV_OK;
}

void apply_spatial_into(char* buf, size_t bytes, hipStream_t st, int64_t n, int64_t s,
                        int64_t p, const double* A, const double* B, const double* X, double* Y,
                        int prec) {
  Carve c(buf, bytes);
  apply_core(c, st, nullptr, n, s, p, A, B, X, Y, prec, -1);
}

}  // namespace tsylv
