// TBAS(m): the restarted Tubal-Block-Arnoldi Sylvester solver of section 5.2
// (Algorithm 8), on the GPU.
//
// In the Fourier domain every step of the Tubal Block Arnoldi process
// (Algorithm 7) is a per-slice complex matrix operation (eq. (5) decouples
// the slices; the T-transpose is the per-slice conjugate transpose):
//   W_k = Ahat_k V_{j,k}                       (A only, not M)
//   H_{ij,k} = V_{i,k}^H W_k,  W_k -= V_{i,k} H_{ij,k}     (block CGS2 here;
//                                               the printed block MGS is
//                                               the same in exact arithmetic)
//   [V_{j+1}, H_{j+1,j}] = Tubal-QR(W)         (Algorithm 6)
// Tubal-QR with the Normalization of section 5.1 read as the symmetric
// positive tube (hat a_k = ||W_k||) is, slice by slice, the thin QR with a
// real positive diagonal; we compute it by shifted Cholesky QR followed by
// two plain Cholesky QR passes (shifted CholQR3: the shift keeps the first
// Cholesky factorisation defined for blocks with condition numbers up to
// about 1/eps, R = R3 R2 R1 keeps the diagonal positive), which reaches the
// same factors as the tubal modified Gram-Schmidt of Algorithm 6.
//
// Representation: R and X are kept in the orthonormal scaled planes of the
// Krylov solvers (slice k scaled by c_k = sqrt(w_k / p)); the basis blocks
// are the unscaled orthonormal Fourier slices Q_k.  Then H_ij is scale free,
// H0 (from the QR of R0) and the projected solution Y carry the factor c_k,
// and X += V Y stays in the scaled representation; the residual estimate of
// the proposition of section 5.2, ||H_{m+1,m} E_m Y||_F, is the plain norm
// of the stored slices (Parseval).
//
// The projected equation H_m Y - Y B = V_m^T R0 = [H0; 0] (eq. (TBslowrank))
// is solved in FP64.  Bhat_k does not change during a solve, so it is
// diagonalised once per solve on the host, Bhat_k = W_k diag(lam) W_k^{-1}
// (from its complex Schur form); with Z = Y W the equation splits into p_h s
// independent shifted block-Hessenberg systems, solved on the device
// (kern::proj_solve), and Y = Z W^{-1}.  Where that is not safe -- s above
// the device kernel's block limit, or an ill-conditioned eigenvector basis
// (kappa(W_k) > 1e8) -- or a shifted system hits a zero pivot, the cycle uses
// the host Bartels-Stewart solve with the Schur form of Bhat_k (triangular
// recursion over the columns, host_linalg), the slices spread over host
// threads.  TSYLV_TBA_HOST_PROJECTED=1 in the environment forces the host
// solve (used by the tests to compare the two).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <thread>
#include <vector>

#include "host_linalg.hpp"
#include "kernels.hpp"
#include "runtime.hpp"
#include "solvers.hpp"

namespace tsylv {

namespace {

using host::cplx;
constexpr double kEps = 2.220446049250313e-16;

// Planar buffer [plane][col][row] <-> per-slice complex matrix (column-major).
void unpack(const double* buf, int p, int k, int rows, int cols, cplx* out) {
  int qr, qi;
  slice_planes(p, k, qr, qi);
  const size_t pl = (size_t)rows * cols;
  for (size_t e = 0; e < pl; ++e)
    out[e] = cplx(buf[qr * pl + e], qi < 0 ? 0.0 : buf[qi * pl + e]);
}

void pack(const cplx* in, int p, int k, int rows, int cols, double* buf) {
  int qr, qi;
  slice_planes(p, k, qr, qi);
  const size_t pl = (size_t)rows * cols;
  for (size_t e = 0; e < pl; ++e) {
    buf[qr * pl + e] = in[e].real();
    if (qi >= 0) buf[qi * pl + e] = in[e].imag();
  }
}

template <typename F>
void parallel_slices(int ph, F&& f) {
  int nt = (int)std::thread::hardware_concurrency();
  if (nt < 1) nt = 1;
  if (nt > 16) nt = 16;
  if (nt > ph) nt = ph;
  if (nt <= 1) {
    for (int k = 0; k < ph; ++k) f(k);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      for (int k = t; k < ph; k += nt) f(k);
    });
  for (auto& x : th) x.join();
}

struct TbaWS {
  int64_t n, s, p, N, ldv;
  int m, ph;
  double *R, *T, *basis, *G, *Gq, *Rinv, *Y, *partial;
  double *part, *d_ww;
  int nchunks;
  double* V(int j) const { return basis + (int64_t)j * ldv; }
};

// Largest split-K partial buffer over the Gram products of one cycle.
int64_t tba_partial_elems(int64_t n, int64_t s, int64_t p, int m) {
  int64_t e = 0;
  for (int j = 1; j <= m; ++j) e = std::max(e, kern::zgemm_partial_elems(j * s, s, n, (int)p));
  return e;
}

// Device buffers of the projected solve (interleaved complex doubles).
// The device-resident cycle: projected solve and Tubal-QR factorisations on
// the GPU (s <= 64).  `out` is the one block read back per cycle: ||R||^2,
// the estimate terms of every slice and the flags (QR of R0, QR of step j,
// projected solve).
struct ProjWS {
  double *Hm = nullptr, *lam = nullptr, *D = nullptr, *z = nullptr, *Wrk = nullptr, *U = nullptr,
         *Gp = nullptr;
  double *W = nullptr, *Winv = nullptr, *Hlast = nullptr, *G2 = nullptr, *H0 = nullptr,
         *Rq = nullptr, *out = nullptr;
  int* info = nullptr;
  static bool possible(int64_t s) {
    return s <= kern::proj_max_block() && s <= kern::cholqr_max_block();
  }
  static int64_t out_doubles(int64_t p, int m) { return 1 + num_slices((int)p) + (m + 3); }
  static size_t bytes(int64_t s, int64_t p, int m) {
    if (!possible(s)) return 0;
    const int64_t ph = num_slices((int)p), ms = (int64_t)m * s, nsys = ph * s;
    return Workspace::bytes_for(2 * ph * ms * ms, 8) + Workspace::bytes_for(2 * nsys, 8) +
           Workspace::bytes_for(2 * ph * s * s, 8) + Workspace::bytes_for(2 * nsys * ms, 8) +
           Workspace::bytes_for(2 * 2 * nsys * s * ms, 8) +
           Workspace::bytes_for(2 * nsys * kern::proj_u_stride((int)s, m), 8) +
           Workspace::bytes_for(kern::proj_g_doubles((int)s, (int)nsys), 8) +
           Workspace::bytes_for(nsys, 4) + 3 * Workspace::bytes_for(2 * ph * s * s, 8) +
           Workspace::bytes_for(p * ms * s, 8) + 2 * Workspace::bytes_for(p * s * s, 8) +
           Workspace::bytes_for(out_doubles(p, m), 8);
  }
  void carve(Workspace& ws, int64_t s, int64_t p, int m) {
    if (!possible(s)) return;
    const int64_t ph = num_slices((int)p), ms = (int64_t)m * s, nsys = ph * s;
    Hm = ws.take<double>(2 * ph * ms * ms);
    lam = ws.take<double>(2 * nsys);
    D = ws.take<double>(2 * ph * s * s);
    z = ws.take<double>(2 * nsys * ms);
    Wrk = ws.take<double>(2 * 2 * nsys * s * ms);  // two buffers (ping-pong by panel)
    U = ws.take<double>(2 * nsys * kern::proj_u_stride((int)s, m));
    Gp = ws.take<double>(kern::proj_g_doubles((int)s, (int)nsys));
    info = ws.take<int>(nsys);
    W = ws.take<double>(2 * ph * s * s);
    Winv = ws.take<double>(2 * ph * s * s);
    Hlast = ws.take<double>(2 * ph * s * s);
    G2 = ws.take<double>(p * ms * s);
    H0 = ws.take<double>(p * s * s);
    Rq = ws.take<double>(p * s * s);
    out = ws.take<double>(out_doubles(p, m));
  }
};

size_t tba_ws_bytes(int64_t n, int64_t s, int64_t p, int m) {
  const int64_t N = n * s * p, ldv = round_up(N, 64), ms = (int64_t)m * s;
  const int64_t part = tba_partial_elems(n, s, p, m);
  return setup_bytes(n, s, p) + 2 * Workspace::bytes_for(N, 8) +
         Workspace::bytes_for((int64_t)(m + 1) * ldv, 8) + Workspace::bytes_for(p * ms * s, 8) +
         2 * Workspace::bytes_for(p * s * s, 8) + Workspace::bytes_for(p * ms * s, 8) +
         Workspace::bytes_for(part, 8) + Workspace::bytes_for(kern::mdot_chunks(N) * 2, 8) +
         Workspace::bytes_for(8, 8) + ProjWS::bytes(s, p, m);
}

double dev_norm2(Ctx& ctx, const TbaWS& w, const double* v) {
  kern::mdot_partial((const double*)nullptr, 0, 0, v, w.N, w.part, 2, 1, ctx.stream);
  kern::reduce_partials(w.part, w.nchunks, 2, 1, w.d_ww, ctx.stream);
  double h = 0.0;
  TSYLV_HIP(hipMemcpyAsync(&h, w.d_ww, sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  ctx.sync();
  return h;
}

// Tubal-QR (Algorithm 6) of the n x s block in `Win`, slice by slice, by
// shifted CholQR3: Qout receives the orthonormal slices, Rk[k] (s x s, upper
// triangular, real positive diagonal) the R factor of slice k.  With
// `scaled` the block is in scaled planes and the diagonal is divided by c_k
// for the tube test.  Returns false on a non-invertible tube (Normalization
// breakdown).
bool tubal_qr(Ctx& ctx, const TbaWS& w, const double* Win, double* Qout,
              std::vector<std::vector<cplx>>& Rk, bool scaled, double* hbuf, double* rinv) {
  const int s = (int)w.s, p = (int)w.p, ph = w.ph;
  const int64_t n = w.n, ns = n * w.s, ss = w.s * w.s;
  std::vector<std::vector<cplx>> Racc(ph, std::vector<cplx>((size_t)s * s));
  bool ok = true;
  const double* src = Win;
  constexpr int kPasses = 3;
  // Shift of the first pass (Fukaya et al., shifted CholeskyQR):
  // sigma = 11 (n s + s (s + 1)) u ||W_k||_2^2, with trace(G_k) >= ||W_k||_2^2.
  const double shift_factor = 11.0 * ((double)n * s + (double)s * (s + 1)) * kEps;
  for (int pass = 0; pass < kPasses; ++pass) {
    // Gram of every slice: W_k^H W_k
    kern::zgemm(kern::dense_pmat(src, ns, n), true, kern::dense_pmat(src, ns, n), w.Gq, ss,
                w.s, w.s, w.s, n, 1.0, 0.0, p, w.partial, ctx.stream);
    TSYLV_HIP(hipMemcpyAsync(hbuf, w.Gq, (size_t)p * ss * 8, hipMemcpyDeviceToHost, ctx.stream));
    ctx.sync();
    std::fill(rinv, rinv + (size_t)p * ss, 0.0);
    std::vector<int> good(ph, 1);
    parallel_slices(ph, [&](int k) {
      std::vector<cplx> G((size_t)s * s), Ri((size_t)s * s);
      unpack(hbuf, p, k, s, s, G.data());
      if (pass == 0) {
        double tr = 0.0;
        for (int i = 0; i < s; ++i) tr += G[i + (size_t)s * i].real();
        for (int i = 0; i < s; ++i) G[i + (size_t)s * i] += shift_factor * tr;
      }
      if (!host::cholesky_upper(G.data(), s, 1e3 * kEps * kEps)) {
        good[k] = 0;
        return;
      }
      host::tri_inv_upper(G.data(), Ri.data(), s);
      pack(Ri.data(), p, k, s, s, rinv);  // writes only this slice's planes
      if (pass == 0) {
        Racc[k] = G;
      } else {
        std::vector<cplx> t((size_t)s * s);
        host::matmul(G.data(), Racc[k].data(), t.data(), s, s, s);  // R = R_pass ... R_1
        Racc[k] = t;
      }
    });
    for (int k = 0; k < ph; ++k) ok = ok && good[k];
    if (!ok) return false;
    TSYLV_HIP(hipMemcpyAsync(w.Rinv, rinv, (size_t)p * ss * 8, hipMemcpyHostToDevice,
                             ctx.stream));
    // passes alternate between the two buffers and end in Qout
    double* dst = ((kPasses - 1 - pass) % 2 == 0) ? Qout : w.T;
    if (dst == src) dst = (dst == w.T) ? Qout : w.T;
    kern::zgemm(kern::dense_pmat(src, ns, n), false, kern::dense_pmat(w.Rinv, ss, w.s), dst, ns, n,
                n, w.s, w.s, 1.0, 0.0, p, nullptr, ctx.stream);
    ctx.sync();  // rinv (host) must outlive the copy
    src = dst;
  }
  if (src != Qout)
    TSYLV_HIP(hipMemcpyAsync(Qout, src, w.N * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
  for (int k = 0; k < ph; ++k) Rk[k] = Racc[k];
  // Tube test of the Normalization: hat a_k = R_k(jj, jj) (/ c_k in scaled planes)
  for (int jj = 0; jj < s; ++jj) {
    double amin = INFINITY, amax = 0.0;
    for (int k = 0; k < ph; ++k) {
      const bool real_slice = (k == 0) || (2 * k == p);
      const double ck = std::sqrt((real_slice ? 1.0 : 2.0) / p);
      double a = Rk[k][jj + (size_t)s * jj].real();
      if (scaled) a /= ck;
      amin = std::min(amin, a);
      amax = std::max(amax, a);
    }
    if (!(amin > 16.0 * kEps * amax)) return false;
  }
  return true;
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

size_t tba_workspace_bytes(int64_t n, int64_t s, int64_t p, int m) {
  return tba_ws_bytes(n, s, p, m);
}

namespace {

// Device Tubal-QR of the n x s block Win into Qout (may alias Win): three
// shifted-Cholesky-QR passes with the small factorisations on the device;
// Racc receives R (planar s x s per slice); *flag |= 1 on a failed
// factorisation or a non-invertible tube.  No host synchronisation.
void tubal_qr_dev(Ctx& ctx, const TbaWS& w, const double* Win, double* Qout, double* Racc,
                  bool scaled, int* flag) {
  const int s = (int)w.s, p = (int)w.p;
  const int64_t n = w.n, ns = n * w.s, ss = w.s * w.s;
  const double shift_factor = 11.0 * ((double)n * s + (double)s * (s + 1)) * kEps;
  constexpr int kPasses = 3;
  const double* src = Win;
  for (int pass = 0; pass < kPasses; ++pass) {
    kern::zgemm(kern::dense_pmat(src, ns, n), true, kern::dense_pmat(src, ns, n), w.Gq, ss,
                w.s, w.s, w.s, n, 1.0, 0.0, p, w.partial, ctx.stream);
    kern::cholqr_pass(w.Gq, w.Rinv, Racc, s, p, shift_factor, pass == 0, 1e3 * kEps * kEps,
                      flag, ctx.stream);
    double* dst = ((kPasses - 1 - pass) % 2 == 0) ? Qout : w.T;
    if (dst == src) dst = (dst == w.T) ? Qout : w.T;
    kern::zgemm(kern::dense_pmat(src, ns, n), false, kern::dense_pmat(w.Rinv, ss, w.s), dst, ns,
                n, n, w.s, w.s, 1.0, 0.0, p, nullptr, ctx.stream);
    src = dst;
  }
  if (src != Qout)
    TSYLV_HIP(hipMemcpyAsync(Qout, src, w.N * sizeof(double), hipMemcpyDeviceToDevice,
                             ctx.stream));
  kern::tube_test(Racc, s, p, scaled, flag, ctx.stream);
}

}  // namespace

int tba_solve(Ctx& ctx, int64_t n, int64_t s, int64_t p, const double* A, const double* B,
              const double* C, double* X, const tsylv_opts& o, tsylv_info& info) {
  auto t0 = std::chrono::steady_clock::now();
  // The block Krylov space of one slice must fit in C^n: (m + 1) s <= n.
  int m = o.m;
  if ((int64_t)(m + 1) * s > n) m = (int)(n / s) - 1;
  if (m < 1) throw Error(TSYLV_EINVAL, "TBA needs n >= 2 s");
  hipStream_t st = ctx.stream;
  Workspace ws(ctx.arena, tba_ws_bytes(n, s, p, m));
  Setup S = setup_fourier(ctx, st, true, ws, n, s, p, A, B, C, X, o.x0_given != 0);
  const int var64 = ctx.tune.get(TSYLV_FP64, n, s, p);
  TbaWS w;
  w.n = n;
  w.s = s;
  w.p = p;
  w.N = n * s * p;
  w.ldv = round_up(w.N, 64);
  w.m = m;
  w.ph = num_slices((int)p);
  const int64_t ms = (int64_t)m * s, ns = n * s, ss = s * s;
  w.R = ws.take<double>(w.N);
  w.T = ws.take<double>(w.N);
  w.basis = ws.take<double>((int64_t)(m + 1) * w.ldv);
  w.G = ws.take<double>(p * ms * s);
  w.Gq = ws.take<double>(p * ss);
  w.Rinv = ws.take<double>(p * ss);
  w.Y = ws.take<double>(p * ms * s);
  w.partial = ws.take<double>(tba_partial_elems(n, s, p, m));
  w.nchunks = kern::mdot_chunks(w.N);
  w.part = ws.take<double>((int64_t)w.nchunks * 2);
  w.d_ww = ws.take<double>(8);
  const int ph = w.ph, si = (int)s, msi = (int)ms;
  ProjWS pw;
  pw.carve(ws, s, p, m);

  // Bhat (operator planes, unscaled) on the host for the projected solves.
  std::vector<double> hB((size_t)p * ss);
  TSYLV_HIP(hipMemcpyAsync(hB.data(), S.Bh, hB.size() * 8, hipMemcpyDeviceToHost, st));
  const double cnorm = std::sqrt(dev_norm2(ctx, w, S.Zc));
  // Bhat_k = W_k diag(lam_k) W_k^{-1}, once per solve, for the device solve.
  const char* force_host = std::getenv("TSYLV_TBA_HOST_PROJECTED");
  bool dev_proj = ProjWS::possible(s) && !(force_host && force_host[0] == '1');
  std::vector<std::vector<cplx>> Wk(ph), Wik(ph);
  std::vector<cplx> lam_all((size_t)ph * si);
  if (dev_proj) {
    std::vector<double> kap(ph, INFINITY);
    parallel_slices(ph, [&](int k) {
      std::vector<cplx> T((size_t)ss), Uq((size_t)ss);
      unpack(hB.data(), (int)p, k, si, si, T.data());
      Wk[k].assign((size_t)ss, 0.0);
      Wik[k].assign((size_t)ss, 0.0);
      if (!host::schur(T.data(), Uq.data(), si)) return;
      kap[k] = host::eig_from_schur(T.data(), Uq.data(), si, &lam_all[(size_t)k * si],
                                    Wk[k].data(), Wik[k].data());
    });
    for (int k = 0; k < ph; ++k) dev_proj = dev_proj && kap[k] < 1e8;
  }
  info.steps = info.cycles = info.outer = 0;
  info.res_hist_len = 0;
  info.relres_est = 0.0;
  if (cnorm == 0.0) {
    TSYLV_HIP(hipMemsetAsync(X, 0, w.N * sizeof(double), st));
    ctx.sync();
    info.relres_true = 0.0;
    info.status = TSYLV_OK;
    info.seconds = seconds_since(t0);
    return TSYLV_OK;
  }
  int status = TSYLV_NOT_CONVERGED;

  if (dev_proj) {
    // eigenvalues and eigenvector bases of the Bhat_k (once per solve)
    std::vector<cplx> hW((size_t)ph * ss), hWi((size_t)ph * ss);
    for (int k = 0; k < ph; ++k) {
      std::copy(Wk[k].begin(), Wk[k].end(), hW.begin() + (size_t)k * ss);
      std::copy(Wik[k].begin(), Wik[k].end(), hWi.begin() + (size_t)k * ss);
    }
    TSYLV_HIP(hipMemcpyAsync(pw.lam, lam_all.data(), lam_all.size() * sizeof(cplx),
                             hipMemcpyHostToDevice, st));
    TSYLV_HIP(hipMemcpyAsync(pw.W, hW.data(), hW.size() * sizeof(cplx), hipMemcpyHostToDevice, st));
    TSYLV_HIP(hipMemcpyAsync(pw.Winv, hWi.data(), hWi.size() * sizeof(cplx),
                             hipMemcpyHostToDevice, st));
    ctx.sync();  // the host vectors go out of scope
    // The cycle out block: [0] ||R||^2, [1 .. ph] estimate terms, then the
    // int flags (QR of R0, QR of steps 0 .. m-1, projected solve).
    const int64_t nout = ProjWS::out_doubles(p, m);
    double* hout = ctx.host_buffer((size_t)nout);
    int* dflags = reinterpret_cast<int*>(pw.out + 1 + ph);
    const int nflags = m + 2;
    bool pending = false;  // a finished cycle whose flags are in `out`
    for (int cycle = 0;; ++cycle) {
      // R0 = C - M(X0) (Algorithm 8 step 2) and its norm, read back with the
      // previous cycle's flags and estimate: the one host round trip of a
      // cycle
      if (cycle == 0 && !o.x0_given) {
        TSYLV_HIP(hipMemcpyAsync(w.R, S.Zc, w.N * sizeof(double), hipMemcpyDeviceToDevice, st));
      } else {
        ProfScope ps(ctx, TSYLV_K_APPLY, st);
        kern::apply_f64(S.Ah, S.Bh, S.Zx, w.R, S.Zc, -1.0, 1.0, n, s, (int)p, st, var64);
      }
      kern::mdot_partial((const double*)nullptr, 0, 0, w.R, w.N, w.part, 2, 1, st);
      kern::reduce_partials(w.part, w.nchunks, 2, 1, pw.out, st);
      TSYLV_HIP(hipMemcpyAsync(hout, pw.out, nout * sizeof(double), hipMemcpyDeviceToHost, st));
      ctx.sync();
      if (pending) {
        const int* hf = reinterpret_cast<const int*>(hout + 1 + ph);
        if (hf[0]) throw Error(TSYLV_EBREAKDOWN, "Tubal-QR(R0)");
        for (int j = 0; j + 1 < m; ++j)
          if (hf[1 + j]) throw Error(TSYLV_EBREAKDOWN, "Tubal-QR in TBA");
        if (hf[m + 1]) throw Error(TSYLV_ESINGULAR, "projected Sylvester equation");
        double est2 = 0.0;
        if (!hf[m])  // a breakdown in the last QR means H_{m+1,m} = 0
          for (int k = 0; k < ph; ++k) est2 += hout[1 + k];
        info.relres_est = std::sqrt(est2) / cnorm;
        if (o.res_hist && info.res_hist_len < o.res_hist_cap)
          o.res_hist[info.res_hist_len++] = info.relres_est;
      }
      info.relres_true = std::sqrt(hout[0]) / cnorm;
      if (info.relres_true <= o.tol) {
        status = TSYLV_OK;
        break;
      }
      if (cycle >= o.max_cycles) break;
      info.cycles++;
      TSYLV_HIP(hipMemsetAsync(dflags, 0, nflags * sizeof(int), st));
      TSYLV_HIP(hipMemsetAsync(pw.Hm, 0, (size_t)ph * ms * ms * sizeof(cplx), st));
      // Algorithm 7 step 2: [V_1, H0] = Tubal-QR(R0)
      tubal_qr_dev(ctx, w, w.R, w.V(0), pw.H0, true, dflags);
      for (int j = 0; j < m; ++j) {
        const int64_t J = (int64_t)(j + 1) * s;
        double* W = w.V(j + 1);
        {
          ProfScope ps(ctx, TSYLV_K_APPLY, st);
          kern::apply_f64(S.Ah, nullptr, w.V(j), W, nullptr, 1.0, 0.0, n, s, (int)p, st,
                          var64);  // A only
        }
        // block CGS2: H_{0..j, j} = V^H W (twice), W -= V H
        const kern::PMat Vb{w.basis, ns, n, s, w.ldv};
        if (ctx.prof.on(TSYLV_K_ORTHO)) ctx.prof.begin(TSYLV_K_ORTHO, st);
        for (int pass = 0; pass < 2; ++pass) {
          double* G = pass == 0 ? w.G : pw.G2;
          kern::zgemm(Vb, true, kern::dense_pmat(W, ns, n), G, J * s, J, J, s, n, 1.0, 0.0,
                      (int)p, w.partial, st);
          kern::zgemm(Vb, false, kern::dense_pmat(G, J * s, J), W, ns, n, n, s, J, -1.0, 1.0,
                      (int)p, nullptr, st);
        }
        if (ctx.prof.on(TSYLV_K_ORTHO)) ctx.prof.end(TSYLV_K_ORTHO, st);
        // Tubal-QR(W) -> V_{j+1}, H_{j+1,j}
        tubal_qr_dev(ctx, w, W, W, pw.Rq, false, dflags + 1 + j);
        kern::hm_column(w.G, pw.G2, pw.Rq, pw.Hm, pw.Hlast, j, si, m, (int)p, st);
        info.steps++;
      }
      // Algorithm 8 step 3(b): Hm Y - Y Bhat = [H0; 0] per slice, through
      // the shifted systems (Hm_k - lam_{k,j} I) z = (H0_k W_k) e_j, then
      // Y_k = Z_k W_k^{-1} and the estimate ||H_{m+1,m} E_m^T Y||
      kern::proj_rhs(pw.H0, pw.W, pw.D, si, (int)p, st);
      kern::proj_solve(pw.Hm, pw.lam, pw.D, pw.z, pw.Wrk, pw.U, pw.Gp, pw.info, msi, si, m,
                       ph * si, st);
      kern::proj_check(pw.info, pw.z, (int64_t)ph * si, (int64_t)ph * si * msi,
                       dflags + m + 1, st);
      kern::proj_y(pw.z, pw.Winv, pw.Hlast, w.Y, pw.out + 1, si, m, (int)p, st);
      // Algorithm 8 step 3(c): X = X0 + V_m Y
      kern::zgemm(kern::PMat{w.basis, ns, n, s, w.ldv}, false, kern::dense_pmat(w.Y, ms * s, ms),
                  S.Zx, ns, n, n, s, ms, 1.0, 1.0, (int)p, nullptr, st);
      pending = true;
    }
  } else {
    // Host path (s > 64, an ill-conditioned eigenvector basis of some Bhat_k,
    // or TSYLV_TBA_HOST_PROJECTED=1): Tubal-QR factorisations and the
    // projected solves (Bartels-Stewart with the Schur form of Bhat_k) on
    // the host, every step's small results copied back.
    const size_t nss = (size_t)p * ss, nG = (size_t)p * ms * s;
    const size_t total = 2 * nss + 3 * nG;
    std::vector<double> stage(total);
    double* q = stage.data();
    double* qr_buf = q;
    q += nss;
    double* qr_rinv = q;
    q += nss;
    double* hG = q;
    q += nG;
    double* hG2 = q;
    q += nG;
    double* hY = q;
    q += nG;
    std::fill(hY, hY + nG, 0.0);
    std::vector<std::vector<cplx>> Hk(ph, std::vector<cplx>((size_t)(ms + s) * ms));
    std::vector<std::vector<cplx>> H0(ph, std::vector<cplx>((size_t)ss));
    std::vector<std::vector<cplx>> Rq(ph, std::vector<cplx>((size_t)ss));

    for (int cycle = 0;; ++cycle) {
      // R0 = C - M(X0) (Algorithm 8 step 2)
      if (cycle == 0 && !o.x0_given) {
        TSYLV_HIP(hipMemcpyAsync(w.R, S.Zc, w.N * sizeof(double), hipMemcpyDeviceToDevice, st));
      } else {
        ProfScope ps(ctx, TSYLV_K_APPLY, st);
        kern::apply_f64(S.Ah, S.Bh, S.Zx, w.R, S.Zc, -1.0, 1.0, n, s, (int)p, st, var64);
      }
      info.relres_true = std::sqrt(dev_norm2(ctx, w, w.R)) / cnorm;
      if (info.relres_true <= o.tol) {
        status = TSYLV_OK;
        break;
      }
      if (cycle >= o.max_cycles) break;
      info.cycles++;
      // Algorithm 7 step 2: [V_1, H0] = Tubal-QR(R0)
      if (!tubal_qr(ctx, w, w.R, w.V(0), H0, true, qr_buf, qr_rinv))
        throw Error(TSYLV_EBREAKDOWN, "Tubal-QR(R0)");
      for (auto& h : Hk) std::fill(h.begin(), h.end(), cplx(0.0));
      for (int j = 0; j < m; ++j) {
        const int64_t J = (int64_t)(j + 1) * s;
        double* W = w.V(j + 1);
        {
          ProfScope ps(ctx, TSYLV_K_APPLY, st);
          kern::apply_f64(S.Ah, nullptr, w.V(j), W, nullptr, 1.0, 0.0, n, s, (int)p, st,
                          var64);  // A only
        }
        // block CGS2: H_{0..j, j} = V^H W (twice), W -= V H
        const kern::PMat Vb{w.basis, ns, n, s, w.ldv};
        if (ctx.prof.on(TSYLV_K_ORTHO)) ctx.prof.begin(TSYLV_K_ORTHO, st);
        for (int pass = 0; pass < 2; ++pass) {
          kern::zgemm(Vb, true, kern::dense_pmat(W, ns, n), w.G, J * s, J, J, s, n, 1.0, 0.0,
                      (int)p, w.partial, st);
          kern::zgemm(Vb, false, kern::dense_pmat(w.G, J * s, J), W, ns, n, n, s, J, -1.0, 1.0,
                      (int)p, nullptr, st);
          double* dst = pass == 0 ? hG : hG2;
          TSYLV_HIP(hipMemcpyAsync(dst, w.G, (size_t)p * J * s * 8, hipMemcpyDeviceToHost, st));
        }
        if (ctx.prof.on(TSYLV_K_ORTHO)) ctx.prof.end(TSYLV_K_ORTHO, st);
        ctx.sync();
        const int Ji = (int)J;
        parallel_slices(ph, [&](int k) {
          std::vector<cplx> g1((size_t)Ji * si), g2((size_t)Ji * si);
          unpack(hG, (int)p, k, Ji, si, g1.data());
          unpack(hG2, (int)p, k, Ji, si, g2.data());
          const int ldh = msi + si;
          for (int c = 0; c < si; ++c)
            for (int r = 0; r < Ji; ++r)
              Hk[k][r + (size_t)ldh * (j * si + c)] = g1[r + (size_t)Ji * c] + g2[r + (size_t)Ji * c];
        });
        // Tubal-QR(W) -> V_{j+1}, H_{j+1,j}
        const bool qr_ok = tubal_qr(ctx, w, W, W, Rq, false, qr_buf, qr_rinv);
        if (!qr_ok) {
          if (j < m - 1) throw Error(TSYLV_EBREAKDOWN, "Tubal-QR in TBA");
          for (auto& r : Rq) std::fill(r.begin(), r.end(), cplx(0.0));  // H_{m+1,m} = 0
        }
        for (int k = 0; k < ph; ++k) {
          const int ldh = msi + si;
          for (int c = 0; c < si; ++c)
            for (int r = 0; r < si; ++r)
              Hk[k][(size_t)(J + r) + (size_t)ldh * (j * si + c)] = Rq[k][r + (size_t)si * c];
        }
        info.steps++;
      }
      // Algorithm 8 step 3(b): H_m Y - Y B = [H0; 0] per slice
      std::vector<int> good(ph, 1);
      double est2 = 0.0;
      std::vector<double> est_k(ph, 0.0);
      auto finish_slice = [&](int k, const std::vector<cplx>& Yk) {
        const int ldh = msi + si;
        pack(Yk.data(), (int)p, k, msi, si, hY);
        // residual estimate: || H_{m+1,m} Y_m ||_F for this slice
        double e = 0.0;
        for (int c = 0; c < si; ++c)
          for (int r = 0; r < si; ++r) {
            cplx v = 0.0;
            for (int l = 0; l < si; ++l)
              v += Hk[k][(size_t)(msi + r) + (size_t)ldh * ((m - 1) * si + l)] *
                   Yk[(size_t)((m - 1) * si + l) + (size_t)msi * c];
            e += (k == 0 || 2 * k == (int)p) ? v.real() * v.real() : std::norm(v);
          }
        est_k[k] = e;
      };
      {
        // host: Bartels-Stewart with the Schur form of Bhat_k (Algorithm 5)
        parallel_slices(ph, [&](int k) {
          const int ldh = msi + si;
          std::vector<cplx> Hm((size_t)msi * msi), Bk((size_t)si * si), C1((size_t)msi * si, 0.0),
              Yk((size_t)msi * si);
          for (int c = 0; c < msi; ++c)
            for (int r = 0; r < msi; ++r) Hm[r + (size_t)msi * c] = Hk[k][r + (size_t)ldh * c];
          unpack(hB.data(), (int)p, k, si, si, Bk.data());
          for (int c = 0; c < si; ++c)
            for (int r = 0; r < si; ++r) C1[r + (size_t)msi * c] = H0[k][r + (size_t)si * c];
          if (!host::sylvester_banded(Hm.data(), msi, si, Bk.data(), si, C1.data(), Yk.data())) {
            good[k] = 0;
            return;
          }
          finish_slice(k, Yk);
        });
      }
      for (int k = 0; k < ph; ++k) {
        if (!good[k]) throw Error(TSYLV_ESINGULAR, "projected Sylvester equation");
        est2 += est_k[k];
      }
      info.relres_est = std::sqrt(est2) / cnorm;
      if (o.res_hist && info.res_hist_len < o.res_hist_cap)
        o.res_hist[info.res_hist_len++] = info.relres_est;
      // Algorithm 8 step 3(c): X = X0 + V_m Y
      TSYLV_HIP(hipMemcpyAsync(w.Y, hY, nG * 8, hipMemcpyHostToDevice, st));
      kern::zgemm(kern::PMat{w.basis, ns, n, s, w.ldv}, false, kern::dense_pmat(w.Y, ms * s, ms),
                  S.Zx, ns, n, n, s, ms, 1.0, 1.0, (int)p, nullptr, st);
      ctx.sync();
    }
  }
  {
    ProfScope ps(ctx, TSYLV_K_XFORM, st);
    kern::tube_xform_f64(S.Zx, X, S.xf_inv, n * s, (int)p, st);
  }
  ctx.sync();
  info.status = status;
  info.seconds = seconds_since(t0);
  return status;
}

}  // namespace tsylv
