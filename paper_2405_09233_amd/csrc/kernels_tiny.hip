// Restarted tGMRES(m) and tFOM(m) (Algorithm 3) of one small instance in
// one workgroup: the whole solve -- every restart cycle, every Arnoldi step
// and the true residual after each cycle -- in a single launch.  For
// instances of a few hundred to a few thousand unknowns a step of the
// multi-launch driver is a handful of dependent launches and a host round
// trip (tens of microseconds); here it is a handful of barriers.
//
// The process is the multi-launch driver's: vectors in the orthonormal
// Fourier planes (M acts slice by slice as Ahat_k V_k - V_k Bhat_k, eq. (5)),
// classical Gram-Schmidt with one reorthogonalisation, the breakdown test
// h_{j+1,j} <= 16 eps ||M v_j||, progressive Givens QR of the Hessenberg
// matrix with the tGMRES estimate |gamma_{j+1}| (section 3.3), the restart
// test on the true residual C - M(X).  tFOM's y solves the square system
// H_k y = beta e1 (section 3.2) through the same rotations: the first k-1 of
// them make H_k upper triangular with the last diagonal entry and the last
// right-hand side entry taken before the k-th rotation, so its estimate
// h_{k+1,k} |y_k| needs no factorisation of its own.
//
// Storage: the iterate, the operator planes, the rotations and as many
// basis vectors as fit in LDS; the other basis vectors and the rotated
// Hessenberg columns in global memory (reached through flat pointers).
// Sums over a vector are fixed-order (eight lanes per sum, a fixed tree):
// runs are bitwise reproducible.
#include <algorithm>

#include "kernels.hpp"

namespace tsylv {
namespace kern {

namespace {

constexpr int kYT = 256;           // threads of the workgroup
constexpr int kYD = 8;             // fewest lanes that share one dot product
constexpr int kYLds = 160 * 1024;  // LDS of one workgroup (bytes)
constexpr int64_t kYMaxN = 8192;   // largest n s p handled here
constexpr int kYMaxM = 1024;       // longest restart handled here
constexpr int64_t kYMaxMN = 1 << 18;  // largest m n s p (bounds a cycle's basis work)
constexpr int kYScal = 16;         // scalars exchanged through LDS

// One solve's arguments (TinyJob): the p planes of Ahat (n x n) and Bhat
// (s x s), unscaled Fourier slices; C in orthonormal planes (N = n s p);
// X0 on entry when x0_given and X on exit in Zx; Vg: (m + 1) N doubles for
// the basis slots past the lslots in LDS; Rg: m x m, the rotated Hessenberg
// columns (column j: j + 1 entries); hist: hist_cap relative residual
// estimates; out: the result record of kTinyRecord doubles.
using TinyArgs = TinyJob;

// LDS doubles besides the basis slots: X, the operator planes, cs, sn, g,
// two projections, the current column, the scalars.
int64_t fixed_doubles(int64_t n, int64_t s, int64_t p, int m) {
  return n * s * p + p * (n * n + s * s) + 6 * ((int64_t)m + 2) + kYScal;
}

// w = M(v) = Ahat v - v Bhat, slice by slice on the planes (slice 0 and,
// for even p, slice p/2 real; slice k otherwise planes 2k-1 (Re), 2k (Im)).
__device__ void tiny_apply(int n, int s, int p, const double* A, const double* B, const double* v,
                           double* w) {
  const int ns = n * s, ph = p / 2 + 1;
  for (int it = threadIdx.x; it < ph * ns; it += kYT) {
    const int k = it / ns, e = it % ns, i = e % n, c = e / n;
    const bool real = k == 0 || 2 * k == p;
    const int qr = k == 0 ? 0 : (real ? p - 1 : 2 * k - 1);
    const double* Ar = A + (int64_t)qr * n * n;
    const double* Br = B + (int64_t)qr * s * s;
    const double* Vr = v + (int64_t)qr * ns;
    if (real) {
      double acc = 0.0;
#pragma unroll 4
      for (int l = 0; l < n; ++l) acc = fma(Ar[i + n * l], Vr[l + n * c], acc);
#pragma unroll 4
      for (int l = 0; l < s; ++l) acc = fma(-Vr[i + n * l], Br[l + s * c], acc);
      w[(int64_t)qr * ns + e] = acc;
    } else {
      const double* Ai = Ar + n * n;
      const double* Bi = Br + s * s;
      const double* Vi = Vr + ns;
      double re = 0.0, im = 0.0;
#pragma unroll 4
      for (int l = 0; l < n; ++l) {
        const double ar = Ar[i + n * l], ai = Ai[i + n * l];
        const double vr = Vr[l + n * c], vi = Vi[l + n * c];
        re = fma(ar, vr, re);
        re = fma(-ai, vi, re);
        im = fma(ar, vi, im);
        im = fma(ai, vr, im);
      }
#pragma unroll 4
      for (int l = 0; l < s; ++l) {
        const double vr = Vr[i + n * l], vi = Vi[i + n * l];
        const double br = Br[l + s * c], bi = Bi[l + s * c];
        re = fma(-vr, br, re);
        re = fma(vi, bi, re);
        im = fma(-vr, bi, im);
        im = fma(-vi, br, im);
      }
      w[(int64_t)qr * ns + e] = re;
      w[(int64_t)(qr + 1) * ns + e] = im;
    }
  }
}

// out[i] = x_i . y for i < cnt (x_i = vec(i)): L adjacent lanes per sum
// (the largest power of two with L cnt <= kYT, 8 <= L <= 64), four partial
// sums per lane over its elements (loads of four elements in flight), then
// a fixed tree.
template <typename Vec>
__device__ void tiny_dots(Vec vec, int cnt, const double* y, int N, double* out) {
  int L = 64;
  while (L > kYD && L * cnt > kYT) L >>= 1;
  const int part = threadIdx.x % L, grp = threadIdx.x / L, per = kYT / L;
  for (int i0 = 0; i0 < cnt; i0 += per) {
    const int i = i0 + grp;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (i < cnt) {
      const double* x = vec(i);
      int e = part;
      for (; e + 3 * L < N; e += 4 * L) {
        a0 = fma(x[e], y[e], a0);
        a1 = fma(x[e + L], y[e + L], a1);
        a2 = fma(x[e + 2 * L], y[e + 2 * L], a2);
        a3 = fma(x[e + 3 * L], y[e + 3 * L], a3);
      }
      for (; e < N; e += L) a0 = fma(x[e], y[e], a0);
    }
    double acc = (a0 + a1) + (a2 + a3);
    for (int o = 1; o < L; o <<= 1) acc += __shfl_xor(acc, o);
    if (part == 0 && i < cnt) out[i] = acc;
  }
}

// w -= sum_{i < cnt} h_i x_i, in index order per element; with wsq, each
// wave's sum of the new w^2 (a fixed tree) to wsq[wave].
template <typename Vec>
__device__ void tiny_sub(double* w, Vec vec, int cnt, const double* h, int N, double* wsq) {
  double sq = 0.0;
  for (int e = threadIdx.x; e < N; e += kYT) {
    double acc = w[e];
#pragma unroll 4
    for (int i = 0; i < cnt; ++i) acc = fma(-h[i], vec(i)[e], acc);
    w[e] = acc;
    sq = fma(acc, acc, sq);
  }
  if (wsq) {
    for (int o = 1; o < 64; o <<= 1) sq += __shfl_xor(sq, o);
    if ((threadIdx.x & 63) == 0) wsq[threadIdx.x >> 6] = sq;
  }
}

// x of lane `l` (wave-uniform)
__device__ __forceinline__ double rlane(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}

// y of R y = r for the k x k upper triangular R (column l at R + m l), with
// the last diagonal entry dlast and the last right-hand side entry rlast in
// place of R's and r's.  Wave 0, row i in lane i (k <= 64), column by
// column from the last, the next column's entries loaded ahead.  Returns
// false on a zero diagonal (or, if `finite`, a non-finite y).
__device__ bool tiny_back_wave(const double* R, int m, int k, const double* r, double dlast,
                               double rlast, bool finite, double* y) {
  const int lane = threadIdx.x;
  double tr = lane < k ? (lane == k - 1 ? rlast : r[lane]) : 0.0;
  double yv = 0.0;
  double rn = lane < k ? R[lane + (int64_t)m * (k - 1)] : 0.0;
  bool ok = true;
  for (int l = k - 1; l >= 0; --l) {
    const double rc = rn;  // column l, rows 0 .. l
    rn = (l > 0 && lane < l) ? R[lane + (int64_t)m * (l - 1)] : 0.0;
    const double d = l == k - 1 ? dlast : rlane(rc, l);
    if (d == 0.0) {
      ok = false;
      break;
    }
    const double yl = rlane(tr, l) / d;
    if (finite && !isfinite(yl)) {
      ok = false;
      break;
    }
    if (lane == l) yv = yl;
    if (lane < l) tr = fma(-rc, yl, tr);
  }
  if (lane < k) y[lane] = yv;
  return ok;
}

// The same solve by one thread, for k > 64.
__device__ bool tiny_back_serial(const double* R, int m, int k, const double* r, double dlast,
                                 double rlast, bool finite, double* y) {
  for (int ii = k - 1; ii >= 0; --ii) {
    double t = ii == k - 1 ? rlast : r[ii];
    for (int l = ii + 1; l < k; ++l) t -= R[ii + (int64_t)m * l] * y[l];
    const double d = ii == k - 1 ? dlast : R[ii + (int64_t)m * ii];
    if (d == 0.0) return false;
    y[ii] = t / d;
    if (finite && !isfinite(y[ii])) return false;
  }
  return true;
}

__device__ void tiny_solve(const TinyArgs& a) {
  extern __shared__ double lds[];
  const int t = threadIdx.x;
  const int n = a.n, s = a.s, p = a.p, m = a.m, N = n * s * p;
  double* X = lds;
  double* A = X + N;
  double* B = A + (int64_t)p * n * n;
  double* cs = B + (int64_t)p * s * s;
  double* sn = cs + (m + 2);
  double* g = sn + (m + 2);
  double* h1 = g + (m + 2);
  double* h2 = h1 + (m + 2);  // second projection; y at the end of a cycle
  double* col = h2 + (m + 2);
  double* sc = col + (m + 2);
  double* Vl = sc + kYScal;
  // basis slot i: in LDS for i < lslots, else in global memory; steps whose
  // slots are all in LDS use lslot, so that their accesses are LDS accesses
  auto lslot = [&](int i) -> double* { return Vl + (int64_t)i * N; };
  auto slot = [&](int i) -> double* {
    return i < a.lslots ? Vl + (int64_t)i * N : a.Vg + (int64_t)i * N;
  };

  for (int e = t; e < p * n * n; e += kYT) A[e] = a.Ah[e];
  for (int e = t; e < p * s * s; e += kYT) B[e] = a.Bh[e];
  for (int e = t; e < N; e += kYT) X[e] = a.x0_given ? a.Zx[e] : 0.0;
  if (t < kYScal) sc[t] = 0.0;
  __syncthreads();
  tiny_dots([&](int) { return a.Zc; }, 1, a.Zc, N, sc);
  __syncthreads();
  const double cnorm = sqrt(sc[0]);
  const double stop = a.tol * cnorm;

  // One Arnoldi step (Algorithm 2 step 3) and its Givens update; returns
  // true when the cycle ends at this step.
  int status = TSYLV_NOT_CONVERGED, steps = 0, cycles = 0;
  double rt = 0.0, est = 0.0;
  bool any_est = false;
  auto step = [&](auto vs, int j) -> bool {
    double* W = vs(j + 1);
    tiny_apply(n, s, p, A, B, vs(j), W);
    __syncthreads();
    tiny_dots(vs, j + 2, W, N, h1);  // h1[0..j], and ||W||^2 in h1[j + 1]
    __syncthreads();
    tiny_sub(W, vs, j + 1, h1, N, (double*)nullptr);
    __syncthreads();
    tiny_dots(vs, j + 1, W, N, h2);
    __syncthreads();
    tiny_sub(W, vs, j + 1, h2, N, sc + 8);  // ||w||^2 by wave in sc[8..11]
    __syncthreads();
    const double w0 = sqrt(h1[j + 1]);
    double hn = sqrt(((sc[8] + sc[9]) + sc[10]) + sc[11]);
    const bool brk = !(hn > 16.0 * 2.220446049250313e-16 * w0);  // h_{j+1,j} = 0
    if (brk) hn = 0.0;
    ++steps;
    // V_{j+1} = W / h_{j+1,j} (Algorithm 2 step 3(e)); unused if the cycle
    // ends here
    if (!brk) {
      const double ih = 1.0 / hn;
      for (int e = t; e < N; e += kYT) W[e] *= ih;
    }
    if (t == 0) {
      // the earlier rotations on column j, the rotated entries to Rg
      double carry = h1[0] + h2[0];
#pragma unroll 4
      for (int i = 0; i < j; ++i) {
        const double y = h1[i + 1] + h2[i + 1];
        const double c = cs[i], sv = sn[i];
        a.Rg[i + (int64_t)m * j] = c * carry + sv * y;
        carry = -sv * carry + c * y;
      }
      const double aa = carry;
      const double r = hypot(aa, hn);
      double c = 1.0, sv = 0.0;
      if (r != 0.0) {
        c = aa / r;
        sv = hn / r;
      }
      cs[j] = c;
      sn[j] = sv;
      a.Rg[j + (int64_t)m * j] = r;
      const double gj = g[j];
      g[j] = c * gj;
      g[j + 1] = -sv * gj;
      double e = fabs(g[j + 1]);
      if (a.fom) e = aa != 0.0 ? hn * fabs(gj / aa) : __builtin_inf();
      sc[3] = e;
      sc[4] = gj;  // last right-hand side entry of the square system
      sc[5] = aa;  // its last diagonal entry
      if (steps - 1 < a.hist_cap) a.hist[steps - 1] = e / cnorm;
    }
    __syncthreads();
    est = sc[3];
    any_est = true;
    return brk || est <= stop || j + 1 >= m;
  };

  if (cnorm == 0.0) {
    for (int e = t; e < N; e += kYT) X[e] = 0.0;
    status = TSYLV_OK;
  } else {
    for (;;) {
      // R = C - M(X) into slot 0 (Algorithm 3 step 3; C itself for X0 = 0)
      double* R = lslot(0);
      if (cycles == 0 && !a.x0_given) {
        for (int e = t; e < N; e += kYT) R[e] = a.Zc[e];
      } else {
        tiny_apply(n, s, p, A, B, X, R);
        __syncthreads();
        for (int e = t; e < N; e += kYT) R[e] = a.Zc[e] - R[e];
      }
      __syncthreads();
      tiny_dots([&](int) { return R; }, 1, R, N, sc + 1);
      __syncthreads();
      const double beta = sqrt(sc[1]);
      rt = beta / cnorm;
      if (rt <= a.tol) {
        status = TSYLV_OK;
        break;
      }
      if (cycles >= a.max_cycles) break;
      ++cycles;
      const double ib = 1.0 / beta;
      for (int e = t; e < N; e += kYT) R[e] *= ib;
      if (t == 0) g[0] = beta;
      __syncthreads();

      int k = 0;
      for (int j = 0; j < m; ++j) {
        k = j + 1;
        if (j + 2 <= a.lslots ? step(lslot, j) : step(slot, j)) break;
      }

      // y (Algorithm 3 step 4(b)): tFOM's square system, or (tGMRES, and
      // tFOM's fallback) the least-squares problem
      double* y = h2;
      if (t < 64) {
        bool ok = false;
        const double dg = a.Rg[(k - 1) + (int64_t)m * (k - 1)];
        if (k <= 64) {
          if (a.fom) ok = tiny_back_wave(a.Rg, m, k, g, sc[5], sc[4], true, y);
          if (a.fom && !ok && t == 0) sc[7] += 1.0;  // falls back to the tGMRES solution
          if (!ok) ok = tiny_back_wave(a.Rg, m, k, g, dg, g[k - 1], false, y);
        } else if (t == 0) {
          if (a.fom) ok = tiny_back_serial(a.Rg, m, k, g, sc[5], sc[4], true, y);
          if (a.fom && !ok) sc[7] += 1.0;
          if (!ok) ok = tiny_back_serial(a.Rg, m, k, g, dg, g[k - 1], false, y);
        }
        if (t == 0) sc[6] = ok ? 0.0 : 1.0;
      }
      __syncthreads();
      if (sc[6] != 0.0) {
        status = TSYLV_ESINGULAR;
        break;
      }
      // X += V_k y (step 4(c))
      if (k <= a.lslots) {
        for (int e = t; e < N; e += kYT) {
          double acc = X[e];
          for (int i = 0; i < k; ++i) acc = fma(y[i], lslot(i)[e], acc);
          X[e] = acc;
        }
      } else {
        for (int e = t; e < N; e += kYT) {
          double acc = X[e];
          for (int i = 0; i < k; ++i) acc = fma(y[i], slot(i)[e], acc);
          X[e] = acc;
        }
      }
      __syncthreads();
    }
  }

  for (int e = t; e < N; e += kYT) a.Zx[e] = X[e];
  if (t == 0) {
    a.out[0] = status;
    a.out[1] = steps;
    a.out[2] = cycles;
    a.out[3] = rt;
    a.out[4] = any_est ? est / cnorm : 0.0;
    a.out[5] = sc[7];
    a.out[6] = steps < a.hist_cap ? steps : a.hist_cap;
  }
}

__global__ __launch_bounds__(kYT) void tiny_krylov_kernel(TinyArgs a) { tiny_solve(a); }

// One workgroup per job of a batch.
__global__ __launch_bounds__(kYT) void tiny_krylov_batch_kernel(const TinyArgs* __restrict__ jobs) {
  const TinyArgs a = jobs[blockIdx.x];
  tiny_solve(a);
}

}  // namespace

bool tiny_krylov_fits(int64_t n, int64_t s, int64_t p, int m) {
  const int64_t N = n * s * p;
  if (n < 1 || s < 1 || p < 1 || m < 1 || N > kYMaxN || m > kYMaxM || m * N > kYMaxMN)
    return false;
  return (fixed_doubles(n, s, p, m) + 2 * N) * (int64_t)sizeof(double) <= kYLds;
}

size_t tiny_krylov_lds(int64_t n, int64_t s, int64_t p, int m) {
  const int64_t need = (fixed_doubles(n, s, p, m) + (int64_t)(m + 1) * n * s * p) * 8;
  return (size_t)std::min<int64_t>(need, kYLds);
}

int tiny_krylov_slots(int64_t n, int64_t s, int64_t p, int m, size_t lds) {
  const int64_t N = n * s * p;
  const int64_t fit = ((int64_t)lds / (int64_t)sizeof(double) - fixed_doubles(n, s, p, m)) / N;
  return (int)std::min<int64_t>(m + 1, fit);
}

void tiny_krylov_batch(const TinyJob* jobs, int count, size_t lds, hipStream_t st) {
  if (count <= 0) return;
  if (lds > (size_t)kYLds) throw Error(TSYLV_EINVAL, "tiny Krylov batch: LDS too large");
  TSYLV_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tiny_krylov_batch_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(tiny_krylov_batch_kernel, dim3(count), dim3(kYT), lds, st, jobs);
  TSYLV_LAUNCH_CHECK();
}

void tiny_krylov(const double* Ah, const double* Bh, const double* Zc, double* Zx, double* basis,
                 double* Rg, double* hist, int hist_cap, double* out, int n, int s, int p, int m,
                 int max_cycles, bool fom, bool x0_given, double tol, hipStream_t st) {
  if (!tiny_krylov_fits(n, s, p, m)) throw Error(TSYLV_EINVAL, "tiny Krylov: sizes too large");
  const int64_t N = (int64_t)n * s * p;
  const int64_t fixed = fixed_doubles(n, s, p, m);
  const int64_t fit = (kYLds / (int64_t)sizeof(double) - fixed) / N;
  const int lslots = (int)std::min<int64_t>(m + 1, fit);
  const size_t lds = (size_t)(fixed + lslots * N) * sizeof(double);
  TinyArgs a;
  a.Ah = Ah;
  a.Bh = Bh;
  a.Zc = Zc;
  a.Zx = Zx;
  a.Vg = basis;
  a.Rg = Rg;
  a.hist = hist;
  a.out = out;
  a.tol = tol;
  a.n = n;
  a.s = s;
  a.p = p;
  a.m = m;
  a.max_cycles = max_cycles;
  a.fom = fom ? 1 : 0;
  a.x0_given = x0_given ? 1 : 0;
  a.hist_cap = hist ? hist_cap : 0;
  a.lslots = lslots;
  TSYLV_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tiny_krylov_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(tiny_krylov_kernel, dim3(1), dim3(kYT), lds, st, a);
  TSYLV_LAUNCH_CHECK();
}

}  // namespace kern
}  // namespace tsylv
