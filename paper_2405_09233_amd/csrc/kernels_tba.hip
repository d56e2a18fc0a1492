// Device-side small linear algebra of the TBAS(m) cycle (section 5), so that
// a cycle runs without host round trips:
//   * Tubal-QR (Algorithm 6, Normalization of section 5.1) by shifted
//     Cholesky QR: per Fourier slice, the Cholesky factor R of the (shifted)
//     Gram matrix W_k^H W_k, its inverse, and the product of the passes'
//     factors, one workgroup per slice with the s x s matrices in LDS; the
//     Normalization's tube test (a non-invertible tube) as a device flag;
//   * the block upper Hessenberg matrix of Algorithm 7 assembled in place
//     from the block Gram-Schmidt coefficients and the QR factors;
//   * the projected equation's right-hand side H0 W, the solution
//     Y = Z W^{-1} in the planar layout of the basis update, and the residual
//     estimate of the proposition of section 5.2, ||H_{m+1,m} E_m^T Y||.
// Planar matrices hold slice k's real and imaginary parts in the planes of
// the half-spectrum layout (slice_planes); real slices have no imaginary
// plane.  The projected solver's matrices are interleaved complex.
#include <algorithm>

#include "kernels.hpp"

namespace tsylv {
namespace kern {

namespace {

constexpr int kTB = 256;    // threads per workgroup
constexpr int kTMax = 64;   // largest block size s
// threads of a Cholesky-QR pass (one workgroup per slice: few workgroups,
// so each is given the most threads) and lanes per column of R^{-1}
constexpr int kQB = 1024;
constexpr int kQL = kQB / kTMax;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ double2 pget(const double* P, int qr, int qi, int64_t plane,
                                        int64_t off) {
  return make_double2(P[qr * plane + off], qi < 0 ? 0.0 : P[qi * plane + off]);
}
__device__ __forceinline__ void pput(double* P, int qr, int qi, int64_t plane, int64_t off,
                                     double2 v) {
  P[qr * plane + off] = v.x;
  if (qi >= 0) P[qi * plane + off] = v.y;
}

// One pass of shifted Cholesky QR for slice blockIdx.x: G (planar s x s
// Gram matrices, ld s) -> Rinv (planar, R^{-1}, zero below the diagonal) and
// Racc <- R Racc (Racc <- R on the first pass).  On the first pass the
// diagonal is shifted by shift_factor * trace(G).  A pivot that is not
// above rel_tol * max_i G(i, i) sets *flag (and leaves the outputs
// undefined).
__global__ __launch_bounds__(kQB) void cholqr_pass_kernel(const double* __restrict__ G,
                                                          double* __restrict__ Rinv,
                                                          double* __restrict__ Racc, int s, int p,
                                                          double shift_factor, int first,
                                                          double rel_tol, int* flag) {
  __shared__ double2 R[kTMax * kTMax];  // Gram, then its Cholesky factor (upper part)
  __shared__ double2 X[kTMax * kTMax];  // R^{-1}, then the previous Racc
  __shared__ double rs[kTMax];          // the factor's diagonal
  __shared__ double sh[1];
  const int k = blockIdx.x, t = threadIdx.x;
  int qr, qi;
  slice_planes(p, k, qr, qi);
  const int64_t ss = (int64_t)s * s;
  for (int e = t; e < s * s; e += kQB) R[e] = pget(G, qr, qi, ss, e);
  __syncthreads();
  if (t == 0) {
    double tr = 0.0, dmax = 0.0;
    for (int i = 0; i < s; ++i) tr += R[i + s * i].x;
    if (first)
      for (int i = 0; i < s; ++i) R[i + s * i].x += shift_factor * tr;
    for (int i = 0; i < s; ++i) dmax = fmax(dmax, R[i + s * i].x);
    sh[0] = dmax;
  }
  __syncthreads();
  const double dmax = sh[0];
  // Right-looking Cholesky G = R^H R (R upper), one barrier per column: the
  // pivot d_j = G(j, j) is read by every thread; the trailing entries lose
  // conj(G(j, i)) G(j, l) / d_j with row j as it stands (unscaled), and the
  // rows are scaled by 1 / sqrt(d_j) at the end (row j is not touched after
  // step j).
  bool bad = !(dmax > 0.0);
  for (int j = 0; j < s && !bad; ++j) {
    const double d = R[j + s * j].x;
    if (!(d > rel_tol * dmax)) {
      bad = true;
      break;
    }
    const double dinv = 1.0 / d;
    const int w = s - j - 1;
    for (int e = t; e < w * w; e += kQB) {
      const int i = j + 1 + e % w, l = j + 1 + e / w;
      if (i > l) continue;
      const double2 u = cconjmul(R[j + s * i], R[j + s * l]);
      R[i + s * l].x -= u.x * dinv;
      R[i + s * l].y -= u.y * dinv;
    }
    __syncthreads();
  }
  if (bad) {
    if (t == 0) atomicOr(flag, 1);
    return;
  }
  for (int i = t; i < s; i += kQB) rs[i] = sqrt(R[i + s * i].x);
  __syncthreads();
  for (int e = t; e < s * s; e += kQB) {
    const int i = e % s, l = e / s;
    if (i < l) {
      const double2 v = R[e];
      R[e] = make_double2(v.x / rs[i], v.y / rs[i]);
    } else if (i == l) {
      R[e] = make_double2(rs[i], 0.0);
    }
  }
  __syncthreads();
  // R^{-1} = X column by column, by back substitution: column j belongs to
  // the kQL adjacent lanes kQL j .. kQL j + kQL - 1 of one wave (lane g takes
  // the rows i = g mod kQL), so each column is finished inside its wave in
  // program order, with no barrier: for kk = j .. 0, x_kk = X(kk, j) /
  // R(kk, kk), then X(i, j) -= R(i, kk) x_kk for i < kk.
  {
    static_assert(64 % kQL == 0, "a column's lanes lie in one wave");
    const int j = t / kQL, g = t % kQL;
    if (j < s) {
      for (int i = g; i < s; i += kQL) X[i + s * j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
      for (int kk = j; kk >= 0; --kk) {
        const double2 xc = X[kk + s * j];
        const double2 xk = make_double2(xc.x / rs[kk], xc.y / rs[kk]);
        if (g == 0) X[kk + s * j] = xk;
        for (int i = g; i < kk; i += kQL) {
          const double2 u = cmul(R[i + s * kk], xk);
          X[i + s * j].x -= u.x;
          X[i + s * j].y -= u.y;
        }
      }
    }
  }
  __syncthreads();
  for (int e = t; e < s * s; e += kQB) {
    const int i = e % s, j = e / s;
    pput(Rinv, qr, qi, ss, e, i <= j ? X[e] : make_double2(0.0, 0.0));
  }
  __syncthreads();
  // Racc <- R Racc (both upper triangular), the previous Racc staged in X
  if (!first)
    for (int e = t; e < s * s; e += kQB) X[e] = pget(Racc, qr, qi, ss, e);
  __syncthreads();
  for (int e = t; e < s * s; e += kQB) {
    const int i = e % s, j = e / s;
    double2 acc = make_double2(0.0, 0.0);
    if (i <= j) {
      if (first) {
        acc = R[e];
      } else {
        for (int l = i; l <= j; ++l) {
          const double2 u = cmul(R[i + s * l], X[l + s * j]);
          acc.x += u.x;
          acc.y += u.y;
        }
      }
    }
    pput(Racc, qr, qi, ss, e, acc);
  }
}

// The Normalization's tube test on the diagonal of the accumulated R: tube
// jj, with Fourier coefficients R_k(jj, jj) (divided by c_k = sqrt(w_k / p)
// for blocks in the scaled planes), is not invertible when min_k <= 16 eps
// max_k; then *flag is set.
__global__ void tube_test_kernel(const double* __restrict__ Racc, int s, int p, int scaled,
                                 int* flag) {
  const int jj = blockIdx.x * blockDim.x + threadIdx.x;
  if (jj >= s) return;
  const int64_t ss = (int64_t)s * s;
  double amin = INFINITY, amax = 0.0;
  for (int k = 0; k < num_slices(p); ++k) {
    int qr, qi;
    slice_planes(p, k, qr, qi);
    double a = Racc[qr * ss + jj + (int64_t)s * jj];
    if (scaled) a /= sqrt((qi < 0 ? 1.0 : 2.0) / p);
    amin = fmin(amin, a);
    amax = fmax(amax, a);
  }
  if (!(amin > 16.0 * 2.220446049250313e-16 * amax)) atomicOr(flag, 1);
}

// Block column j of Hm (interleaved, ms x ms per slice): rows 0 .. J-1 the
// two Gram passes G1 + G2 (planar J x s, ld J), rows J .. J+s-1 the QR
// factor Rq (planar s x s) when J < ms; for the last block column the
// factor goes to Hlast (interleaved s x s per slice) instead.
__global__ void hm_column_kernel(const double* __restrict__ G1, const double* __restrict__ G2,
                                 const double* __restrict__ Rq, double2* __restrict__ Hm,
                                 double2* __restrict__ Hlast, int j, int s, int m, int p) {
  const int k = blockIdx.y;
  int qr, qi;
  slice_planes(p, k, qr, qi);
  const int ms = m * s, J = (j + 1) * s;
  const int64_t gplane = (int64_t)J * s, ss = (int64_t)s * s;
  double2* H = Hm + (int64_t)k * ms * ms;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < (J + s) * s;
       e += gridDim.x * blockDim.x) {
    const int r = e % (J + s), c = e / (J + s);
    if (r < J) {
      const double2 a = pget(G1, qr, qi, gplane, r + (int64_t)J * c);
      const double2 b = pget(G2, qr, qi, gplane, r + (int64_t)J * c);
      H[r + (int64_t)ms * (j * s + c)] = make_double2(a.x + b.x, a.y + b.y);
    } else {
      const double2 v = pget(Rq, qr, qi, ss, (r - J) + (int64_t)s * c);
      if (J < ms)
        H[r + (int64_t)ms * (j * s + c)] = v;
      else
        Hlast[(int64_t)k * ss + (r - J) + (int64_t)s * c] = v;
    }
  }
}

// D_k = H0_k W_k (s x s per slice): H0 planar, W and D interleaved.
__global__ void proj_rhs_kernel(const double* __restrict__ H0, const double2* __restrict__ W,
                                double2* __restrict__ D, int s, int p) {
  const int k = blockIdx.x;
  int qr, qi;
  slice_planes(p, k, qr, qi);
  const int64_t ss = (int64_t)s * s;
  for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
    const int i = e % s, j = e / s;
    double2 acc = make_double2(0.0, 0.0);
    for (int l = 0; l < s; ++l) {
      const double2 u = cmul(pget(H0, qr, qi, ss, i + (int64_t)s * l), W[k * ss + l + s * j]);
      acc.x += u.x;
      acc.y += u.y;
    }
    D[k * ss + e] = acc;
  }
}

// Y_k = Z_k W_k^{-1} for the rows of one 64-row chunk of one slice (grid:
// slices x chunks), W_k^{-1} staged in LDS; thread t takes row t % 64 of
// the chunk and the columns t / 64 + 4 q.
constexpr int kYRows = 64;
__global__ __launch_bounds__(256) void proj_y_kernel(const double2* __restrict__ z,
                                                     const double2* __restrict__ Winv,
                                                     double* __restrict__ Y, int s, int m, int p) {
  __shared__ double2 Wl[kTMax * kTMax];
  const int k = blockIdx.y, t = threadIdx.x;
  int qr, qi;
  slice_planes(p, k, qr, qi);
  const int ms = m * s;
  const int64_t ss = (int64_t)s * s, yplane = (int64_t)ms * s;
  for (int e = t; e < s * s; e += 256) Wl[e] = Winv[k * ss + e];
  __syncthreads();
  const int r = blockIdx.x * kYRows + (t % kYRows);
  if (r >= ms) return;
  const double2* Z = z + (int64_t)k * s * ms;
  constexpr int kCols = kTMax / 4;
  double2 acc[kCols];
#pragma unroll
  for (int q = 0; q < kCols; ++q) acc[q] = make_double2(0.0, 0.0);
  const int c0 = t / kYRows;
  for (int l = 0; l < s; ++l) {
    const double2 zv = Z[(int64_t)l * ms + r];
#pragma unroll
    for (int q = 0; q < kCols; ++q) {
      const int c = c0 + 4 * q;
      if (c < s) {
        const double2 u = cmul(zv, Wl[l + s * c]);
        acc[q].x += u.x;
        acc[q].y += u.y;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kCols; ++q) {
    const int c = c0 + 4 * q;
    if (c < s) pput(Y, qr, qi, yplane, r + (int64_t)ms * c, acc[q]);
  }
}

// The estimate of the proposition of section 5.2 for slice blockIdx.x:
// est[k] = ||Hlast_k Y_k(last s rows, :)||_F^2 (real slices: the real part).
__global__ __launch_bounds__(kTB) void proj_est_kernel(const double* __restrict__ Y,
                                                       const double2* __restrict__ Hlast,
                                                       double* __restrict__ est, int s, int m,
                                                       int p) {
  __shared__ double2 Hl[kTMax * kTMax];
  __shared__ double2 Yl[kTMax * kTMax];
  __shared__ double red[kTB];
  const int k = blockIdx.x, t = threadIdx.x;
  int qr, qi;
  slice_planes(p, k, qr, qi);
  const int ms = m * s;
  const int64_t ss = (int64_t)s * s, yplane = (int64_t)ms * s;
  for (int e = t; e < s * s; e += kTB) {
    const int r = e % s, c = e / s;
    Hl[e] = Hlast[k * ss + e];
    Yl[e] = pget(Y, qr, qi, yplane, (ms - s + r) + (int64_t)ms * c);
  }
  __syncthreads();
  double part = 0.0;
  for (int e = t; e < s * s; e += kTB) {
    const int r = e % s, c = e / s;
    double2 v = make_double2(0.0, 0.0);
    for (int l = 0; l < s; ++l) {
      const double2 u = cmul(Hl[r + s * l], Yl[l + s * c]);
      v.x += u.x;
      v.y += u.y;
    }
    part += qi < 0 ? v.x * v.x : v.x * v.x + v.y * v.y;
  }
  red[t] = part;
  __syncthreads();
  for (int w = kTB / 2; w > 0; w /= 2) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) est[k] = red[0];
}

// flag[1] <- 1 when a projected system had a zero pivot or a non-finite
// solution.
__global__ void proj_check_kernel(const int* __restrict__ info, const double2* __restrict__ z,
                                  int64_t nsys, int64_t nz, int* flag) {
  int bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nz;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nsys && info[e] != 0) bad = 1;
    if (!isfinite(z[e].x) || !isfinite(z[e].y)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

}  // namespace

int cholqr_max_block() { return kTMax; }

void cholqr_pass(const double* G, double* Rinv, double* Racc, int s, int p, double shift_factor,
                 bool first, double rel_tol, int* flag, hipStream_t st) {
  if (s < 1 || s > kTMax) throw Error(TSYLV_EINVAL, "cholqr_pass: block too large");
  hipLaunchKernelGGL(cholqr_pass_kernel, dim3(num_slices(p)), dim3(kQB), 0, st, G, Rinv, Racc,
                     s, p, shift_factor, first ? 1 : 0, rel_tol, flag);
  TSYLV_LAUNCH_CHECK();
}

void tube_test(const double* Racc, int s, int p, bool scaled, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(tube_test_kernel, dim3((s + 63) / 64), dim3(64), 0, st, Racc, s, p,
                     scaled ? 1 : 0, flag);
  TSYLV_LAUNCH_CHECK();
}

void hm_column(const double* G1, const double* G2, const double* Rq, double* Hm, double* Hlast,
               int j, int s, int m, int p, hipStream_t st) {
  const int elems = ((j + 2) * s) * s;
  const int bx = std::min(64, (elems + 255) / 256);
  hipLaunchKernelGGL(hm_column_kernel, dim3(bx, num_slices(p)), dim3(256), 0, st, G1, G2, Rq,
                     reinterpret_cast<double2*>(Hm), reinterpret_cast<double2*>(Hlast), j, s, m,
                     p);
  TSYLV_LAUNCH_CHECK();
}

void proj_rhs(const double* H0, const double* W, double* D, int s, int p, hipStream_t st) {
  hipLaunchKernelGGL(proj_rhs_kernel, dim3(num_slices(p)), dim3(256), 0, st, H0,
                     reinterpret_cast<const double2*>(W), reinterpret_cast<double2*>(D), s, p);
  TSYLV_LAUNCH_CHECK();
}

void proj_y(const double* z, const double* Winv, const double* Hlast, double* Y, double* est,
            int s, int m, int p, hipStream_t st) {
  if (s < 1 || s > kTMax) throw Error(TSYLV_EINVAL, "proj_y: block too large");
  const int chunks = (m * s + kYRows - 1) / kYRows;
  hipLaunchKernelGGL(proj_y_kernel, dim3(chunks, num_slices(p)), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(z), reinterpret_cast<const double2*>(Winv),
                     Y, s, m, p);
  TSYLV_LAUNCH_CHECK();
  hipLaunchKernelGGL(proj_est_kernel, dim3(num_slices(p)), dim3(kTB), 0, st, Y,
                     reinterpret_cast<const double2*>(Hlast), est, s, m, p);
  TSYLV_LAUNCH_CHECK();
}

void proj_check(const int* info, const double* z, int64_t nsys, int64_t nz, int* flag,
                hipStream_t st) {
  const int blocks = (int)std::min<int64_t>((nz + 255) / 256, 1024);
  hipLaunchKernelGGL(proj_check_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, st, info,
                     reinterpret_cast<const double2*>(z), nsys, nz, flag);
  TSYLV_LAUNCH_CHECK();
}

}  // namespace kern
}  // namespace tsylv
