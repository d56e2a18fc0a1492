// t-Bartels-Stewart direct solve for small sizes (section 4: the t-Schur
// decomposition of Algorithm 4 and the t-Bartels-Stewart method of
// Algorithm 5), done slice by slice in the Fourier domain:
//   Ahat_k = U_k T_k U_k^H,  Bhat_k = V_k S_k V_k^H   (complex Schur forms),
//   T_k Y - Y S_k = U_k^H Chat_k V_k                (triangular equation),
//   Xhat_k = U_k Y V_k^H.
// With the T-product's sign A*X - X*B the column recursion is
//   (T_k - S_k[j,j] I) y_j = f_j + sum_{l<j} y_l S_k[l,j],
// each a back substitution (the t-back-substitution of the paper, which on
// the Fourier side is the matrix one on every slice).  The complex Schur
// form replaces the real (quasi-triangular) one: the slices are complex, and
// the conjugate slices the half spectrum leaves out are the conjugates.
//
// One workgroup of a single wavefront per Fourier slice, n, s <= 64: the
// matrix being reduced and its Schur vectors sit in LDS (lane i owns row or
// column i), so every rotation of the QR iteration costs two LDS sweeps and
// no barrier beyond the wave's own.  Schur reduction: Householder to
// Hessenberg form, then implicit single-shift QR sweeps (Wilkinson shift,
// exceptional shift every 10 iterations without deflation) with deflation on
// negligible subdiagonal entries, the full triangle and the Schur vectors
// updated by every rotation.
#include <cfloat>

#include "kernels.hpp"

namespace tsylv {
namespace kern {

namespace {

constexpr int kTbsMax = 64;       // largest n and s
constexpr int kTbsLd = kTbsMax + 1;  // LDS leading dimension (row sweeps hit distinct banks)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cscale(double2 a, double r) { return make_double2(a.x * r, a.y * r); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double cabs2(double2 a) { return hypot(a.x, a.y); }
// a / b by Smith's scaling
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const double r = b.x / b.y, d = b.y + b.x * r;
  return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
// principal square root
__device__ __forceinline__ double2 csqrt(double2 z) {
  const double r = cabs2(z);
  if (r == 0.0) return make_double2(0.0, 0.0);
  const double re = sqrt(0.5 * (r + fabs(z.x)));
  const double t = z.y / (2.0 * re);
  return z.x >= 0.0 ? make_double2(re, t) : make_double2(fabs(t), copysign(re, z.y));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Complex Schur form of the n x n matrix in W (LDS, column-major, leading
// dimension kTbsLd): on return W holds the upper triangular T and U the
// unitary factor with W_in = U T U^H.  One wavefront; returns false if the QR
// iteration did not converge within 30 n sweeps.
__device__ bool schur_wave(double2* W, double2* U, double2* v, int n) {
  const int lane = threadIdx.x;
  auto at = [&](double2* M, int i, int j) -> double2& { return M[i + kTbsLd * j]; };
  for (int j = 0; j < n; ++j)
    if (lane < n) at(U, lane, j) = make_double2(lane == j ? 1.0 : 0.0, 0.0);
  __syncthreads();

  // Householder reduction to upper Hessenberg form.
  for (int k = 0; k + 2 < n; ++k) {
    const double2 xi = (lane > k && lane < n) ? at(W, lane, k) : make_double2(0.0, 0.0);
    const double xn2 = wave_sum(xi.x * xi.x + xi.y * xi.y);
    const double2 x0 = at(W, k + 1, k);
    const double a0 = cabs2(x0);
    const double xn = sqrt(xn2);
    if (xn == 0.0) continue;
    const double2 ph = a0 > 0.0 ? cscale(x0, 1.0 / a0) : make_double2(1.0, 0.0);
    const double2 alpha = cscale(ph, -xn);  // x -> alpha e1
    const double2 v0 = csub(x0, alpha);
    const double vn2 = xn2 - a0 * a0 + (v0.x * v0.x + v0.y * v0.y);
    if (!(vn2 > 0.0)) continue;
    const double beta = 2.0 / vn2;
    if (lane < n) v[lane] = lane <= k ? make_double2(0.0, 0.0) : (lane == k + 1 ? v0 : xi);
    __syncthreads();
    // rows k+1.. of columns k..n-1:  A <- (I - beta v v^H) A
    if (lane >= k && lane < n) {
      double2 sdot = make_double2(0.0, 0.0);
      for (int i = k + 1; i < n; ++i) sdot = cadd(sdot, cmulc(v[i], at(W, i, lane)));
      sdot = cscale(sdot, beta);
      for (int i = k + 1; i < n; ++i) at(W, i, lane) = csub(at(W, i, lane), cmul(v[i], sdot));
    }
    __syncthreads();
    // columns k+1.. of every row:  A <- A (I - beta v v^H),  U <- U (...)
    if (lane < n) {
      double2 ta = make_double2(0.0, 0.0), tu = make_double2(0.0, 0.0);
      for (int j = k + 1; j < n; ++j) {
        ta = cadd(ta, cmul(at(W, lane, j), v[j]));
        tu = cadd(tu, cmul(at(U, lane, j), v[j]));
      }
      ta = cscale(ta, beta);
      tu = cscale(tu, beta);
      for (int j = k + 1; j < n; ++j) {
        at(W, lane, j) = csub(at(W, lane, j), cmul(ta, cconj(v[j])));
        at(U, lane, j) = csub(at(U, lane, j), cmul(tu, cconj(v[j])));
      }
    }
    __syncthreads();
    if (lane > k + 1 && lane < n) at(W, lane, k) = make_double2(0.0, 0.0);
    if (lane == 0) at(W, k + 1, k) = alpha;
    __syncthreads();
  }

  // Implicit single-shift QR on the active window [l, hi].
  int hi = n - 1, iter = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    while (l > 0) {
      const double2 h = at(W, l, l - 1);
      const double2 a = at(W, l - 1, l - 1), b = at(W, l, l);
      const double tst = fabs(a.x) + fabs(a.y) + fabs(b.x) + fabs(b.y);
      if (fabs(h.x) + fabs(h.y) <= DBL_EPSILON * tst) break;
      --l;
    }
    __syncthreads();
    if (l > 0 && lane == 0) at(W, l, l - 1) = make_double2(0.0, 0.0);
    __syncthreads();
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 30 * n) return false;
    ++iter;
    double2 mu;
    {
      const double2 a = at(W, hi - 1, hi - 1), b = at(W, hi - 1, hi), c = at(W, hi, hi - 1),
                    d = at(W, hi, hi);
      if (iter % 10 == 0) {
        mu = cadd(d, make_double2(0.75 * cabs2(c), 0.0));  // exceptional shift
      } else {
        const double2 half = cscale(csub(a, d), 0.5);
        const double2 disc = csqrt(cadd(cmul(half, half), cmul(b, c)));
        const double2 mid = cscale(cadd(a, d), 0.5);
        const double2 m1 = cadd(mid, disc), m2 = csub(mid, disc);
        mu = cabs2(csub(m1, d)) <= cabs2(csub(m2, d)) ? m1 : m2;
      }
    }
    double2 x = csub(at(W, l, l), mu), y = at(W, l + 1, l);
    for (int k = l; k < hi; ++k) {
      if (k > l) {
        x = at(W, k, k - 1);
        y = at(W, k + 1, k - 1);
      }
      // G = [[c, s], [-conj(s), c]] with G [x; y] = [r; 0]
      double c, rr;
      double2 s;
      const double ax = cabs2(x), ay = cabs2(y);
      if (ay == 0.0) {
        c = 1.0;
        s = make_double2(0.0, 0.0);
      } else if (ax == 0.0) {
        c = 0.0;
        s = cscale(cconj(y), 1.0 / ay);
      } else {
        rr = hypot(ax, ay);
        c = ax / rr;
        s = cscale(cmul(x, cconj(y)), 1.0 / (ax * rr));
      }
      __syncthreads();
      // rows k, k+1 (columns from the bulge on):  W <- G W
      const int c0 = k > l ? k - 1 : l;
      if (lane >= c0 && lane < n) {
        const double2 p = at(W, k, lane), q = at(W, k + 1, lane);
        at(W, k, lane) = cadd(cscale(p, c), cmul(s, q));
        at(W, k + 1, lane) = csub(cscale(q, c), cmulc(s, p));
      }
      __syncthreads();
      // columns k, k+1:  W <- W G^H (rows above the bulge), U <- U G^H
      const int r1 = min(k + 2, hi);
      if (lane < n) {
        if (lane <= r1) {
          const double2 p = at(W, lane, k), q = at(W, lane, k + 1);
          at(W, lane, k) = cadd(cscale(p, c), cmul(cconj(s), q));
          at(W, lane, k + 1) = csub(cscale(q, c), cmul(s, p));
        }
        const double2 p = at(U, lane, k), q = at(U, lane, k + 1);
        at(U, lane, k) = cadd(cscale(p, c), cmul(cconj(s), q));
        at(U, lane, k + 1) = csub(cscale(q, c), cmul(s, p));
      }
      __syncthreads();
      if (k > l && lane == 0) at(W, k + 1, k - 1) = make_double2(0.0, 0.0);
      __syncthreads();
    }
  }
  // clean the strictly lower triangle
  for (int j = 0; j < n; ++j)
    if (lane > j && lane < n) at(W, lane, j) = make_double2(0.0, 0.0);
  __syncthreads();
  return true;
}

// Slice k of one instance, by the one wavefront of the workgroup.
__device__ void tbs_slice(const TbsArgs& a, int k) {
  extern __shared__ __attribute__((aligned(16))) double2 tbs_lds[];
  double2* W = tbs_lds;
  double2* U = W + kTbsLd * kTbsMax;
  double2* v = U + kTbsLd * kTbsMax;
  const int lane = threadIdx.x;
  const int n = a.n, s = a.s;
  int qr, qi;
  slice_planes(a.p, k, qr, qi);
  const int64_t per = 2 * (int64_t)s * s + 2 * (int64_t)n * s;
  double2* S = a.scr + k * per;
  double2* V = S + (int64_t)s * s;
  double2* G = V + (int64_t)s * s;
  double2* F = G + (int64_t)n * s;
  auto plane_at = [&](const double* P, int64_t rows, int64_t cols, int i, int j) -> double2 {
    const int64_t off = i + rows * j;
    return make_double2(P[qr * rows * cols + off], qi >= 0 ? P[qi * rows * cols + off] : 0.0);
  };
  int status = 0;

  // Schur form of Bhat_k -> S, V (global scratch)
  for (int j = 0; j < s; ++j)
    if (lane < s) W[lane + kTbsLd * j] = plane_at(a.Bh, s, s, lane, j);
  __syncthreads();
  if (!schur_wave(W, U, v, s)) status = 1;
  for (int j = 0; j < s; ++j)
    if (lane < s) {
      S[lane + (int64_t)s * j] = W[lane + kTbsLd * j];
      V[lane + (int64_t)s * j] = U[lane + kTbsLd * j];
    }
  __syncthreads();

  // Schur form of Ahat_k, kept in LDS (W = T, U)
  for (int j = 0; j < n; ++j)
    if (lane < n) W[lane + kTbsLd * j] = plane_at(a.Ah, n, n, lane, j);
  __syncthreads();
  if (!schur_wave(W, U, v, n)) status = 1;

  // G = Chat_k V, then F = U^H G (lane = row)
  if (lane < n) {
    for (int j = 0; j < s; ++j) {
      double2 acc = make_double2(0.0, 0.0);
      for (int l = 0; l < s; ++l)
        acc = cadd(acc, cmul(plane_at(a.Zc, n, s, lane, l), V[l + (int64_t)s * j]));
      G[lane + (int64_t)n * j] = acc;
    }
  }
  __syncthreads();
  if (lane < n) {
    for (int j = 0; j < s; ++j) {
      double2 acc = make_double2(0.0, 0.0);
      for (int l = 0; l < n; ++l) acc = cadd(acc, cmulc(U[l + kTbsLd * lane], G[l + (int64_t)n * j]));
      F[lane + (int64_t)n * j] = acc;
    }
  }
  __syncthreads();

  // T Y - Y S = F column by column; Y overwrites G.
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale = fmax(scale, cabs2(W[i + kTbsLd * i]));
  for (int j = 0; j < s; ++j) scale = fmax(scale, cabs2(S[j + (int64_t)s * j]));
  const double tiny = 16.0 * DBL_EPSILON * fmax(scale, DBL_MIN);
  for (int j = 0; j < s; ++j) {
    const double2 sjj = S[j + (int64_t)s * j];
    double2 rhs = make_double2(0.0, 0.0);
    if (lane < n) {
      rhs = F[lane + (int64_t)n * j];
      for (int l = 0; l < j; ++l)
        rhs = cadd(rhs, cmul(G[lane + (int64_t)n * l], S[l + (int64_t)s * j]));
    }
    for (int i = n - 1; i >= 0; --i) {
      const double2 d = csub(W[i + kTbsLd * i], sjj);
      double2 yi = make_double2(0.0, 0.0);
      if (lane == i) {
        if (cabs2(d) <= tiny) status = 2;
        else yi = cdiv(rhs, d);
      }
      yi.x = __shfl(yi.x, i, 64);
      yi.y = __shfl(yi.y, i, 64);
      if (lane == i) G[i + (int64_t)n * j] = yi;
      if (lane < i) rhs = csub(rhs, cmul(W[lane + kTbsLd * i], yi));
    }
  }
  __syncthreads();

  // Z = U Y (into F), then Xhat = Z V^H (lane = row)
  if (lane < n) {
    for (int j = 0; j < s; ++j) {
      double2 acc = make_double2(0.0, 0.0);
      for (int l = 0; l < n; ++l) acc = cadd(acc, cmul(U[lane + kTbsLd * l], G[l + (int64_t)n * j]));
      F[lane + (int64_t)n * j] = acc;
    }
  }
  __syncthreads();
  if (lane < n) {
    const int64_t ns = (int64_t)n * s;
    for (int j = 0; j < s; ++j) {
      double2 acc = make_double2(0.0, 0.0);
      for (int l = 0; l < s; ++l)
        acc = cadd(acc, cmul(F[lane + (int64_t)n * l], cconj(V[j + (int64_t)s * l])));
      a.Zx[qr * ns + lane + (int64_t)n * j] = acc.x;
      if (qi >= 0) a.Zx[qi * ns + lane + (int64_t)n * j] = acc.y;
    }
  }
  // every lane saw the same Schur status; singular pivots were found by one lane
  int any = status;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) any = max(any, __shfl_xor(any, off, 64));
  if (lane == 0 && any) atomicMax(a.info, any);
}

__global__ __launch_bounds__(64) void tbs_slice_kernel(TbsArgs a) { tbs_slice(a, blockIdx.x); }

// Many instances in one launch: workgroup b serves slice b - first[i] of
// the instance i whose range [first[i], first[i + 1]) holds b.
__global__ __launch_bounds__(64) void tbs_batch_slice_kernel(const TbsArgs* __restrict__ args,
                                                             const int* __restrict__ first,
                                                             int count) {
  const int b = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {  // last instance with first[i] <= b
    const int mid = (lo + hi + 1) / 2;
    if (first[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  tbs_slice(args[lo], b - first[lo]);
}

// Residual of the direct solve in the Fourier planes, per (instance,
// slice): R_k = Chat_k - (Ahat_k Xhat_k - Xhat_k Bhat_k) on the scaled
// planes, so that sum_k ||R_k||^2 over the stored reals is ||C - M(X)||^2
// (Parseval); part[2 (first[i] + k)] receives slice k's ||R_k||^2 and
// part[2 (first[i] + k) + 1] its ||Chat_k||^2.  One wavefront per slice,
// lane = row.
__global__ __launch_bounds__(64) void tbs_batch_residual_kernel(const TbsArgs* __restrict__ args,
                                                                const int* __restrict__ first,
                                                                int count,
                                                                double* __restrict__ part) {
  const int b = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (first[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const TbsArgs& a = args[lo];
  const int k = b - first[lo], lane = threadIdx.x;
  const int n = a.n, s = a.s;
  int qr, qi;
  slice_planes(a.p, k, qr, qi);
  const int64_t ns = (int64_t)n * s, nn = (int64_t)n * n, ss = (int64_t)s * s;
  auto pl = [&](const double* P, int64_t plane, int64_t off) -> double2 {
    return make_double2(P[qr * plane + off], qi >= 0 ? P[qi * plane + off] : 0.0);
  };
  double rr = 0.0, cc = 0.0;
  if (lane < n) {
    for (int j = 0; j < s; ++j) {
      double2 acc = make_double2(0.0, 0.0);
      for (int l = 0; l < n; ++l)
        acc = cadd(acc, cmul(pl(a.Ah, nn, lane + (int64_t)n * l), pl(a.Zx, ns, l + (int64_t)n * j)));
      for (int l = 0; l < s; ++l)
        acc = csub(acc, cmul(pl(a.Zx, ns, lane + (int64_t)n * l), pl(a.Bh, ss, l + (int64_t)s * j)));
      const double2 c = pl(a.Zc, ns, lane + (int64_t)n * j);
      const double2 r = csub(c, acc);
      rr += r.x * r.x + (qi >= 0 ? r.y * r.y : 0.0);
      cc += c.x * c.x + (qi >= 0 ? c.y * c.y : 0.0);
    }
  }
  // fixed-order wave sums
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    rr += __shfl_xor(rr, off, 64);
    cc += __shfl_xor(cc, off, 64);
  }
  if (lane == 0) {
    part[2 * (int64_t)b] = rr;
    part[2 * (int64_t)b + 1] = cc;
  }
}

// out[2 i] = sum_k ||R_k||^2, out[2 i + 1] = sum_k ||Chat_k||^2 of instance
// i, in slice order.
__global__ void tbs_batch_norms_kernel(const double* __restrict__ part,
                                       const int* __restrict__ first, int count,
                                       double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double rr = 0.0, cc = 0.0;
  for (int b = first[i]; b < first[i + 1]; ++b) {
    rr += part[2 * (int64_t)b];
    cc += part[2 * (int64_t)b + 1];
  }
  out[2 * i] = rr;
  out[2 * i + 1] = cc;
}

// Tube transforms of many tensors in one launch: descriptor d maps the
// tubes of its tensor, out[q E + e] = sum_j M[q p + j] in[j E + e], with
// blocks [bfirst[d], bfirst[d + 1]) of kBatchXformBlock tubes each.
__global__ __launch_bounds__(kBatchXformBlock) void batch_xform_kernel(
    const XformDesc* __restrict__ descs, const int* __restrict__ bfirst, int ndesc) {
  const int b = blockIdx.x;
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (bfirst[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const XformDesc& d = descs[lo];
  const int64_t e = (int64_t)(b - bfirst[lo]) * kBatchXformBlock + threadIdx.x;
  if (e >= d.E) return;
  const int p = d.p;
  for (int q = 0; q < p; ++q) {
    double acc = 0.0;
    for (int j = 0; j < p; ++j) acc = fma(d.M[q * p + j], d.in[j * d.E + e], acc);
    d.out[q * d.E + e] = acc;
  }
}

}  // namespace

int tbs_max_size() { return kTbsMax; }

void tbs_batch(const TbsArgs* d_args, const int* d_first, int count, int total_slices,
               double* d_part, double* d_norms, hipStream_t st) {
  const size_t lds = (2 * (size_t)kTbsLd * kTbsMax + kTbsMax) * sizeof(double2);
  TSYLV_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tbs_batch_slice_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(tbs_batch_slice_kernel, dim3(total_slices), dim3(64), lds, st, d_args,
                     d_first, count);
  TSYLV_LAUNCH_CHECK();
  hipLaunchKernelGGL(tbs_batch_residual_kernel, dim3(total_slices), dim3(64), 0, st, d_args,
                     d_first, count, d_part);
  TSYLV_LAUNCH_CHECK();
  hipLaunchKernelGGL(tbs_batch_norms_kernel, dim3((count + 63) / 64), dim3(64), 0, st, d_part,
                     d_first, count, d_norms);
  TSYLV_LAUNCH_CHECK();
}

void batch_xform(const XformDesc* d_descs, const int* d_bfirst, int ndesc, int total_blocks,
                 hipStream_t st) {
  if (total_blocks <= 0) return;
  hipLaunchKernelGGL(batch_xform_kernel, dim3(total_blocks), dim3(kBatchXformBlock), 0, st,
                     d_descs, d_bfirst, ndesc);
  TSYLV_LAUNCH_CHECK();
}

int64_t tbs_scratch_complex(int64_t n, int64_t s, int p) {
  return (int64_t)num_slices(p) * (2 * s * s + 2 * n * s);
}

void tbs_solve(const double* Ah, const double* Bh, const double* Zc, double* Zx, int64_t n,
               int64_t s, int p, double* scratch, int* info, hipStream_t st) {
  if (n < 1 || s < 1 || n > kTbsMax || s > kTbsMax || p < 1)
    throw Error(TSYLV_EINVAL, "tbs: n and s must lie in [1, 64]");
  TbsArgs a{Ah, Bh, Zc, Zx, reinterpret_cast<double2*>(scratch), info, (int)n, (int)s, p};
  const size_t lds = (2 * (size_t)kTbsLd * kTbsMax + kTbsMax) * sizeof(double2);
  TSYLV_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tbs_slice_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(tbs_slice_kernel, dim3(num_slices(p)), dim3(64), lds, st, a);
  TSYLV_LAUNCH_CHECK();
}

}  // namespace kern
}  // namespace tsylv
