// Device solve of the TBAS(m) projected equations (eq. (TBslowrank)),
//   Hm_k Y_k - Y_k Bhat_k = [H0_k; 0]        for every Fourier slice k,
// after diagonalising Bhat_k = W_k diag(lam_k) W_k^{-1} on the host: with
// Z = Y W the columns decouple into the shifted systems
//   (Hm_k - lam_{k,j} I) z_{k,j} = d_{k,j},   d = [H0_k W_k; 0] e_j,
// one per (slice, eigenvalue) -- p_h s independent solves instead of s
// dependent ones per slice (Bartels-Stewart's triangular recursion).
//
// Hm_k (ms x ms, ms = m s) is block upper Hessenberg with s x s blocks
// (lower bandwidth s).  Each system is solved by block LU with s x s blocks:
// panel b is the 2s x s block column [row block b as updated so far; row
// block b + 1 as built], factorised with partial pivoting inside the panel
// (band-limited pivoting, as in banded LU), applied on the fly to the
// right-hand side and, through explicit L11^{-1} and L21, to the trailing
// columns of the two block rows.  The finished row blocks of U are kept for
// the back substitution.  One workgroup per system; the panel lives in LDS.
#include "kernels.hpp"

namespace tsylv {
namespace kern {

namespace {

constexpr int kPB = 256;     // threads per workgroup
constexpr int kPMax = 64;    // largest block size s handled here
constexpr int kTC = 8;       // trailing columns per tile

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
// a / b by Smith's scaling (no overflow for |b| near the range limits)
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const double r = b.x / b.y, d = b.y + b.x * r;
  return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__device__ __forceinline__ double cnorm2(double2 a) { return a.x * a.x + a.y * a.y; }

struct ProjArgs {
  const double2* Hm;  // p_h slices of ms x ms, column-major
  const double2* lam; // nsys shifts, system k s + j
  const double2* D;   // p_h slices of s x s: first s rows of the right-hand sides
  double2* z;         // nsys x ms: right-hand side, then solution
  double2* Wrk;       // nsys x (s x ms): the current row block
  double2* U;         // nsys x ustride: finished row blocks of U
  int* info;          // nsys flags (1: zero pivot)
  int ms, s, m, nsys;
  int64_t ustride;
};

__device__ __forceinline__ int64_t uoff(const ProjArgs& a, int b) {
  return (int64_t)a.s * a.s * ((int64_t)b * a.m - (int64_t)b * (b - 1) / 2);
}

__global__ void proj_init_kernel(ProjArgs a) {
  const int64_t nw = (int64_t)a.nsys * a.s * a.ms;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nw;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sys = e / ((int64_t)a.s * a.ms);
    const int64_t rem = e % ((int64_t)a.s * a.ms);
    const int r = (int)(rem % a.s), c = (int)(rem / a.s);
    const int k = (int)(sys / a.s);
    double2 v = a.Hm[(int64_t)k * a.ms * a.ms + r + (int64_t)a.ms * c];
    if (r == c) v = csub(v, a.lam[sys]);
    a.Wrk[e] = v;
  }
  const int64_t nz = (int64_t)a.nsys * a.ms;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sys = e / a.ms;
    const int i = (int)(e % a.ms);
    const int k = (int)(sys / a.s), j = (int)(sys % a.s);
    a.z[e] = i < a.s ? a.D[(int64_t)k * a.s * a.s + i + (int64_t)a.s * j] : make_double2(0.0, 0.0);
    if (i == 0) a.info[sys] = 0;
  }
}

// Panel b of every system.  Dynamic LDS: P (2 kPMax x kPMax), tile
// (2 kPMax x kTC), r2 (2 kPMax), tmp (kPMax), perm/piv.
__global__ __launch_bounds__(kPB) void proj_panel_kernel(ProjArgs a, int b) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  constexpr int LD = 2 * kPMax;
  double2* P = reinterpret_cast<double2*>(smem);
  double2* tile = P + LD * kPMax;
  double2* r2 = tile + LD * kTC;
  double2* tmp = r2 + LD;
  int* piv = reinterpret_cast<int*>(tmp + kPMax);
  int* perm = piv + kPMax;
  int* sflag = perm + LD;
  double* wbest = reinterpret_cast<double*>(sflag + 4);

  const int sys = blockIdx.x, tid = threadIdx.x;
  const int s = a.s, ms = a.ms, m = a.m;
  const int k = sys / s;
  const double2 lamv = a.lam[sys];
  const bool has_bot = b + 1 < m;
  const int nr = has_bot ? 2 * s : s;
  const int col0 = b * s;
  const double2* Hk = a.Hm + (int64_t)k * ms * ms;
  double2* W = a.Wrk + (int64_t)sys * s * ms;
  double2* zs = a.z + (int64_t)sys * ms;
  // row r of the panel: r < s current row block b, else original row (b+1)s + r - s
  for (int e = tid; e < nr * s; e += kPB) {
    const int r = e % nr, c = e / nr;
    P[r + LD * c] = r < s ? W[r + (int64_t)s * (col0 + c)]
                          : Hk[(int64_t)(col0 + s + r - s) + (int64_t)ms * (col0 + c)];
  }
  for (int i = tid; i < nr; i += kPB) r2[i] = zs[col0 + i];  // rows b s .. b s + nr - 1
  if (tid == 0) sflag[0] = 0;
  __syncthreads();

  for (int c = 0; c < s; ++c) {
    if (tid < 64) {  // pivot: largest |P(r, c)| over r >= c, smallest index on ties
      double best = -1.0;
      int bi = c;
      for (int r = c + tid; r < nr; r += 64) {
        const double v = cnorm2(P[r + LD * c]);
        if (v > best) {
          best = v;
          bi = r;
        }
      }
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (tid == 0) {
        piv[c] = bi;
        wbest[0] = best;
        if (!(best > 0.0) || !isfinite(best)) sflag[0] = 1;
      }
    }
    __syncthreads();
    const int pr = piv[c];
    if (pr != c) {
      for (int cc = tid; cc <= s; cc += kPB) {
        if (cc < s) {
          const double2 t = P[c + LD * cc];
          P[c + LD * cc] = P[pr + LD * cc];
          P[pr + LD * cc] = t;
        } else {
          const double2 t = r2[c];
          r2[c] = r2[pr];
          r2[pr] = t;
        }
      }
    }
    __syncthreads();
    const double2 d = sflag[0] ? make_double2(1.0, 0.0) : P[c + LD * c];
    for (int r = c + 1 + tid; r < nr; r += kPB) P[r + LD * c] = cdiv(P[r + LD * c], d);
    __syncthreads();
    // rank-1 update of the rows below c, columns c+1 .. s-1 and the right-hand side
    const int rows = nr - c - 1, cols = s - c;  // column index s - c - 1 + ... ; last = rhs
    for (int e = tid; e < rows * cols; e += kPB) {
      const int r = c + 1 + e % rows, q = e / rows;  // q in [0, cols): column c+1+q or rhs
      const double2 l = P[r + LD * c];
      if (q < cols - 1) {
        const int cc = c + 1 + q;
        P[r + LD * cc] = csub(P[r + LD * cc], cmul(l, P[c + LD * cc]));
      } else {
        r2[r] = csub(r2[r], cmul(l, r2[c]));
      }
    }
    __syncthreads();
  }
  if (tid == 0 && sflag[0]) a.info[sys] = 1;

  // finished U block (s x s, zero below the diagonal) and the eliminated rhs
  double2* Ub = a.U + (int64_t)sys * a.ustride + uoff(a, b);
  for (int e = tid; e < s * s; e += kPB) {
    const int r = e % s, c = e / s;
    Ub[r + (int64_t)s * c] = r <= c ? P[r + LD * c] : make_double2(0.0, 0.0);
  }
  for (int i = tid; i < nr; i += kPB) zs[col0 + i] = r2[i];
  if (!has_bot) return;

  // L11 (unit lower, top s rows) inverted in place, column by column from the
  // right: X(i, j) = -(L(i, j) + sum_{j<l<i} X(i, l) L(l, j)).
  for (int j = s - 2; j >= 0; --j) {
    for (int i = j + 1 + tid; i < s; i += kPB) tmp[i] = P[i + LD * j];
    __syncthreads();
    for (int i = j + 1 + tid; i < s; i += kPB) {
      double2 t = tmp[i];
      for (int l = j + 1; l < i; ++l) t = cadd(t, cmul(P[i + LD * l], tmp[l]));
      P[i + LD * j] = make_double2(-t.x, -t.y);
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int r = 0; r < nr; ++r) perm[r] = r;
    for (int c = 0; c < s; ++c) {
      const int t = perm[c];
      perm[c] = perm[piv[c]];
      perm[piv[c]] = t;
    }
  }
  __syncthreads();

  // trailing columns (b+1) s .. ms-1 of the two block rows, kTC at a time
  for (int col = col0 + s; col < ms; col += kTC) {
    for (int e = tid; e < nr * kTC; e += kPB) {
      const int r = e % nr, cc = e / nr, gc = col + cc;
      double2 v = make_double2(0.0, 0.0);
      if (gc < ms) {
        const int orow = perm[r];
        if (orow < s) {
          v = W[orow + (int64_t)s * gc];
        } else {
          const int grow = col0 + orow;  // (b+1) s + orow - s
          v = Hk[grow + (int64_t)ms * gc];
          if (grow == gc) v = csub(v, lamv);
        }
      }
      tile[r + LD * cc] = v;
    }
    __syncthreads();
    // Thread (rr, g): row rr, tile columns g, g + G, ... (at most CPT of
    // them), so each L entry read from LDS serves all of the thread's columns.
    constexpr int CPT = kTC / (kPB / kPMax);
    const int G = kPB / s, rr = tid % s, g = tid / s;
    const bool act = g < G;
    // U rows: L11^{-1} times the top half (X holds L11^{-1} below the diagonal)
    double2 acc[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int cc = g + G * q;
      acc[q] = (act && cc < kTC) ? tile[rr + LD * cc] : make_double2(0.0, 0.0);
    }
    if (act) {
#pragma unroll 4
      for (int l = 0; l < rr; ++l) {
        const double2 x = P[rr + LD * l];
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
          const int cc = g + G * q;
          if (cc < kTC) acc[q] = cadd(acc[q], cmul(x, tile[l + LD * cc]));
        }
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        const int cc = g + G * q, gc = col + cc;
        if (cc < kTC) {
          tile[rr + LD * cc] = acc[q];
          if (gc < ms) Ub[rr + (int64_t)s * (gc - col0)] = acc[q];
        }
      }
    }
    __syncthreads();
    // next row block: bottom half minus L21 times the U rows
    if (act) {
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        const int cc = g + G * q;
        acc[q] = cc < kTC ? tile[s + rr + LD * cc] : make_double2(0.0, 0.0);
      }
#pragma unroll 4
      for (int l = 0; l < s; ++l) {
        const double2 x = P[s + rr + LD * l];
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
          const int cc = g + G * q;
          if (cc < kTC) acc[q] = csub(acc[q], cmul(x, tile[l + LD * cc]));
        }
      }
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        const int cc = g + G * q, gc = col + cc;
        if (cc < kTC && gc < ms) W[rr + (int64_t)s * gc] = acc[q];
      }
    }
    __syncthreads();
  }
}

// Back substitution U z = y per system, row block by row block from the
// bottom; z is kept in LDS (ms complex values).
__global__ __launch_bounds__(kPB) void proj_back_kernel(ProjArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  double2* zl = reinterpret_cast<double2*>(smem);      // ms
  double2* part = zl + a.ms;                           // kPB
  double2* t = part + kPB;                             // kPMax
  const int sys = blockIdx.x, tid = threadIdx.x;
  const int s = a.s, ms = a.ms, m = a.m;
  double2* zs = a.z + (int64_t)sys * ms;
  for (int i = tid; i < ms; i += kPB) zl[i] = zs[i];
  __syncthreads();
  const int groups = kPB / s;  // threads per row of the mat-vec
  for (int b = m - 1; b >= 0; --b) {
    const double2* Ub = a.U + (int64_t)sys * a.ustride + uoff(a, b);
    const int c0 = (b + 1) * s;  // columns already solved
    if (tid < s * groups) {
      const int r = tid % s, g = tid / s;
      double2 acc = make_double2(0.0, 0.0);
      for (int c = c0 + g; c < ms; c += groups)
        acc = cadd(acc, cmul(Ub[r + (int64_t)s * (c - b * s)], zl[c]));
      part[tid] = acc;
    }
    __syncthreads();
    if (tid < s) {
      double2 acc = zl[b * s + tid];
      for (int g = 0; g < groups; ++g) acc = csub(acc, part[tid + s * g]);
      t[tid] = acc;
    }
    __syncthreads();
    // triangular solve with the s x s diagonal block, one wave: lane q holds
    // z(b s + q); row r's sum over the solved lanes q > r is a wave reduction
    if (tid < 64) {
      double2 zq = make_double2(0.0, 0.0);
      for (int r = s - 1; r >= 0; --r) {
        double2 acc = make_double2(0.0, 0.0);
        if (tid > r && tid < s) acc = cmul(Ub[r + (int64_t)s * tid], zq);
        for (int off = 32; off >= 1; off >>= 1) {
          acc.x += __shfl_xor(acc.x, off, 64);
          acc.y += __shfl_xor(acc.y, off, 64);
        }
        const double2 zr = cdiv(csub(t[r], acc), Ub[r + (int64_t)s * r]);
        if (tid == r) zq = zr;
      }
      if (tid < s) zl[b * s + tid] = zq;
    }
    __syncthreads();
  }
  for (int i = tid; i < ms; i += kPB) zs[i] = zl[i];
}

}  // namespace

int proj_max_block() { return kPMax; }

int64_t proj_u_stride(int s, int m) { return (int64_t)s * s * ((int64_t)m * (m + 1) / 2); }

void proj_solve(const double* Hm, const double* lam, const double* D, double* z, double* Wrk,
                double* U, int* info, int ms, int s, int m, int nsys, hipStream_t st) {
  if (s < 1 || s > kPMax || ms != m * s || nsys < 1)
    throw Error(TSYLV_EINVAL, "projected solve: unsupported sizes");
  ProjArgs a;
  a.Hm = reinterpret_cast<const double2*>(Hm);
  a.lam = reinterpret_cast<const double2*>(lam);
  a.D = reinterpret_cast<const double2*>(D);
  a.z = reinterpret_cast<double2*>(z);
  a.Wrk = reinterpret_cast<double2*>(Wrk);
  a.U = reinterpret_cast<double2*>(U);
  a.info = info;
  a.ms = ms;
  a.s = s;
  a.m = m;
  a.nsys = nsys;
  a.ustride = proj_u_stride(s, m);
  const int64_t work = (int64_t)nsys * s * ms;
  const int gi = (int)std::min<int64_t>((work + 255) / 256, 16384);
  hipLaunchKernelGGL(proj_init_kernel, dim3(gi), dim3(256), 0, st, a);
  TSYLV_LAUNCH_CHECK();
  constexpr int LD = 2 * kPMax;
  const size_t lds_panel = sizeof(double2) * ((size_t)LD * kPMax + (size_t)LD * kTC + LD + kPMax) +
                           sizeof(int) * (kPMax + LD + 4) + 16;
  TSYLV_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&proj_panel_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_panel));
  for (int b = 0; b < m; ++b) {
    hipLaunchKernelGGL(proj_panel_kernel, dim3(nsys), dim3(kPB), lds_panel, st, a, b);
    TSYLV_LAUNCH_CHECK();
  }
  const size_t lds_back = sizeof(double2) * ((size_t)ms + kPB + kPMax);
  if (lds_back > 160 * 1024) throw Error(TSYLV_EINVAL, "projected solve: ms too large");
  TSYLV_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&proj_back_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_back));
  hipLaunchKernelGGL(proj_back_kernel, dim3(nsys), dim3(kPB), lds_back, st, a);
  TSYLV_LAUNCH_CHECK();
}

}  // namespace kern
}  // namespace tsylv
