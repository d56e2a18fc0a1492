// Facewise Sylvester apply in the Fourier half spectrum (FP64, vector ALU).
//
// Algorithm 1 of section 2.1 computes a T-product as independent products
// of the Fourier slices; for M(X) = A*X - X*B (eq. (2)) that is
//     W_k = Ahat_k V_k - V_k Bhat_k,   k = 0 .. floor(p/2),
// with complex slices stored as (Re, Im) plane pairs and the real DC and
// Nyquist slices as single planes.  One workgroup computes a 64 x 64 tile
// of W_k: the n x n slice of A is streamed once through LDS in 64 x 16
// panels, the matching 16 x 64 panels of V_k come from L2, and each thread
// accumulates a 4 x 4 complex micro-tile.  The small V_k Bhat_k product
// (n x s times s x s) and the alpha/beta epilogue are fused at the end.
#include "kernels.hpp"

namespace tsylv {
namespace kern {

namespace {

constexpr int TM = 64, TN = 64, TK = 16;
constexpr int NT = 256;

template <bool CPLX>
__device__ __forceinline__ void apply_tile(
    const double* __restrict__ Ar, const double* __restrict__ Ai,
    const double* __restrict__ Vr, const double* __restrict__ Vi,
    const double* __restrict__ Br, const double* __restrict__ Bi,
    const double* __restrict__ Yr, const double* __restrict__ Yi,
    double* __restrict__ Or, double* __restrict__ Oi, double alpha, double beta,
    int64_t n, int64_t s, int64_t m0, int64_t c0,
    double (*As)[TK][TM], double (*Vs)[TK][TN + 1]) {
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  double accr[4][4], acci[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      accr[i][j] = 0.0;
      acci[i][j] = 0.0;
    }

  for (int64_t k0 = 0; k0 < n; k0 += TK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int idx = tid + NT * u;
      int row = idx & (TM - 1), kk = idx >> 6;
      int64_t gr = m0 + row, gk = k0 + kk;
      bool ok = (gr < n) && (gk < n);
      int64_t off = gr + n * gk;
      As[0][kk][row] = ok ? Ar[off] : 0.0;
      if (CPLX) As[1][kk][row] = ok ? Ai[off] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int idx = tid + NT * u;
      int kk = idx & (TK - 1), col = idx >> 4;
      int64_t gk = k0 + kk, gc = c0 + col;
      bool ok = (gk < n) && (gc < s);
      int64_t off = gk + n * gc;
      Vs[0][kk][col] = ok ? Vr[off] : 0.0;
      if (CPLX) Vs[1][kk][col] = ok ? Vi[off] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < TK; ++kk) {
      double ar[4], ai[4], vr[4], vi[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ar[i] = As[0][kk][tx + 16 * i];
        if (CPLX) ai[i] = As[1][kk][tx + 16 * i];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        vr[j] = Vs[0][kk][ty + 16 * j];
        if (CPLX) vi[j] = Vs[1][kk][ty + 16 * j];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          accr[i][j] = fma(ar[i], vr[j], accr[i][j]);
          if (CPLX) {
            accr[i][j] = fma(-ai[i], vi[j], accr[i][j]);
            acci[i][j] = fma(ar[i], vi[j], acci[i][j]);
            acci[i][j] = fma(ai[i], vr[j], acci[i][j]);
          }
        }
    }
    __syncthreads();
  }

  // Fused epilogue: subtract V_k Bhat_k, then alpha/beta.
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int64_t r = m0 + tx + 16 * i;
    if (r >= n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int64_t c = c0 + ty + 16 * j;
      if (c >= s) continue;
      double tr = accr[i][j], ti = CPLX ? acci[i][j] : 0.0;
      if (Br != nullptr) {
        for (int64_t l = 0; l < s; ++l) {
          double vr = Vr[r + n * l], br = Br[l + s * c];
          tr = fma(-vr, br, tr);
          if (CPLX) {
            double vi = Vi[r + n * l], bi = Bi[l + s * c];
            tr = fma(vi, bi, tr);
            ti = fma(-vr, bi, ti);
            ti = fma(-vi, br, ti);
          }
        }
      }
      int64_t off = r + n * c;
      double outr = alpha * tr, outi = alpha * ti;
      if (beta != 0.0) {
        outr = fma(beta, Yr[off], outr);
        if (CPLX) outi = fma(beta, Yi[off], outi);
      }
      Or[off] = outr;
      if (CPLX) Oi[off] = outi;
    }
  }
}

__global__ __launch_bounds__(NT) void apply_f64_kernel(
    const double* __restrict__ Ah, const double* __restrict__ Bh,
    const double* __restrict__ V, double* __restrict__ out, const double* __restrict__ Y,
    double alpha, double beta, int64_t n, int64_t s, int p) {
  __shared__ double As[2][TK][TM];
  __shared__ double Vs[2][TK][TN + 1];
  const int k = blockIdx.z;
  int qr, qi;
  slice_planes(p, k, qr, qi);
  const int64_t nn = n * n, ns = n * s, ss = s * s;
  const int64_t m0 = (int64_t)blockIdx.x * TM, c0 = (int64_t)blockIdx.y * TN;
  const double* Br = Bh ? Bh + qr * ss : nullptr;
  const double* Yr = Y ? Y + qr * ns : nullptr;
  if (qi < 0) {
    apply_tile<false>(Ah + qr * nn, nullptr, V + qr * ns, nullptr, Br, nullptr, Yr, nullptr,
                      out + qr * ns, nullptr, alpha, beta, n, s, m0, c0, As, Vs);
  } else {
    const double* Bi = Bh ? Bh + qi * ss : nullptr;
    const double* Yi = Y ? Y + qi * ns : nullptr;
    apply_tile<true>(Ah + qr * nn, Ah + qi * nn, V + qr * ns, V + qi * ns, Br, Bi, Yr, Yi,
                     out + qr * ns, out + qi * ns, alpha, beta, n, s, m0, c0, As, Vs);
  }
}

}  // namespace

void apply_f64(const double* Ah, const double* Bh, const double* V, double* out, const double* Y,
               double alpha, double beta, int64_t n, int64_t s, int p, hipStream_t st) {
  if (n <= 0 || s <= 0 || p <= 0) return;
  dim3 grid((unsigned)((n + TM - 1) / TM), (unsigned)((s + TN - 1) / TN), num_slices(p));
  hipLaunchKernelGGL(apply_f64_kernel, grid, dim3(NT), 0, st, Ah, Bh, V, out, Y, alpha, beta, n,
                     s, p);
  TSYLV_LAUNCH_CHECK();
}

}  // namespace kern
}  // namespace tsylv
