// Batched planar-complex FP64 GEMM over the Fourier slices, on MFMA.
//
// The Tubal Block Arnoldi process (section 5.1, Algorithms 6 and 7) works
// slice by slice in the Fourier domain with tube-valued coefficients: the
// T-transpose becomes the conjugate transpose of every slice (Def. 2.2
// item 4) and every tube product a complex scalar product.  Its block
// Gram-Schmidt (H_ij = V_i^T * W, W -= V_i * H_ij), its Tubal-QR (Cholesky QR
// of every slice) and the solution update X += V_m * Y are therefore one
// batched complex GEMM per operation,
//     C_k = alpha op(A_k) B_k + beta C_k,   op = identity or conjugate transpose,
// over the slices k = 0 .. floor(p/2) (real DC/Nyquist slices as real GEMMs).
//
// Operands are addressed through plane descriptors so the Krylov basis can be
// used in place: element (r, c) of slice k is at
//     base + q * plane + r + (c % cb) * ld + (c / cb) * bs
// with q the Re or Im plane of slice k (cb = columns per block, bs = block
// stride: the basis blocks are separate vectors).  Long contractions (the
// Gram matrices contract over n) are split over K into partial products that a
// second kernel sums in a fixed order.
#include <algorithm>

#include "kernels.hpp"

namespace tsylv {
namespace kern {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NT = 256;
constexpr int TK = 16;

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct GemmArgs {
  PMat A, B;
  double* C;
  int64_t planeC, ldC;
  int64_t M, N, K;
  double alpha, beta;
  int p;
  int conjA;
  int nmt, nnt, ksplit, total;
  int64_t kchunk;
  double* partial;  // ksplit * p * M * N when ksplit > 1
};

__device__ __forceinline__ int64_t pm_off(const PMat& m, int q, int64_t r, int64_t c) {
  return q * m.plane + r + (c % m.cb) * m.ld + (c / m.cb) * m.bs;
}

__device__ __forceinline__ int xcd_tile(int b, int total) {
  const int q = total / 8, r = total % 8;
  const int x = b % 8;
  return x * q + (x < r ? x : r) + b / 8;
}

template <int TM, int TN, int RB, int CB, bool CPLX, bool CONJA, int NTH>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int k, int mt, int nt, int split,
                                          double (*As)[TK][TM + 1], double (*Bs)[TK][TN + 1]) {
  constexpr int WR = TM / (16 * RB);
  constexpr int WC = TN / (16 * CB);
  static_assert(WR * WC == NTH / 64, "one wave per RB x CB block group");
  constexpr int NA = TM * TK / NTH;
  constexpr int NB = TK * TN / NTH;
  static_assert(NA * NTH == TM * TK && NB * NTH == TK * TN, "panel split");

  int qr, qi;
  slice_planes(g.p, k, qr, qi);
  const int64_t m0 = (int64_t)mt * TM, c0 = (int64_t)nt * TN;
  const int64_t kbeg = (int64_t)split * g.kchunk;
  const int64_t kend = min(g.K, kbeg + g.kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave % WR, wc = wave / WR;
  const int lr = lane & 15, lk = lane >> 4;

  d4 accr[RB][CB], acci[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      accr[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      acci[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  double pa_r[NA], pa_i[NA], pb_r[NB], pb_i[NB];

  auto load = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int idx = tid + NTH * u;
      // op(A)(m, kk): contiguous along kk for the conjugate transpose, along m otherwise
      const int m = CONJA ? idx / TK : idx % TM;
      const int kk = CONJA ? idx % TK : idx / TM;
      const int64_t gm = m0 + m, gk = k0 + kk;
      double vr = 0.0, vi = 0.0;
      if (gm < g.M && gk < kend) {
        const int64_t off = CONJA ? pm_off(g.A, qr, gk, gm) : pm_off(g.A, qr, gm, gk);
        vr = g.A.base[off];
        if (CPLX) {
          const int64_t offi = off + (int64_t)(qi - qr) * g.A.plane;
          vi = CONJA ? -g.A.base[offi] : g.A.base[offi];
        }
      }
      pa_r[u] = vr;
      pa_i[u] = vi;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = tid + NTH * u;
      const int kk = idx % TK, c = idx / TK;
      const int64_t gk = k0 + kk, gc = c0 + c;
      double vr = 0.0, vi = 0.0;
      if (gc < g.N && gk < kend) {
        const int64_t off = pm_off(g.B, qr, gk, gc);
        vr = g.B.base[off];
        if (CPLX) vi = g.B.base[off + (int64_t)(qi - qr) * g.B.plane];
      }
      pb_r[u] = vr;
      pb_i[u] = vi;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int idx = tid + NTH * u;
      const int m = CONJA ? idx / TK : idx % TM;
      const int kk = CONJA ? idx % TK : idx / TM;
      As[0][kk][m] = pa_r[u];
      if (CPLX) As[1][kk][m] = pa_i[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = tid + NTH * u;
      const int kk = idx % TK, c = idx / TK;
      Bs[0][kk][c] = pb_r[u];
      if (CPLX) Bs[1][kk][c] = pb_i[u];
    }
  };

  if (kbeg < kend) load(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += TK) {
    store();
    __syncthreads();
    if (k0 + TK < kend) load(k0 + TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      double far_[RB], fai[RB], fain[RB], fbr[CB], fbi[CB];
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const int row = (wr * RB + i) * 16 + lr;
        far_[i] = As[0][ks + lk][row];
        if (CPLX) {
          fai[i] = As[1][ks + lk][row];
          fain[i] = -fai[i];
        }
      }
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        const int col = (wc * CB + j) * 16 + lr;
        fbr[j] = Bs[0][ks + lk][col];
        if (CPLX) fbi[j] = Bs[1][ks + lk][col];
      }
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          accr[i][j] = mfma(far_[i], fbr[j], accr[i][j]);
          if (CPLX) acci[i][j] = mfma(far_[i], fbi[j], acci[i][j]);
        }
      if (CPLX) {
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j) {
            accr[i][j] = mfma(fain[i], fbi[j], accr[i][j]);
            acci[i][j] = mfma(fai[i], fbr[j], acci[i][j]);
          }
      }
    }
    __syncthreads();
  }

  // Result element (i, j) of a 16 x 16 FP64 block: lane j + 16 (i % 4), register i / 4.
  const int64_t MN = g.M * g.N;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int64_t col = c0 + (wc * CB + j) * 16 + lr;
      if (col >= g.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + (wr * RB + i) * 16 + 4 * r + lk;
        if (row >= g.M) continue;
        if (g.ksplit > 1) {
          double* P = g.partial + (int64_t)split * g.p * MN;
          P[qr * MN + row + g.M * col] = accr[i][j][r];
          if (CPLX) P[qi * MN + row + g.M * col] = acci[i][j][r];
        } else {
          const int64_t off = row + g.ldC * col;
          double* Cr = g.C + qr * g.planeC;
          double vr = g.alpha * accr[i][j][r];
          if (g.beta != 0.0) vr = fma(g.beta, Cr[off], vr);
          Cr[off] = vr;
          if (CPLX) {
            double* Ci = g.C + qi * g.planeC;
            double vi = g.alpha * acci[i][j][r];
            if (g.beta != 0.0) vi = fma(g.beta, Ci[off], vi);
            Ci[off] = vi;
          }
        }
      }
    }
}

template <int TM, int TN, int RB, int CB, bool CONJA, int NTH>
__global__ __launch_bounds__(NTH) void zgemm_kernel(GemmArgs g) {
  __shared__ double As[2][TK][TM + 1];
  __shared__ double Bs[2][TK][TN + 1];
  const int t = xcd_tile(blockIdx.x, g.total);
  const int nt = t % g.nnt;
  const int mt = (t / g.nnt) % g.nmt;
  const int split = (t / (g.nnt * g.nmt)) % g.ksplit;
  const int k = t / (g.nnt * g.nmt * g.ksplit);
  const bool real_slice = (k == 0) || (2 * k == g.p);
  if (real_slice)
    gemm_tile<TM, TN, RB, CB, false, CONJA, NTH>(g, k, mt, nt, split, As, Bs);
  else
    gemm_tile<TM, TN, RB, CB, true, CONJA, NTH>(g, k, mt, nt, split, As, Bs);
}

// C = alpha * sum_split partial + beta * C over all p planes (fixed order).
__global__ void splitk_reduce_kernel(const double* __restrict__ partial, int ksplit, int p,
                                     int64_t M, int64_t N, double* __restrict__ C, int64_t planeC,
                                     int64_t ldC, double alpha, double beta) {
  const int64_t MN = M * N, tot = (int64_t)p * MN;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = i / MN, rc = i % MN, r = rc % M, c = rc / M;
    double acc = 0.0;
    for (int sp = 0; sp < ksplit; ++sp) acc += partial[(int64_t)sp * tot + i];
    double* cp = C + q * planeC + r + ldC * c;
    double v = alpha * acc;
    if (beta != 0.0) v = fma(beta, *cp, v);
    *cp = v;
  }
}

template <int TM, int TN, int RB, int CB, int NTH = NT>
void launch(GemmArgs g, hipStream_t st) {
  g.nmt = (int)((g.M + TM - 1) / TM);
  g.nnt = (int)((g.N + TN - 1) / TN);
  g.total = num_slices(g.p) * g.nmt * g.nnt * g.ksplit;
  if (g.conjA)
    hipLaunchKernelGGL((zgemm_kernel<TM, TN, RB, CB, true, NTH>), dim3(g.total), dim3(NTH), 0,
                       st, g);
  else
    hipLaunchKernelGGL((zgemm_kernel<TM, TN, RB, CB, false, NTH>), dim3(g.total), dim3(NTH), 0,
                       st, g);
  TSYLV_LAUNCH_CHECK();
}

}  // namespace

int64_t zgemm_partial_elems(int64_t M, int64_t N, int64_t K, int p) {
  return (int64_t)zgemm_splits(M, N, K, p) * p * M * N;
}

int zgemm_splits(int64_t M, int64_t N, int64_t K, int p) {
  const int64_t tm = N <= 16 ? 128 : 64;
  const int64_t tn = N <= 16 ? 16 : (N <= 32 ? 32 : 64);
  const int64_t tiles = num_slices(p) * ((M + tm - 1) / tm) * ((N + tn - 1) / tn);
  int64_t split = (2048 + tiles - 1) / tiles;
  const int64_t maxsplit = K / 256;
  if (split > maxsplit) split = maxsplit;
  if (split < 1) split = 1;
  if (split > 64) split = 64;
  return (int)split;
}

void zgemm(const PMat& A, bool conjA, const PMat& B, double* C, int64_t planeC, int64_t ldC,
           int64_t M, int64_t N, int64_t K, double alpha, double beta, int p, double* partial,
           hipStream_t st) {
  if (M <= 0 || N <= 0 || p <= 0) return;
  GemmArgs g{};
  g.A = A;
  g.B = B;
  g.C = C;
  g.planeC = planeC;
  g.ldC = ldC;
  g.M = M;
  g.N = N;
  g.K = K;
  g.alpha = alpha;
  g.beta = beta;
  g.p = p;
  g.conjA = conjA ? 1 : 0;
  g.ksplit = partial ? zgemm_splits(M, N, K, p) : 1;
  g.kchunk = round_up((K + g.ksplit - 1) / g.ksplit, TK);
  g.partial = partial;
  if (N <= 16)
    launch<128, 16, 2, 1>(g, st);
  else if (N <= 32)
    launch<64, 32, 1, 2>(g, st);
  else  // 64 x 64 tiles of 8 waves (16 x 32 each): twice the products per loaded byte
    launch<64, 64, 1, 2, 512>(g, st);
  if (g.ksplit > 1) {
    const int64_t tot = (int64_t)p * M * N;
    int blocks = (int)std::min<int64_t>((tot + 255) / 256, 4096);
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks), dim3(256), 0, st, partial, g.ksplit, p,
                       M, N, C, planeC, ldC, alpha, beta);
    TSYLV_LAUNCH_CHECK();
  }
}

}  // namespace kern
}  // namespace tsylv
