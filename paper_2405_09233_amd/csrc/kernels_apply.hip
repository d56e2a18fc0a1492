// Facewise Sylvester apply in the Fourier half spectrum, FP64 on MFMA.
//
// Algorithm 1 of section 2.1 computes a T-product as independent products
// of the Fourier slices; for M(X) = A*X - X*B (eq. (2)) that is
//     W_k = Ahat_k V_k - V_k Bhat_k,   k = 0 .. floor(p/2),
// complex slices stored as (Re, Im) plane pairs, the real DC and Nyquist
// slices as single planes.  Both products are one contraction over
// K = n + s:
//     W_k = [ Ahat_k | -V_k ] [ V_k ; Bhat_k ],
// so the whole apply is a batched complex GEMM with the small V_k Bhat_k
// term riding in the last K panel.  Complex products are four real
// v_mfma_f64_16x16x4 per 16 x 16 x 4 block (Re += Ar Vr - Ai Vi,
// Im += Ar Vi + Ai Vr).
//
// Tiling: a workgroup (4 waves) owns a TM x TN tile of W_k and streams the
// TM rows of [Ahat_k | -V_k] once through LDS in TK-deep panels, the matching
// panels of [V_k ; Bhat_k] come from L2.  The next panel is loaded into
// registers while the current one is multiplied.  Tiles are numbered slice
// major and handed out so that each XCD (workgroups go round-robin over the
// 8 XCDs) works through a contiguous range: the V_k of a slice stays in one
// XCD's L2 instead of being fetched by all eight.
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

struct ApplyArgs {
  const double* Ah;
  const double* Bh;
  const double* V;
  double* out;
  const double* Y;
  double alpha, beta;
  int64_t n, s;
  int p;
  int nrt, nct;  // row tiles, column tiles per slice
  int total;     // tiles over all slices
};

// Maps the hardware block index to a tile so that consecutive tiles land on
// the same XCD (a bijection on [0, total)).
__device__ __forceinline__ int xcd_tile(int b, int total) {
  const int q = total / 8, r = total % 8;
  const int x = b % 8;
  return x * q + (x < r ? x : r) + b / 8;
}

template <int TM, int TN, int RB, int CB, bool CPLX>
__device__ __forceinline__ void apply_tile(const ApplyArgs& a, int k, int rt, int ct,
                                           double (*As)[TK][TM], double (*Bs)[TK][TN + 1]) {
  constexpr int WR = TM / (16 * RB);  // waves along rows
  constexpr int WC = TN / (16 * CB);  // waves along columns
  static_assert(WR * WC == NT / 64, "4 waves per workgroup");
  constexpr int NA = TM * TK / NT;    // A-panel elements per thread and plane
  constexpr int NB = TK * TN / NT;    // B-panel elements per thread and plane
  static_assert(NA * NT == TM * TK && NB * NT == TK * TN, "panel split");

  const int64_t n = a.n, s = a.s, K = n + s;
  int qr, qi;
  slice_planes(a.p, k, qr, qi);
  const int64_t nn = n * n, ns = n * s, ss = s * s;
  const double* Ar = a.Ah + qr * nn;
  const double* Ai = CPLX ? a.Ah + qi * nn : nullptr;
  const double* Vr = a.V + qr * ns;
  const double* Vi = CPLX ? a.V + qi * ns : nullptr;
  const double* Br = a.Bh + qr * ss;
  const double* Bi = CPLX ? a.Bh + qi * ss : nullptr;
  const int64_t m0 = (int64_t)rt * TM, c0 = (int64_t)ct * TN;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
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

  // Element (row, kk) of the [Ahat | -V] panel and (kk, col) of [V ; Bhat].
  auto load_panels = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int idx = tid + NT * u;
      const int row = idx % TM, kk = idx / TM;
      const int64_t gr = m0 + row, gk = k0 + kk;
      double vr = 0.0, vi = 0.0;
      if (gr < n) {
        if (gk < n) {
          const int64_t off = gr + n * gk;
          vr = Ar[off];
          if (CPLX) vi = Ai[off];
        } else if (gk < K) {
          const int64_t off = gr + n * (gk - n);
          vr = -Vr[off];
          if (CPLX) vi = -Vi[off];
        }
      }
      pa_r[u] = vr;
      pa_i[u] = vi;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = tid + NT * u;
      const int kk = idx % TK, col = idx / TK;
      const int64_t gk = k0 + kk, gc = c0 + col;
      double vr = 0.0, vi = 0.0;
      if (gc < s) {
        if (gk < n) {
          const int64_t off = gk + n * gc;
          vr = Vr[off];
          if (CPLX) vi = Vi[off];
        } else if (gk < K) {
          const int64_t off = (gk - n) + s * gc;
          vr = Br[off];
          if (CPLX) vi = Bi[off];
        }
      }
      pb_r[u] = vr;
      pb_i[u] = vi;
    }
  };
  auto store_panels = [&]() {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int idx = tid + NT * u;
      const int row = idx % TM, kk = idx / TM;
      As[0][kk][row] = pa_r[u];
      if (CPLX) As[1][kk][row] = pa_i[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = tid + NT * u;
      const int kk = idx % TK, col = idx / TK;
      Bs[0][kk][col] = pb_r[u];
      if (CPLX) Bs[1][kk][col] = pb_i[u];
    }
  };

  load_panels(0);
  for (int64_t k0 = 0; k0 < K; k0 += TK) {
    store_panels();
    __syncthreads();
    if (k0 + TK < K) load_panels(k0 + TK);  // in flight during the MFMAs below
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      double far_[RB], fai[RB], fbr[CB], fbi[CB];
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const int row = (wr * RB + i) * 16 + lr;
        far_[i] = As[0][ks + lk][row];
        if (CPLX) fai[i] = As[1][ks + lk][row];
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
          if (CPLX) {
            accr[i][j] = mfma(-fai[i], fbi[j], accr[i][j]);
            acci[i][j] = mfma(far_[i], fbi[j], acci[i][j]);
            acci[i][j] = mfma(fai[i], fbr[j], acci[i][j]);
          }
        }
    }
    __syncthreads();
  }

  // Epilogue: out = alpha * W + beta * Y.  The FP64 16 x 16 result block
  // keeps element (i, j) in lane j + 16 (i mod 4), register i / 4, so lane
  // (lr, lk) holds rows lk, lk + 4, lk + 8, lk + 12 of column lr.
  double* Or = a.out + qr * ns;
  double* Oi = CPLX ? a.out + qi * ns : nullptr;
  const double* Yr = a.Y ? a.Y + qr * ns : nullptr;
  const double* Yi = (a.Y && CPLX) ? a.Y + qi * ns : nullptr;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int64_t col = c0 + (wc * CB + j) * 16 + lr;
      if (col >= s) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + (wr * RB + i) * 16 + 4 * r + lk;
        if (row >= n) continue;
        const int64_t off = row + n * col;
        double vr = a.alpha * accr[i][j][r];
        if (a.beta != 0.0) vr = fma(a.beta, Yr[off], vr);
        Or[off] = vr;
        if (CPLX) {
          double vi = a.alpha * acci[i][j][r];
          if (a.beta != 0.0) vi = fma(a.beta, Yi[off], vi);
          Oi[off] = vi;
        }
      }
    }
}

template <int TM, int TN, int RB, int CB>
__global__ __launch_bounds__(NT) void apply_mfma_f64_kernel(ApplyArgs a) {
  __shared__ double As[2][TK][TM];
  __shared__ double Bs[2][TK][TN + 1];
  const int t = xcd_tile(blockIdx.x, a.total);
  const int ct = t % a.nct;
  const int rt = (t / a.nct) % a.nrt;
  const int k = t / (a.nct * a.nrt);
  const bool real_slice = (k == 0) || (2 * k == a.p);
  if (real_slice)
    apply_tile<TM, TN, RB, CB, false>(a, k, rt, ct, As, Bs);
  else
    apply_tile<TM, TN, RB, CB, true>(a, k, rt, ct, As, Bs);
}

template <int TM, int TN, int RB, int CB>
void launch_apply(ApplyArgs a, hipStream_t st) {
  a.nrt = (int)((a.n + TM - 1) / TM);
  a.nct = (int)((a.s + TN - 1) / TN);
  a.total = num_slices(a.p) * a.nrt * a.nct;
  hipLaunchKernelGGL((apply_mfma_f64_kernel<TM, TN, RB, CB>), dim3(a.total), dim3(NT), 0, st, a);
  TSYLV_LAUNCH_CHECK();
}

}  // namespace

void apply_f64(const double* Ah, const double* Bh, const double* V, double* out, const double* Y,
               double alpha, double beta, int64_t n, int64_t s, int p, hipStream_t st) {
  if (n <= 0 || s <= 0 || p <= 0) return;
  if (beta != 0.0 && Y == nullptr) throw Error(TSYLV_EINVAL, "apply: beta != 0 needs Y");
  ApplyArgs a{Ah, Bh, V, out, beta != 0.0 ? Y : nullptr, alpha, beta, n, s, p, 0, 0, 0};
  // Column tile as wide as s needs (up to 64) so small s does not waste MFMA work.
  if (s <= 16)
    launch_apply<128, 16, 2, 1>(a, st);
  else if (s <= 32)
    launch_apply<64, 32, 1, 2>(a, st);
  else
    launch_apply<32, 64, 1, 2>(a, st);
}

}  // namespace kern
}  // namespace tsylv
