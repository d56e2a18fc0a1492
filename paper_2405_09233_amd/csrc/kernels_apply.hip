// Facewise Sylvester apply in the Fourier half spectrum on MFMA (FP64 and
// FP32; the BF16 variant is kernels_apply_bf16.hip).
//
// Algorithm 1 of section 2.1 computes a T-product as independent products
// of the Fourier slices; for M(X) = A*X - X*B (eq. (2)) that is
//     W_k = Ahat_k V_k - V_k Bhat_k,   k = 0 .. floor(p/2),
// complex slices stored as (Re, Im) plane pairs, the real DC and Nyquist
// slices as single planes.  Both products are one contraction over
// K = n + s:
//     W_k = [ Ahat_k | -V_k ] [ V_k ; Bhat_k ],
// so the whole apply is a batched complex GEMM with the small V_k Bhat_k
// term riding in the last K panels.  A complex product is three real MFMAs
// per block (Gauss's three-multiplication form: T1 = Ar Vr, T2 = Ai Vi,
// T3 = (Ar + Ai)(Vr + Vi), then Re = T1 - T2 and Im = T3 - T1 - T2 in the
// epilogue), a quarter fewer matrix-core cycles than the four-product form
// at the same operand traffic; the operand sums are formed per fragment from
// the LDS panels.  The Tubal Block Arnoldi process needs Ahat_k V_k alone
// (useB = 0, K = n).
//
// Tiling: a workgroup (4 waves) owns a TM x TN tile of W_k and streams the
// TM rows of [Ahat_k | -V_k] once through LDS in TK-deep panels; the
// matching panels of [V_k ; Bhat_k] come from L2.  The next panel is loaded
// into registers while the current one is multiplied.  Tiles are numbered
// slice major and handed out so that each XCD (workgroups go round-robin over
// the 8 XCDs) works through a contiguous range: the V_k of a slice stays in
// one XCD's L2 instead of being fetched by all eight.
#include <type_traits>

#include "kernels.hpp"

namespace tsylv {
namespace kern {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;

// Per-precision MFMA traits.  TA: storage type of the operator planes, TV:
// of the vectors, L: LDS element type, frag: one lane's MFMA operand.
//   FP64: v_mfma_f64_16x16x4; A element (i, k) in lane i + 16 k; result
//         (i, j) in lane j + 16 (i % 4), register i / 4.
//   FP32: v_mfma_f32_16x16x4; same operand layout; result (i, j) in lane
//         j + 16 (i / 4), register i % 4.
template <typename TA>
struct Mma;

template <>
struct Mma<double> {
  using TV = double;
  using L = double;
  using frag = double;
  using acc_t = d4;
  static constexpr int TK = 16, KB = 4;
  // LDS row padding (elements) and the column swizzle of the B panel
  static constexpr int PADA = 0, PADB = 1, SWB = 0;
  __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static int row(int r, int lk) { return 4 * r + lk; }
  __device__ static L a_in(double x) { return x; }
  __device__ static L v_in(double x) { return x; }
  __device__ static L neg(L x) { return -x; }
  template <int LD>
  __device__ static frag ld(const L (*S)[LD], int ks, int lk, int i) { return S[ks + lk][i]; }
  __device__ static acc_t mma(frag a, frag b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <>
struct Mma<float> {
  using TV = float;
  using L = float;
  using frag = float;
  using acc_t = f4;
  static constexpr int TK = 16, KB = 4;
  // 4-byte elements: rows padded by 16 so that the 4 k rows a wave reads at
  // once fall into disjoint bank ranges; the B panel is written with k
  // fastest across lanes, so its column is XORed with bits 2..3 of k, which
  // spreads those writes over all banks and leaves each 16-column block of a
  // row where it was (reads of one k step see one constant XOR)
  static constexpr int PADA = 16, PADB = 16, SWB = 12;
  __device__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static int row(int r, int lk) { return 4 * lk + r; }
  __device__ static L a_in(float x) { return x; }
  __device__ static L v_in(float x) { return x; }
  __device__ static L neg(L x) { return -x; }
  template <int LD>
  __device__ static frag ld(const L (*S)[LD], int ks, int lk, int i) { return S[ks + lk][i]; }
  __device__ static acc_t mma(frag a, frag b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// storage type of the operator planes for a traits tag
template <typename Tag> struct Store { using T = Tag; };

template <typename Tag>
struct ApplyArgs {
  using TA = typename Store<Tag>::T;
  using TV = typename Mma<Tag>::TV;
  const TA* Ah;
  const TA* Bh;
  const TV* V;
  TV* out;
  const TV* Y;
  double alpha, beta;
  int64_t n, s;
  int p;
  int useB;      // include the -V_k Bhat_k term
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

template <typename Tag, int TM, int TN, int RB, int CB, int TK, bool CPLX>
__device__ __forceinline__ void apply_tile(
    const ApplyArgs<Tag>& a, int k, int rt, int ct,
    typename Mma<Tag>::L (*As)[TK][TM + Mma<Tag>::PADA],
    typename Mma<Tag>::L (*Bs)[TK][TN + Mma<Tag>::PADB]) {
  using M = Mma<Tag>;
  using L = typename M::L;
  using TA = typename Store<Tag>::T;
  using TV = typename M::TV;
  using frag = typename M::frag;
  using acc_t = typename M::acc_t;
  constexpr int KB = M::KB;
  constexpr int WR = TM / (16 * RB);  // waves along rows
  constexpr int WC = TN / (16 * CB);  // waves along columns
  static_assert(WR * WC == NT / 64, "4 waves per workgroup");
  constexpr int NA = TM * TK / NT;    // A-panel elements per thread and plane
  constexpr int NB = TK * TN / NT;    // B-panel elements per thread and plane
  static_assert(NA * NT == TM * TK && NB * NT == TK * TN, "panel split");

  const int64_t n = a.n, s = a.s, K = a.useB ? n + s : n;
  int qr, qi;
  slice_planes(a.p, k, qr, qi);
  const int64_t nn = n * n, ns = n * s, ss = s * s;
  const TA* Ar = a.Ah + qr * nn;
  const TA* Ai = CPLX ? a.Ah + qi * nn : nullptr;
  const TV* Vr = a.V + qr * ns;
  const TV* Vi = CPLX ? a.V + qi * ns : nullptr;
  const TA* Br = a.Bh + qr * ss;
  const TA* Bi = CPLX ? a.Bh + qi * ss : nullptr;
  const int64_t m0 = (int64_t)rt * TM, c0 = (int64_t)ct * TN;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave % WR, wc = wave / WR;
  const int lr = lane & 15, lk = lane >> 4;

  // real slices: accr = Ar Vr; complex: accr = T1, acci = T2, accs = T3
  acc_t accr[RB][CB], acci[RB][CB], accs[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      accr[i][j] = M::zero();
      acci[i][j] = M::zero();
      accs[i][j] = M::zero();
    }

  L pa_r[NA], pa_i[NA], pb_r[NB], pb_i[NB];
  const L zl = M::v_in((TV)0);

  // Element (row, kk) of the [Ahat | -V] panel and (kk, col) of [V ; Bhat].
  auto load_panels = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int idx = tid + NT * u;
      const int row = idx % TM, kk = idx / TM;
      const int64_t gr = m0 + row, gk = k0 + kk;
      L vr = zl, vi = zl;
      if (gr < n) {
        if (gk < n) {
          const int64_t off = gr + n * gk;
          vr = M::a_in(Ar[off]);
          if (CPLX) vi = M::a_in(Ai[off]);
        } else if (gk < K) {
          const int64_t off = gr + n * (gk - n);
          vr = M::neg(M::v_in(Vr[off]));
          if (CPLX) vi = M::neg(M::v_in(Vi[off]));
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
      L vr = zl, vi = zl;
      if (gc < s) {
        if (gk < n) {
          const int64_t off = gk + n * gc;
          vr = M::v_in(Vr[off]);
          if (CPLX) vi = M::v_in(Vi[off]);
        } else if (gk < K) {
          const int64_t off = (gk - n) + s * gc;
          vr = M::a_in(Br[off]);
          if (CPLX) vi = M::a_in(Bi[off]);
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
      const int pc = col ^ (kk & M::SWB);
      Bs[0][kk][pc] = pb_r[u];
      if (CPLX) Bs[1][kk][pc] = pb_i[u];
    }
  };

  load_panels(0);
  for (int64_t k0 = 0; k0 < K; k0 += TK) {
    store_panels();
    __syncthreads();
    if (k0 + TK < K) load_panels(k0 + TK);  // in flight during the MFMAs below
#pragma unroll
    for (int ks = 0; ks < TK; ks += KB) {
      frag far_[RB], fai[RB], fas[RB], fbr[CB], fbi[CB], fbs[CB];
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const int row = (wr * RB + i) * 16 + lr;
        far_[i] = M::template ld<TM + M::PADA>(As[0], ks, lk, row);
        if (CPLX) {
          fai[i] = M::template ld<TM + M::PADA>(As[1], ks, lk, row);
          fas[i] = far_[i] + fai[i];
        }
      }
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        // ks is a multiple of 4, so (ks + lk) & SWB == ks & SWB
        const int col = ((wc * CB + j) * 16 + lr) ^ (ks & M::SWB);
        fbr[j] = M::template ld<TN + M::PADB>(Bs[0], ks, lk, col);
        if (CPLX) {
          fbi[j] = M::template ld<TN + M::PADB>(Bs[1], ks, lk, col);
          fbs[j] = fbr[j] + fbi[j];
        }
      }
      // Every accumulator is updated once per k step, so a full sweep over
      // the blocks separates dependent MFMAs.
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          accr[i][j] = M::mma(far_[i], fbr[j], accr[i][j]);
          if (CPLX) {
            acci[i][j] = M::mma(fai[i], fbi[j], acci[i][j]);
            accs[i][j] = M::mma(fas[i], fbs[j], accs[i][j]);
          }
        }
    }
    __syncthreads();
  }

  // Epilogue: out = alpha * W + beta * Y (row of result register r given by
  // the traits; column lr of each 16 x 16 block).
  TV* Or = a.out + qr * ns;
  TV* Oi = CPLX ? a.out + qi * ns : nullptr;
  const TV* Yr = a.Y ? a.Y + qr * ns : nullptr;
  const TV* Yi = (a.Y && CPLX) ? a.Y + qi * ns : nullptr;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int64_t col = c0 + (wc * CB + j) * 16 + lr;
      if (col >= s) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + (wr * RB + i) * 16 + M::row(r, lk);
        if (row >= n) continue;
        const int64_t off = row + n * col;
        const double t1 = (double)accr[i][j][r];
        double vr;
        if (CPLX) {
          const double t2 = (double)acci[i][j][r];
          vr = a.alpha * (t1 - t2);
          double vi = a.alpha * ((double)accs[i][j][r] - t1 - t2);
          if (a.beta != 0.0) vi = fma(a.beta, (double)Yi[off], vi);
          Oi[off] = (TV)vi;
        } else {
          vr = a.alpha * t1;
        }
        if (a.beta != 0.0) vr = fma(a.beta, (double)Yr[off], vr);
        Or[off] = (TV)vr;
      }
    }
}

// MINW: waves per SIMD the register allocation must leave room for (1: the
// compiler's choice).
template <typename Tag, int TM, int TN, int RB, int CB, int TK, int MINW>
__global__ __launch_bounds__(NT, MINW) void apply_mfma_kernel(ApplyArgs<Tag> a) {
  using L = typename Mma<Tag>::L;
  __shared__ L As[2][TK][TM + Mma<Tag>::PADA];
  __shared__ L Bs[2][TK][TN + Mma<Tag>::PADB];
  const int t = xcd_tile(blockIdx.x, a.total);
  const int ct = t % a.nct;
  const int rt = (t / a.nct) % a.nrt;
  const int k = t / (a.nct * a.nrt);
  const bool real_slice = (k == 0) || (2 * k == a.p);
  if (real_slice)
    apply_tile<Tag, TM, TN, RB, CB, TK, false>(a, k, rt, ct, As, Bs);
  else
    apply_tile<Tag, TM, TN, RB, CB, TK, true>(a, k, rt, ct, As, Bs);
}

template <typename Tag, int TM, int TN, int RB, int CB, int TK = Mma<Tag>::TK, int MINW = 1>
void launch_apply(ApplyArgs<Tag> a, hipStream_t st) {
  a.nrt = (int)((a.n + TM - 1) / TM);
  a.nct = (int)((a.s + TN - 1) / TN);
  a.total = num_slices(a.p) * a.nrt * a.nct;
  hipLaunchKernelGGL((apply_mfma_kernel<Tag, TM, TN, RB, CB, TK, MINW>), dim3(a.total), dim3(NT),
                     0, st, a);
  TSYLV_LAUNCH_CHECK();
}

// Tile variants (TM x TN workgroup tile, RB x CB 16 x 16 blocks per wave, k
// panel depth), the candidates of the autotuner; every one is valid for
// every shape.
template <typename Tag>
void launch_variant(int v, ApplyArgs<Tag> a, hipStream_t st) {
  switch (v) {
    case 0: launch_apply<Tag, 128, 16, 2, 1>(a, st); break;
    case 1: launch_apply<Tag, 64, 32, 1, 2>(a, st); break;
    case 2: launch_apply<Tag, 32, 64, 1, 2>(a, st); break;
    case 3: launch_apply<Tag, 64, 64, 1, 4>(a, st); break;
    case 4: launch_apply<Tag, 64, 64, 2, 2>(a, st); break;
    case 5: launch_apply<Tag, 128, 32, 2, 2>(a, st); break;
    case 6: launch_apply<Tag, 32, 64, 1, 2, 32>(a, st); break;  // 32-deep k panels
    case 7: launch_apply<Tag, 64, 32, 1, 2, 32>(a, st); break;
    case 8: launch_apply<Tag, 128, 16, 2, 1, 32>(a, st); break;
    case 9: launch_apply<Tag, 64, 16, 1, 1, 32>(a, st); break;
    // registers capped for three / four waves per SIMD
    case 10: launch_apply<Tag, 64, 32, 1, 2, 16, 3>(a, st); break;
    case 11: launch_apply<Tag, 64, 32, 1, 2, 16, 4>(a, st); break;
    case 12: launch_apply<Tag, 32, 64, 1, 2, 16, 3>(a, st); break;
    case 13: launch_apply<Tag, 64, 64, 1, 4, 16, 2>(a, st); break;
    case 14: launch_apply<Tag, 64, 16, 1, 1, 16, 3>(a, st); break;
    case 15: launch_apply<Tag, 64, 16, 1, 1, 16, 4>(a, st); break;
    case 16: launch_apply<Tag, 64, 16, 1, 1, 32, 2>(a, st); break;
    default: throw Error(TSYLV_EINVAL, "apply: unknown tile variant");
  }
}

// Without a tuned choice: a column tile as wide as s needs, so small s does
// not waste MFMA work.  FP64 above s = 16 takes the tiles whose registers
// are capped so that three waves share a SIMD (two with the compiler's
// allocation of 212 registers): 64 x 32 up to s = 64 (2.41 vs 2.90 ms
// uncapped at n = 4096, s = 64, p = 32) and 64 x 64 at two waves beyond
// (32.4 vs 40.4 ms for the uncapped 64 x 32 at n = 8192, s = 128, p = 64).
// FP32 (at most 196 registers, four waves already) keeps 64 x 32 up to
// s = 64 (1.35 vs 1.40 ms for 64 x 64 at n = 4096) and 64 x 64 beyond
// (17.2 vs 18.2 ms for 64 x 32 at n = 8192).
template <typename Tag>
int default_variant(int64_t n, int64_t s) {
  constexpr bool f64 = std::is_same<Tag, double>::value;
  // FP64 at small s streams its operator (HBM-bound): from n = 2048 on,
  // 64 x 16 tiles with 16-deep k panels at four waves per SIMD keep the most
  // of it in flight (0.90 ms = 4.8 TB/s at n = 4096, s = 16, p = 32,
  // against 1.06 ms with 32-deep panels at two waves and 1.49 ms for
  // 128 x 16; 0.25 vs 0.29 ms for the capped 64 x 32 at n = 2048, s = 24,
  // p = 16); smaller operators (a few k panels per tile) run 3-6 % faster
  // with the 32-deep panels
  if (s <= 24) return f64 ? (n >= 2048 ? 15 : (s <= 16 ? 9 : 10)) : (s <= 16 ? 0 : 1);
  if (s <= 64) return f64 ? 10 : 1;
  return f64 ? 13 : 3;
}

// Batched apply: the tiles of many instances in one launch (their first
// tiles in refs, ascending).  STEP: W = M(V_j) for the stepping instances;
// RESID: V_0 = Zc - M(Zx) for the instances not done.
// (The mode is a template parameter, as in the batched vector kernels.)
template <int TM, int TN, int RB, int CB, int TK, int MODE, int MINW>
__global__ __launch_bounds__(NT, MINW) void apply_batch_kernel(const BatchItem* __restrict__ items,
                                                         const BatchApplyRef* __restrict__ refs,
                                                         int nref, int total,
                                                         const BatchState* __restrict__ st,
                                                         const int* __restrict__ jp) {
  using M = Mma<double>;
  using L = typename M::L;
  __shared__ L As[2][TK][TM + M::PADA];
  __shared__ L Bs[2][TK][TN + M::PADB];
  const int t = xcd_tile(blockIdx.x, total);
  int lo = 0, hi = nref - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (refs[mid].tile0 <= t) lo = mid;
    else hi = mid - 1;
  }
  const BatchApplyRef r = refs[lo];
  const BatchItem& it = items[r.item];
  const bool on = (MODE == BM_STEP) ? st[r.item].active != 0 : st[r.item].done == 0;
  if (!on) return;
  const int lt = t - r.tile0;
  const int ct = lt % r.nct;
  const int rt = (lt / r.nct) % r.nrt;
  const int k = lt / (r.nct * r.nrt);
  ApplyArgs<double> a{};
  a.Ah = it.Ah;
  a.Bh = it.Bh;
  a.n = it.n;
  a.s = it.s;
  a.p = it.p;
  a.useB = 1;
  if constexpr (MODE == BM_STEP) {
    a.V = it.V + (int64_t)(*jp) * it.ldv;
    a.out = it.W;
    a.Y = nullptr;
    a.alpha = 1.0;
    a.beta = 0.0;
  } else {
    a.V = it.Zx;
    a.out = it.V;
    a.Y = it.Zc;
    a.alpha = -1.0;
    a.beta = 1.0;
  }
  if ((k == 0) || (2 * k == a.p))
    apply_tile<double, TM, TN, RB, CB, TK, false>(a, k, rt, ct, As, Bs);
  else
    apply_tile<double, TM, TN, RB, CB, TK, true>(a, k, rt, ct, As, Bs);
}

template <typename Tag>
void apply_any(const typename Store<Tag>::T* Ah, const typename Store<Tag>::T* Bh,
               const typename Mma<Tag>::TV* V, typename Mma<Tag>::TV* out,
               const typename Mma<Tag>::TV* Y, double alpha, double beta, int64_t n, int64_t s,
               int p, bool useB, int variant, hipStream_t st) {
  if (n <= 0 || s <= 0 || p <= 0) return;
  if (beta != 0.0 && Y == nullptr) throw Error(TSYLV_EINVAL, "apply: beta != 0 needs Y");
  if (useB && Bh == nullptr) throw Error(TSYLV_EINVAL, "apply: missing Bhat");
  ApplyArgs<Tag> a{Ah, Bh, V, out, beta != 0.0 ? Y : nullptr, alpha, beta, n, s, p,
                   useB ? 1 : 0, 0, 0, 0};
  launch_variant<Tag>(variant >= 0 ? variant : default_variant<Tag>(n, s), a, st);
}

}  // namespace

void apply_f64(const double* Ah, const double* Bh, const double* V, double* out, const double* Y,
               double alpha, double beta, int64_t n, int64_t s, int p, hipStream_t st,
               int variant) {
  apply_any<double>(Ah, Bh, V, out, Y, alpha, beta, n, s, p, Bh != nullptr, variant, st);
}

void apply_f32(const float* Ah, const float* Bh, const float* V, float* out, const float* Y,
               double alpha, double beta, int64_t n, int64_t s, int p, hipStream_t st,
               int variant) {
  apply_any<float>(Ah, Bh, V, out, Y, alpha, beta, n, s, p, Bh != nullptr, variant, st);
}

template <int TM, int TN, int RB, int CB, int TK = Mma<double>::TK, int MINW = 1>
static void launch_batch(const BatchItem* items, const BatchApplyRef* refs, int nref, int total,
                         BatchState* st, const int* jp, int mode, hipStream_t s) {
  if (mode == BM_STEP)
    klaunch(apply_batch_kernel<TM, TN, RB, CB, TK, BM_STEP, MINW>, dim3(total), dim3(NT), 0, s,
            items, refs, nref, total, st, jp);
  else if (mode == BM_RESID)
    klaunch(apply_batch_kernel<TM, TN, RB, CB, TK, BM_RESID, MINW>, dim3(total), dim3(NT), 0, s,
            items, refs, nref, total, st, jp);
  else
    throw Error(TSYLV_EINVAL, "batch apply: mode");
}

void batch_apply(const BatchItem* items, const BatchApplyRef* refs, int nref, int total_tiles,
                 int variant, BatchState* st, const int* jp, int mode, hipStream_t st_) {
  if (nref <= 0 || total_tiles <= 0) return;
  switch (variant) {
    case 0: launch_batch<128, 16, 2, 1>(items, refs, nref, total_tiles, st, jp, mode, st_); break;
    // 64 x 32 with the register cap of the single-instance default (three
    // waves per SIMD); 64 x 16 keeps 32-deep panels, uncapped: the batched
    // instances with s <= 16 are small (few k panels, latency-bound), and
    // the capped 16-deep form ran the 256-instance small mix at 5.9k
    // instead of 7.6k solves/s
    case 1:
      launch_batch<64, 32, 1, 2, 16, 3>(items, refs, nref, total_tiles, st, jp, mode, st_);
      break;
    case 2: launch_batch<32, 64, 1, 2>(items, refs, nref, total_tiles, st, jp, mode, st_); break;
    case 9: launch_batch<64, 16, 1, 1, 32>(items, refs, nref, total_tiles, st, jp, mode, st_); break;
    default: throw Error(TSYLV_EINVAL, "batch apply: unsupported tile variant");
  }
  TSYLV_LAUNCH_CHECK();
}

// Tile shape of an instance in a batched apply: the default of its s, so an
// instance computes the same bits in any batch.
// the batched kernel's tiles (batch_apply_tiles): 64 x 16 up to s = 16,
// 64 x 32 beyond
int batch_apply_variant(int64_t s) { return s <= 16 ? 9 : 1; }
int batch_apply_tiles(int variant, int64_t n, int64_t s, int p, int* nrt, int* nct) {
  int tm, tn;
  switch (variant) {
    case 0: tm = 128; tn = 16; break;
    case 1: tm = 64; tn = 32; break;
    case 2: tm = 32; tn = 64; break;
    case 9: tm = 64; tn = 16; break;
    default: throw Error(TSYLV_EINVAL, "batch apply: unsupported tile variant");
  }
  *nrt = (int)((n + tm - 1) / tm);
  *nct = (int)((s + tn - 1) / tn);
  return num_slices(p) * *nrt * *nct;
}

int apply_variant_count(int prec) { return prec == TSYLV_BF16 ? 11 : 17; }

int apply_default_variant(int prec, int64_t n, int64_t s) {
  if (prec == TSYLV_FP64) return default_variant<double>(n, s);
  if (prec == TSYLV_FP32) return default_variant<float>(n, s);
  return bf16_default_variant(s);
}

}  // namespace kern
}  // namespace tsylv
