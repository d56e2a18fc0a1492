// Facewise Sylvester apply with BF16 Fourier slices (FP32 accumulation),
// HBM-bound path of the mixed-precision inner solves.
//
// W_k = Ahat_k V_k - V_k Bhat_k (Algorithm 1 step 2 for eq. (2)).  Both MFMA
// operands are stored in the lane order of v_mfma_f32_16x16x32_bf16, so every
// operand fragment is one coalesced 16-byte access per lane:
//   * the operator planes, rounded to BF16 once at setup: plane q, 16-row
//     block rb, 32-deep k block kb form one 1 KB chunk whose lane i + 16 g
//     holds A(16 rb + i, 32 kb + 8 g .. 8 g + 7).  Within a plane the chunks
//     run in the order (rb / 8, kb, rb % 8), so the 8 row blocks that waves
//     of one workgroup stream side by side read 8 KB of contiguous memory
//     per k block;
//   * the Krylov vector, rounded to BF16 at the start of every apply into a
//     scratch buffer: plane q, 16-column block cb, k block kb form one chunk
//     whose lane i + 16 g holds V(32 kb + 8 g .. 8 g + 7, 16 cb + i).
// A workgroup owns a column tile and a row range of one slice sized so that
// all workgroups stream the same number of operator bytes (a complex slice
// has two planes, a real one one) and the grid fills whole rounds of the
// CUs.  Each wave streams its own 16 operator rows straight from HBM into a
// register ring D k blocks deep; the V chunks of the column tile, needed by
// every wave, pass through LDS in double-buffered phases of P k blocks (one
// barrier per phase).  The operator is read from HBM once; V (s n / 8 KB per
// slice) once per workgroup, mostly from L2, which the XCD-contiguous tile
// order keeps on one XCD.  The small -V_k Bhat_k term is a short extra
// contraction over s in the epilogue.
#include "kernels.hpp"

namespace tsylv {
namespace kern {

namespace {

// Row blocks per group of the operator's chunk order (divides the row-block
// padding).
constexpr int64_t kRowGroup = 8;

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}

// Double -> bf16 with a single rounding (via the tie check on the double).
__device__ __forceinline__ uint16_t bf16_bits_d(double x) {
  float f = (float)x;
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  uint32_t lower = u & 0xffffu, up = u >> 16;
  if (lower > 0x8000u) {
    up += 1;
  } else if (lower == 0x8000u) {
    double lo = (double)__uint_as_float(up << 16), hi = (double)__uint_as_float((up + 1) << 16);
    double dl = fabs(x - lo), dh = fabs(hi - x);
    if (dh < dl || (dh == dl && (up & 1u))) up += 1;
  }
  return (uint16_t)up;
}

__device__ __forceinline__ f4 mma(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf8 neg8(bf8 x) {
  u16x8 u = __builtin_bit_cast(u16x8, x);
  u ^= (unsigned short)0x8000u;
  return __builtin_bit_cast(bf8, u);
}

// grid-stride over lane chunks: (q, rb, kb, lane) -> 8 bf16
__global__ void tile_bf16_kernel(const double* __restrict__ Ah, uint16_t* __restrict__ At,
                                 int64_t n, int p, int64_t nrb, int64_t nkb) {
  const int64_t total = (int64_t)p * nrb * nkb * 64;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int L = (int)(t % 64);
    const int64_t chunk = t / 64;
    const int64_t q = chunk / (nkb * nrb), c = chunk % (nkb * nrb);
    const int64_t kb = (c % (nkb * kRowGroup)) / kRowGroup;
    const int64_t rb = c / (nkb * kRowGroup) * kRowGroup + c % kRowGroup;
    const int64_t row = 16 * rb + (L % 16), k0 = 32 * kb + 8 * (L / 16);
    u16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t k = k0 + e;
      const double a = (row < n && k < n) ? Ah[q * n * n + row + n * k] : 0.0;
      v[e] = bf16_bits_d(a);
    }
    *reinterpret_cast<u16x8*>(At + t * 8) = v;
  }
}

// grid-stride over lane chunks: (q, cb, kb, lane) -> 8 bf16 of V's columns
__global__ void tile_v_bf16_kernel(const float* __restrict__ V, uint16_t* __restrict__ Vt,
                                   int64_t n, int64_t s, int p, int64_t ncb, int64_t nkb) {
  const int64_t total = (int64_t)p * ncb * nkb * 64;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int L = (int)(t % 64);
    const int64_t chunk = t / 64;
    const int64_t kb = chunk % nkb, cb = (chunk / nkb) % ncb, q = chunk / (nkb * ncb);
    const int64_t col = 16 * cb + (L % 16), k0 = 32 * kb + 8 * (L / 16);
    const float* src = V + q * n * s + n * col;
    u16x8 v;
    if (col < s && k0 + 8 <= n) {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = bf16_bits(src[k0 + e]);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (col < s && k0 + e < n) ? bf16_bits(src[k0 + e]) : 0;
    }
    *reinterpret_cast<u16x8*>(Vt + t * 8) = v;
  }
}

// Tiled BF16 copy of a X for FP64 planes X (same order as tile_v_bf16_kernel;
// a X rounded to FP32, then to the nearest-even BF16).
__global__ void tile_scale_bf16_kernel(const double* __restrict__ X, uint16_t* __restrict__ Xt,
                                       double a, int64_t n, int64_t s, int p, int64_t ncb,
                                       int64_t nkb) {
  const int64_t total = (int64_t)p * ncb * nkb * 64;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int L = (int)(t % 64);
    const int64_t chunk = t / 64;
    const int64_t kb = chunk % nkb, cb = (chunk / nkb) % ncb, q = chunk / (nkb * ncb);
    const int64_t col = 16 * cb + (L % 16), k0 = 32 * kb + 8 * (L / 16);
    const double* src = X + q * n * s + n * col;
    u16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e)
      v[e] = (col < s && k0 + e < n) ? bf16_bits((float)(a * src[k0 + e])) : (uint16_t)0;
    *reinterpret_cast<u16x8*>(Xt + t * 8) = v;
  }
}

// X -= sum_i y[i] V_i for tiled BF16 vectors V_i and FP64 planes X: every
// thread owns one lane slot of a chunk (8 consecutive rows of one column),
// sums the nv vectors in FP64 in index order and subtracts from the 8 rows
// of X.
__global__ void untile_update_bf16_kernel(const uint16_t* __restrict__ V, int64_t ldv, int nv,
                                          const double* __restrict__ y, double* __restrict__ X,
                                          int64_t n, int64_t s, int p, int64_t ncb,
                                          int64_t nkb) {
  const int64_t total = (int64_t)p * ncb * nkb * 64;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int L = (int)(t % 64);
    const int64_t chunk = t / 64;
    const int64_t kb = chunk % nkb, cb = (chunk / nkb) % ncb, q = chunk / (nkb * ncb);
    const int64_t col = 16 * cb + (L % 16), k0 = 32 * kb + 8 * (L / 16);
    if (col >= s || k0 >= n) continue;
    double acc[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] = 0.0;
    for (int i = 0; i < nv; ++i) {
      const u16x8 v = *reinterpret_cast<const u16x8*>(V + i * ldv + t * 8);
      const double c = y[i];
#pragma unroll
      for (int e = 0; e < 8; ++e)
        acc[e] = fma(c, (double)__uint_as_float((uint32_t)v[e] << 16), acc[e]);
    }
    double* dst = X + q * n * s + n * col;
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (k0 + e < n) dst[k0 + e] -= acc[e];
  }
}

struct Bf16Args {
  const uint16_t* At;  // tiled operator planes (nrb x nkb chunks per plane)
  const uint16_t* Bb;  // bf16 planes of Bhat (s x s column-major), or null
  const uint16_t* Vt;  // tiled V planes (ncb x nkb chunks per plane)
  const float* V;      // V in FP32 planes (null when the vectors are tiled)
  float* out;
  uint16_t* outt;      // tiled BF16 output (the tiled-vector form)
  const float* Y;
  double alpha, beta;
  int64_t n, s;
  int p;
  int64_t nrb, nkb, ncb;
  int nrt, nct, total;
};

__device__ __forceinline__ int xcd_tile(int b, int total) {
  const int q = total / 8, r = total % 8;
  const int x = b % 8;
  return x * q + (x < r ? x : r) + b / 8;
}

// Operator chunks are read exactly once per apply: non-temporal loads keep
// them from pushing the V chunks, which every workgroup of a slice re-reads,
// out of L2.
__device__ __forceinline__ bf8 ld8_stream(const uint16_t* p) {
  return __builtin_bit_cast(bf8, __builtin_nontemporal_load(reinterpret_cast<const u16x8*>(p)));
}

// The -V_k Bhat_k term (a short contraction over s straight from global
// memory) and the epilogue out = alpha W + beta Y for R x CB blocks.
// Element (row, col) of plane q of a tiled vector (see tile_v_bf16_kernel).
__device__ __forceinline__ int64_t tiled_at(const Bf16Args& a, int q, int64_t row, int64_t col) {
  return (((int64_t)q * a.ncb + col / 16) * a.nkb + row / 32) * 512 +
         ((col % 16) + 16 * ((row % 32) / 8)) * 8 + row % 8;
}

template <int CB, int R, bool CPLX, bool TIO>
__device__ __forceinline__ void bf16_finish(const Bf16Args& a, int qr, int qi, int64_t rb0,
                                            int64_t cb0, f4 (&accr)[R][CB], f4 (&acci)[R][CB]) {
  const int64_t n = a.n, s = a.s, ns = n * s;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lg = lane >> 4;
  const float* Vr = TIO ? nullptr : a.V + qr * ns;
  const float* Vi = (CPLX && !TIO) ? a.V + qi * ns : nullptr;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t row = 16 * (rb0 + r) + li;
    // -V_k Bhat_k: a short contraction over s straight from global memory.
    if (a.Bb) {
      const uint16_t* Bbr = a.Bb + qr * s * s;
      const uint16_t* Bbi = CPLX ? a.Bb + qi * s * s : nullptr;
      for (int64_t k1 = 0; k1 < s; k1 += 32) {
        u16x8 fr, fi;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t kk = k1 + 8 * lg + e;
          const bool ok = row < n && kk < s;
          if (TIO) {
            fr[e] = ok ? (uint16_t)(a.Vt[tiled_at(a, qr, row, kk)] ^ 0x8000u) : (uint16_t)0;
            if (CPLX)
              fi[e] = ok ? (uint16_t)(a.Vt[tiled_at(a, qi, row, kk)] ^ 0x8000u) : (uint16_t)0;
          } else {
            fr[e] = ok ? (uint16_t)(bf16_bits(Vr[row + n * kk]) ^ 0x8000u) : (uint16_t)0;
            if (CPLX)
              fi[e] = ok ? (uint16_t)(bf16_bits(Vi[row + n * kk]) ^ 0x8000u) : (uint16_t)0;
          }
        }
        const bf8 nvr = __builtin_bit_cast(bf8, fr);  // -Re V
        bf8 nvi, pvi;
        if (CPLX) {
          nvi = __builtin_bit_cast(bf8, fi);  // -Im V
          pvi = neg8(nvi);                    // +Im V
        }
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          const int64_t col = 16 * (cb0 + j) + li;
          u16x8 gr, gi;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int64_t kk = k1 + 8 * lg + e;
            const bool ok = col < s && kk < s;
            gr[e] = ok ? Bbr[kk + s * col] : (uint16_t)0;
            if (CPLX) gi[e] = ok ? Bbi[kk + s * col] : (uint16_t)0;
          }
          const bf8 gbr = __builtin_bit_cast(bf8, gr);
          accr[r][j] = mma(nvr, gbr, accr[r][j]);  // -Vr Br
          if (CPLX) {
            const bf8 gbi = __builtin_bit_cast(bf8, gi);
            acci[r][j] = mma(nvr, gbi, acci[r][j]);  // -Vr Bi
            accr[r][j] = mma(pvi, gbi, accr[r][j]);  // +Vi Bi
            acci[r][j] = mma(nvi, gbr, acci[r][j]);  // -Vi Br
          }
        }
      }
    }

    // Epilogue (FP32 result layout: element (i, j) in lane j + 16 (i / 4),
    // register i % 4).
    if (TIO) {
      // Rows 16 rb + 4 lg .. + 3 of column col are 4 consecutive elements of
      // one lane slot of the tiled output: one 8-byte store.  Rows >= n and
      // columns >= s are written as zero (they are the tiled padding).
      const int64_t rb = rb0 + r;
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        const int64_t col = 16 * (cb0 + j) + li;
        const int64_t at = tiled_at(a, 0, 16 * rb + 4 * lg, col);
        const int64_t plane = a.ncb * a.nkb * 512;
        u16x4 vr, vi;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = col < s && 16 * rb + 4 * lg + e < n;
          vr[e] = ok ? bf16_bits((float)(a.alpha * (double)accr[r][j][e])) : (uint16_t)0;
          if (CPLX) vi[e] = ok ? bf16_bits((float)(a.alpha * (double)acci[r][j][e])) : (uint16_t)0;
        }
        *reinterpret_cast<u16x4*>(a.outt + qr * plane + at) = vr;
        if (CPLX) *reinterpret_cast<u16x4*>(a.outt + qi * plane + at) = vi;
      }
      continue;
    }
    float* Or = a.out + qr * ns;
    float* Oi = CPLX ? a.out + qi * ns : nullptr;
    const float* Yr = a.Y ? a.Y + qr * ns : nullptr;
    const float* Yi = (a.Y && CPLX) ? a.Y + qi * ns : nullptr;
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int64_t col = 16 * (cb0 + j) + li;
      if (col >= s) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t rr = 16 * (rb0 + r) + 4 * lg + e;
        if (rr >= n) continue;
        const int64_t off = rr + n * col;
        double vr = a.alpha * (double)accr[r][j][e];
        if (a.beta != 0.0) vr += a.beta * (double)Yr[off];
        Or[off] = (float)vr;
        if (CPLX) {
          double vi = a.alpha * (double)acci[r][j][e];
          if (a.beta != 0.0) vi += a.beta * (double)Yi[off];
          Oi[off] = (float)vi;
        }
      }
    }
  }
}

// Balanced variant: a workgroup of NW waves owns one column tile and a
// contiguous range of row blocks of ONE slice -- G row blocks of a complex
// slice or 2 G of a real one (half the work each) -- so every workgroup has
// the same amount of operator to stream and the launch has no ragged last
// round.  Its waves walk their row blocks (one per wave at a time, 16 rows)
// in lock step, sharing each phase of V chunks through LDS.
struct WgPlan {
  int G;        // complex row blocks per workgroup (multiple of NW)
  int wr, wc;   // workgroups per real / complex slice and column tile
};

template <int CB, int D, int P, int NW, int R, bool CPLX, bool TIO>
__device__ __forceinline__ void bf16_wg_tasks(const Bf16Args& a, const WgPlan& pl, int k,
                                              int64_t rb_begin, int64_t rb_count, int64_t cb0,
                                              uint16_t* lds) {
  constexpr int NPL = CPLX ? 2 : 1;
  constexpr int CPK = NPL * CB;
  constexpr int CH = P * CPK;
  static_assert(CH % NW == 0, "every wave stages the same number of chunks");
  constexpr int NPASS = CH / NW;
  int qr, qi;
  slice_planes(a.p, k, qr, qi);
  const int64_t nkb = a.nkb, nrb_real = (a.n + 15) / 16;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint16_t* Vsrc[NPASS];
#pragma unroll
  for (int v = 0; v < NPASS; ++v) {
    const int c = v * NW + wave;
    const int kl = c / CPK, pln = (c % CPK) / CB, j = c % CB;
    const int q = pln ? qi : qr;
    Vsrc[v] = a.Vt + (((int64_t)q * a.ncb + cb0 + j) * nkb + kl) * 512 + lane * 8;
  }
  const int64_t nph = nkb / P;
  const int64_t ntask = (rb_count + NW * R - 1) / (NW * R);
  for (int64_t task = 0; task < ntask; ++task) {
    // this wave's R consecutive row blocks
    const uint16_t* Ar[R];
    const uint16_t* Ai[R];
    int64_t rbs[R];
    bool store[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t rb_want = rb_begin + (task * NW + wave) * R + r;
      store[r] = rb_want < rb_begin + rb_count && rb_want < nrb_real;
      rbs[r] = min(rb_want, a.nrb - 1);  // past the end: any valid block, not stored
      // chunk (rb, kb) of a plane sits at ((rb / 8) nkb + kb) 8 + rb % 8
      const int64_t rofs = ((rbs[r] / kRowGroup) * nkb * kRowGroup + rbs[r] % kRowGroup) * 512;
      Ar[r] = a.At + (int64_t)qr * a.nrb * nkb * 512 + rofs + lane * 8;
      Ai[r] = CPLX ? a.At + (int64_t)qi * a.nrb * nkb * 512 + rofs + lane * 8 : nullptr;
    }
    u16x8 stage[NPASS];
    auto fetch = [&](int64_t ph) {
#pragma unroll
      for (int v = 0; v < NPASS; ++v)
        stage[v] = *reinterpret_cast<const u16x8*>(Vsrc[v] + ph * P * 512);
    };
    auto put = [&](int buf) {
#pragma unroll
      for (int v = 0; v < NPASS; ++v)
        *reinterpret_cast<u16x8*>(lds + ((int64_t)buf * CH + v * NW + wave) * 512 + lane * 8) =
            stage[v];
    };
    auto frag = [&](int buf, int kl, int pln, int j) -> bf8 {
      return __builtin_bit_cast(
          bf8, *reinterpret_cast<const u16x8*>(
                   lds + ((int64_t)buf * CH + kl * CPK + pln * CB + j) * 512 + lane * 8));
    };
    f4 accr[R][CB], acci[R][CB];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        accr[r][j] = f4{0.f, 0.f, 0.f, 0.f};
        acci[r][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
    bf8 ar[D][R], ai[D][R];
    auto loadA = [&](int64_t kb, int u) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        ar[u][r] = ld8_stream(Ar[r] + kb * (kRowGroup * 512));
        if (CPLX) ai[u][r] = ld8_stream(Ai[r] + kb * (kRowGroup * 512));
      }
    };
    fetch(0);
#pragma unroll
    for (int u = 0; u < D; ++u) loadA(u, u);
    put(0);
    __syncthreads();
    for (int64_t ph = 0; ph < nph; ++ph) {
      const int buf = (int)(ph & 1);
      fetch(min(ph + 1, nph - 1));
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < P; ++u) {
        const int d = u % D;
        bf8 mai[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (CPLX) mai[r] = neg8(ai[d][r]);
        // one column block's V fragments at a time (fewer live registers,
        // so a deeper operator ring fits)
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          const bf8 br = frag(buf, u, 0, j);
          bf8 bi;
          if (CPLX) bi = frag(buf, u, 1, j);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            accr[r][j] = mma(ar[d][r], br, accr[r][j]);
            if (CPLX) {
              acci[r][j] = mma(ar[d][r], bi, acci[r][j]);
              accr[r][j] = mma(mai[r], bi, accr[r][j]);
              acci[r][j] = mma(ai[d][r], br, acci[r][j]);
            }
          }
        }
        // keep the refill right behind the MFMAs that free its slot
        __builtin_amdgcn_sched_barrier(0);
        loadA(min(ph * P + u + D, nkb - 1), d);
        __builtin_amdgcn_sched_barrier(0);
      }
      put(buf ^ 1);
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!store[r]) continue;
      f4 fr[1][CB], fi[1][CB];
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        fr[0][j] = accr[r][j];
        fi[0][j] = acci[r][j];
      }
      bf16_finish<CB, 1, CPLX, TIO>(a, qr, qi, rbs[r], cb0, fr, fi);
    }
  }
}

template <int CB, int D, int P, int NW, int R, bool TIO>
__global__ __launch_bounds__(NW * 64) void apply_bf16_wg_kernel(Bf16Args a, WgPlan pl) {
  extern __shared__ __attribute__((aligned(16))) uint16_t lds[];
  const int t = xcd_tile(blockIdx.x, a.total);
  const int ct = t % a.nct;
  int w = t / a.nct;  // workgroup index within the slice-major order
  const int nsl = num_slices(a.p);
  int k = 0;
  for (; k < nsl; ++k) {
    const bool real = (k == 0) || (2 * k == a.p);
    const int wk = real ? pl.wr : pl.wc;
    if (w < wk) break;
    w -= wk;
  }
  const bool real = (k == 0) || (2 * k == a.p);
  const int64_t span = real ? 2 * (int64_t)pl.G : pl.G;
  const int64_t rb_begin = (int64_t)w * span;
  const int64_t cb0 = (int64_t)ct * CB;
  if (real)
    bf16_wg_tasks<CB, D, P, NW, R, false, TIO>(a, pl, k, rb_begin, span, cb0, lds);
  else
    bf16_wg_tasks<CB, D, P, NW, R, true, TIO>(a, pl, k, rb_begin, span, cb0, lds);
}

// Row blocks are padded to a multiple of kRowPad and column blocks to a
// multiple of kColPad (the largest CB).
constexpr int64_t kRowPad = 16, kColPad = 4;
static_assert(kRowPad % kRowGroup == 0, "row groups tile the padded row blocks");
// k blocks are padded to a multiple of kKPad, which every ring depth divides.
constexpr int64_t kKPad = 8;

// Picks G (complex row blocks per workgroup, a multiple of NW) so that the
// number of workgroups fills whole rounds of one workgroup per CU.
inline WgPlan plan_wg(int64_t n, int p, int nct, int nw, int ncu) {
  const int64_t nrb = (n + 15) / 16;
  const int nsl = num_slices(p), nreal = (p % 2 == 0 && p > 1) ? 2 : 1;
  const int ncplx = nsl - nreal;
  WgPlan best{nw, 0, 0};
  double best_cost = 1e300;
  for (int64_t G = nw; G <= std::max<int64_t>(nw, ((nrb + nw - 1) / nw) * nw); G += nw) {
    const int wr = (int)((nrb + 2 * G - 1) / (2 * G)), wc = (int)((nrb + G - 1) / G);
    const int64_t total = (int64_t)nct * (nreal * wr + ncplx * wc);
    const double cost = (double)((total + ncu - 1) / ncu) * (double)G;
    if (cost < best_cost) {
      best_cost = cost;
      best = WgPlan{(int)G, wr, wc};
    }
  }
  return best;
}

template <int CB, int D, int P, int NW, int R, bool TIO>
void launch_wg(Bf16Args a, int ncu, hipStream_t st) {
  static_assert(kKPad % P == 0 && P % D == 0, "phase and ring must divide the k padding");
  a.nct = (int)((a.s + 16 * CB - 1) / (16 * CB));
  const WgPlan pl = plan_wg(a.n, a.p, a.nct, NW * R, ncu);
  const int nsl = num_slices(a.p), nreal = (a.p % 2 == 0 && a.p > 1) ? 2 : 1;
  a.total = a.nct * (nreal * pl.wr + (nsl - nreal) * pl.wc);
  const size_t lds = 2 * (size_t)P * 2 * CB * 1024;  // two buffers of complex phases
  TSYLV_HIP(hipFuncSetAttribute(
      reinterpret_cast<const void*>(&apply_bf16_wg_kernel<CB, D, P, NW, R, TIO>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((apply_bf16_wg_kernel<CB, D, P, NW, R, TIO>), dim3(a.total), dim3(NW * 64), lds,
                     st, a, pl);
  TSYLV_LAUNCH_CHECK();
}


// ---------------------------------------------------------------------------
// Wide variant for s > 64: 32 x 32 x 16 MFMAs, one workgroup per 128-column
// tile, so at s = 128 the operator is streamed from HBM exactly once (the
// 16 x 16 x 32 variants above hold at most 64 columns per workgroup and
// read it once per column tile).  A 32 x 32 block of W takes half the LDS
// bytes per flop of four 16 x 16 blocks (each V fragment feeds a 32-row
// operator fragment), which is what keeps the V reads from LDS off the
// critical path at this width.
//
// The tiled layouts stay those of the 16 x 16 x 32 kernels; the fragments
// of the 32 x 32 x 16 instruction are gathered from them:
//   A operand (32 rows x 16 k), lane l: row l % 32, k = 8 (l / 32) + e.
//     Rows 32 R .. 32 R + 31 are the 16-row chunks 2 R and 2 R + 1 (adjacent
//     in the grouped chunk order), so lane l reads 16 bytes of chunk
//     2 R + (l / 16) % 2 at lane slot (l % 16) + 16 (2 h + l / 32), where
//     h = 0, 1 picks the 16-deep half of the chunk's 32 k;
//   B operand (16 k x 32 columns), lane l: column l % 32, k = 8 (l / 32) + e:
//     the same offsets in the two 16-column chunks of V;
//   D (32 x 32), lane l, register r: column l % 32, row
//     8 (r / 4) + 4 (l / 32) + r % 4.
// Both operands of a product use the same (lane group, element) -> k map,
// so the sum over k is the full one whatever order the hardware pairs them.
typedef float f16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f16v mma32(bf8 a, bf8 b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Lane offset (in bf16 elements) of a 32-wide fragment inside a pair of
// adjacent 1 KB chunks, for k half h.
__device__ __forceinline__ int frag32_off(int lane, int h) {
  return ((lane >> 4) & 1) * 512 + ((lane & 15) + 16 * (2 * h + (lane >> 5))) * 8;
}

// -V_k Bhat_k (a contraction over s, gathered from global memory) into the
// 32 x 32 accumulators of rows 32 R32 .., and the epilogue.
template <int CB32, bool CPLX, bool TIO>
__device__ __forceinline__ void w32_finish(const Bf16Args& a, int qr, int qi, int64_t R32,
                                           int64_t ct, f16v (&accr)[CB32], f16v (&acci)[CB32]) {
  const int64_t n = a.n, s = a.s, ns = n * s;
  const int lane = threadIdx.x & 63;
  const int lc = lane & 31, lg = lane >> 5;
  const int64_t row = 32 * R32 + lc;
  const int64_t col0 = ct * 32 * CB32;
  if (a.Bb) {
    const uint16_t* Bbr = a.Bb + (int64_t)qr * s * s;
    const uint16_t* Bbi = CPLX ? a.Bb + (int64_t)qi * s * s : nullptr;
    const float* Vr = TIO ? nullptr : a.V + (int64_t)qr * ns;
    const float* Vi = (CPLX && !TIO) ? a.V + (int64_t)qi * ns : nullptr;
    for (int64_t k1 = 0; k1 < s; k1 += 16) {
      u16x8 fr, fi;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t kk = k1 + 8 * lg + e;
        const bool ok = row < n && kk < s;
        if (TIO) {
          fr[e] = ok ? (uint16_t)(a.Vt[tiled_at(a, qr, row, kk)] ^ 0x8000u) : (uint16_t)0;
          if (CPLX)
            fi[e] = ok ? (uint16_t)(a.Vt[tiled_at(a, qi, row, kk)] ^ 0x8000u) : (uint16_t)0;
        } else {
          fr[e] = ok ? (uint16_t)(bf16_bits(Vr[row + n * kk]) ^ 0x8000u) : (uint16_t)0;
          if (CPLX) fi[e] = ok ? (uint16_t)(bf16_bits(Vi[row + n * kk]) ^ 0x8000u) : (uint16_t)0;
        }
      }
      const bf8 nvr = __builtin_bit_cast(bf8, fr);  // -Re V
      bf8 nvi, pvi;
      if (CPLX) {
        nvi = __builtin_bit_cast(bf8, fi);  // -Im V
        pvi = neg8(nvi);                    // +Im V
      }
#pragma unroll
      for (int j = 0; j < CB32; ++j) {
        const int64_t col = col0 + 32 * j + lc;
        u16x8 gr, gi;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t kk = k1 + 8 * lg + e;
          const bool ok = col < s && kk < s;
          gr[e] = ok ? Bbr[kk + s * col] : (uint16_t)0;
          if (CPLX) gi[e] = ok ? Bbi[kk + s * col] : (uint16_t)0;
        }
        const bf8 gbr = __builtin_bit_cast(bf8, gr);
        accr[j] = mma32(nvr, gbr, accr[j]);  // -Vr Br
        if (CPLX) {
          const bf8 gbi = __builtin_bit_cast(bf8, gi);
          acci[j] = mma32(nvr, gbi, acci[j]);  // -Vr Bi
          accr[j] = mma32(pvi, gbi, accr[j]);  // +Vi Bi
          acci[j] = mma32(nvi, gbr, acci[j]);  // -Vi Br
        }
      }
    }
  }
  if (TIO) {
    // Rows 32 R32 + 8 t + 4 lg .. + 3 of a column are 4 consecutive elements
    // of one lane slot of the tiled output: one 8-byte store.  Rows >= n and
    // columns >= s inside existing chunks are written as zero (the tiled
    // padding); chunks past the padded column count are not written.
    const int64_t plane = a.ncb * a.nkb * 512;
#pragma unroll
    for (int j = 0; j < CB32; ++j) {
      const int64_t col = col0 + 32 * j + lc;
      if (col / 16 >= a.ncb) continue;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t r0 = 32 * R32 + 8 * t + 4 * lg;
        const int64_t at = tiled_at(a, 0, r0, col);
        u16x4 vr, vi;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = col < s && r0 + e < n;
          vr[e] = ok ? bf16_bits((float)(a.alpha * (double)accr[j][4 * t + e])) : (uint16_t)0;
          if (CPLX)
            vi[e] = ok ? bf16_bits((float)(a.alpha * (double)acci[j][4 * t + e])) : (uint16_t)0;
        }
        *reinterpret_cast<u16x4*>(a.outt + qr * plane + at) = vr;
        if (CPLX) *reinterpret_cast<u16x4*>(a.outt + qi * plane + at) = vi;
      }
    }
    return;
  }
  float* Or = a.out + (int64_t)qr * ns;
  float* Oi = CPLX ? a.out + (int64_t)qi * ns : nullptr;
  const float* Yr = a.Y ? a.Y + (int64_t)qr * ns : nullptr;
  const float* Yi = (a.Y && CPLX) ? a.Y + (int64_t)qi * ns : nullptr;
#pragma unroll
  for (int j = 0; j < CB32; ++j) {
    const int64_t col = col0 + 32 * j + lc;
    if (col >= s) continue;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t rr = 32 * R32 + 8 * (r / 4) + 4 * lg + r % 4;
      if (rr >= n) continue;
      const int64_t off = rr + n * col;
      double vr = a.alpha * (double)accr[j][r];
      if (a.beta != 0.0) vr += a.beta * (double)Yr[off];
      Or[off] = (float)vr;
      if (CPLX) {
        double vi = a.alpha * (double)acci[j][r];
        if (a.beta != 0.0) vi += a.beta * (double)Yi[off];
        Oi[off] = (float)vi;
      }
    }
  }
}

// A workgroup of NW waves owns column tile ct (32 CB32 columns) and span32
// 32-row blocks of one slice; its waves walk RW blocks each at a time in
// lock step, sharing each phase of P k blocks of V through LDS (double
// buffered), each streaming its operator rows from HBM into a register ring
// D k blocks deep.
template <int CB32, int D, int P, int NW, int RW, bool CPLX, bool TIO>
__device__ __forceinline__ void w32_tasks(const Bf16Args& a, int k, int64_t rb32_begin,
                                          int64_t rb32_count, int64_t ct, uint16_t* lds) {
  constexpr int NPL = CPLX ? 2 : 1;
  constexpr int CB16 = 2 * CB32;
  constexpr int CPK = NPL * CB16;  // 1 KB chunks of V per k block
  constexpr int CH = P * CPK;      // per phase
  static_assert(CH % NW == 0, "every wave stages the same number of chunks");
  constexpr int NPASS = CH / NW;
  int qr, qi;
  slice_planes(a.p, k, qr, qi);
  const int64_t nkb = a.nkb;
  const int64_t nrb32_real = (a.n + 31) / 32;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int off0 = frag32_off(lane, 0), off1 = frag32_off(lane, 1);
  // V chunks this wave stages (null: a chunk past the padded columns, zero)
  const uint16_t* Vsrc[NPASS];
#pragma unroll
  for (int v = 0; v < NPASS; ++v) {
    const int c = v * NW + wave;
    const int kl = c / CPK, pln = (c % CPK) / CB16, j16 = c % CB16;
    const int q = pln ? qi : qr;
    const int64_t cb = ct * CB16 + j16;
    Vsrc[v] = cb < a.ncb ? a.Vt + (((int64_t)q * a.ncb + cb) * nkb + kl) * 512 + lane * 8
                         : nullptr;
  }
  const int64_t nph = nkb / P;
  const int64_t ntask = (rb32_count + NW * RW - 1) / (NW * RW);
  for (int64_t task = 0; task < ntask; ++task) {
    const uint16_t* Ar[RW];
    const uint16_t* Ai[RW];
    int64_t rbs[RW];
    bool store[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int64_t want = rb32_begin + (task * NW + wave) * RW + r;
      store[r] = want < rb32_begin + rb32_count && want < nrb32_real;
      rbs[r] = min(want, a.nrb / 2 - 1);  // past the end: any valid block, not stored
      const int64_t rb = 2 * rbs[r];      // first of its two 16-row chunks
      const int64_t rofs = ((rb / kRowGroup) * nkb * kRowGroup + rb % kRowGroup) * 512;
      Ar[r] = a.At + (int64_t)qr * a.nrb * nkb * 512 + rofs;
      Ai[r] = CPLX ? a.At + (int64_t)qi * a.nrb * nkb * 512 + rofs : nullptr;
    }
    u16x8 stage[NPASS];
    auto fetch = [&](int64_t ph) {
#pragma unroll
      for (int v = 0; v < NPASS; ++v)
        stage[v] = Vsrc[v] ? *reinterpret_cast<const u16x8*>(Vsrc[v] + ph * P * 512)
                           : u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    };
    auto put = [&](int buf) {
#pragma unroll
      for (int v = 0; v < NPASS; ++v)
        *reinterpret_cast<u16x8*>(lds + ((int64_t)buf * CH + v * NW + wave) * 512 + lane * 8) =
            stage[v];
    };
    auto frag = [&](int buf, int kl, int pln, int j, int off) -> bf8 {
      return __builtin_bit_cast(
          bf8, *reinterpret_cast<const u16x8*>(
                   lds + ((int64_t)buf * CH + kl * CPK + pln * CB16 + 2 * j) * 512 + off));
    };
    f16v accr[RW][CB32], acci[RW][CB32];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int j = 0; j < CB32; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          accr[r][j][e] = 0.f;
          acci[r][j][e] = 0.f;
        }
    // ring slot u: [row block][k half] fragments of the real / imaginary plane
    bf8 ar[D][RW][2], ai[D][RW][2];
    auto loadA = [&](int64_t kb, int u) {
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int64_t base = kb * (kRowGroup * 512);
        ar[u][r][0] = ld8_stream(Ar[r] + base + off0);
        ar[u][r][1] = ld8_stream(Ar[r] + base + off1);
        if (CPLX) {
          ai[u][r][0] = ld8_stream(Ai[r] + base + off0);
          ai[u][r][1] = ld8_stream(Ai[r] + base + off1);
        }
      }
    };
    fetch(0);
#pragma unroll
    for (int u = 0; u < D; ++u) loadA(u, u);
    put(0);
    __syncthreads();
    // Super-phases of L = lcm(P, D) k blocks, so that the ring slot of every
    // k block is known at compile time (it is kb % D) whatever P and D are.
    constexpr int L = (P % D == 0) ? P : ((D % P == 0) ? D : P * D);
    static_assert(kKPad % L == 0, "a super-phase must divide the k padding");
    for (int64_t sp = 0; sp < nkb / L; ++sp)
#pragma unroll
    for (int q = 0; q < L / P; ++q) {
      const int64_t ph = sp * (L / P) + q;
      const int buf = (int)(ph & 1);
      fetch(min(ph + 1, nph - 1));
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < P; ++u) {
        const int d = (q * P + u) % D;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int off = h ? off1 : off0;
          bf8 mai[RW];
#pragma unroll
          for (int r = 0; r < RW; ++r)
            if (CPLX) mai[r] = neg8(ai[d][r][h]);
#pragma unroll
          for (int j = 0; j < CB32; ++j) {
            const bf8 br = frag(buf, u, 0, j, off);
            bf8 bi;
            if (CPLX) bi = frag(buf, u, 1, j, off);
#pragma unroll
            for (int r = 0; r < RW; ++r) {
              accr[r][j] = mma32(ar[d][r][h], br, accr[r][j]);
              if (CPLX) {
                acci[r][j] = mma32(ar[d][r][h], bi, acci[r][j]);
                accr[r][j] = mma32(mai[r], bi, accr[r][j]);
                acci[r][j] = mma32(ai[d][r][h], br, acci[r][j]);
              }
            }
          }
        }
        // the refill right behind the MFMAs that free its slot
        __builtin_amdgcn_sched_barrier(0);
        loadA(min(ph * P + u + D, nkb - 1), d);
        __builtin_amdgcn_sched_barrier(0);
      }
      put(buf ^ 1);
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < RW; ++r)
      if (store[r]) w32_finish<CB32, CPLX, TIO>(a, qr, qi, rbs[r], ct, accr[r], acci[r]);
  }
}

template <int CB32, int D, int P, int NW, int RW, bool TIO>
__global__ __launch_bounds__(NW * 64) void apply_bf16_w32_kernel(Bf16Args a, WgPlan pl) {
  extern __shared__ __attribute__((aligned(16))) uint16_t lds[];
  const int t = xcd_tile(blockIdx.x, a.total);
  const int ct = t % a.nct;
  int w = t / a.nct;
  const int nsl = num_slices(a.p);
  int k = 0;
  for (; k < nsl; ++k) {
    const bool real = (k == 0) || (2 * k == a.p);
    const int wk = real ? pl.wr : pl.wc;
    if (w < wk) break;
    w -= wk;
  }
  const bool real = (k == 0) || (2 * k == a.p);
  // G counts 16-row blocks: a complex slice's workgroup owns G of them, a
  // real one's 2 G (G is a multiple of 2 NW RW)
  const int64_t span32 = real ? (int64_t)pl.G : pl.G / 2;
  const int64_t rb32_begin = (int64_t)w * span32;
  if (real)
    w32_tasks<CB32, D, P, NW, RW, false, TIO>(a, k, rb32_begin, span32, ct, lds);
  else
    w32_tasks<CB32, D, P, NW, RW, true, TIO>(a, k, rb32_begin, span32, ct, lds);
}

template <int CB32, int D, int P, int NW, int RW, bool TIO>
void launch_w32(Bf16Args a, int ncu, hipStream_t st) {
  static_assert(kKPad % P == 0 && kKPad % D == 0, "phase and ring must divide the k padding");
  a.nct = (int)((a.s + 32 * CB32 - 1) / (32 * CB32));
  const WgPlan pl = plan_wg(a.n, a.p, a.nct, 2 * NW * RW, ncu);
  const int nsl = num_slices(a.p), nreal = (a.p % 2 == 0 && a.p > 1) ? 2 : 1;
  a.total = a.nct * (nreal * pl.wr + (nsl - nreal) * pl.wc);
  const size_t lds = 2 * (size_t)P * 2 * (2 * CB32) * 1024;  // two buffers of complex phases
  TSYLV_HIP(hipFuncSetAttribute(
      reinterpret_cast<const void*>(&apply_bf16_w32_kernel<CB32, D, P, NW, RW, TIO>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((apply_bf16_w32_kernel<CB32, D, P, NW, RW, TIO>), dim3(a.total),
                     dim3(NW * 64), lds, st, a, pl);
  TSYLV_LAUNCH_CHECK();
}


}  // namespace

int bf16_default_variant(int64_t s) { return s <= 16 ? 0 : (s <= 32 ? 1 : (s <= 64 ? 2 : 10)); }

static int64_t row_blocks(int64_t n) { return ((n + 15) / 16 + kRowPad - 1) / kRowPad * kRowPad; }
static int64_t k_blocks(int64_t n) { return ((n + 31) / 32 + kKPad - 1) / kKPad * kKPad; }
static int64_t col_blocks(int64_t s) { return ((s + 15) / 16 + kColPad - 1) / kColPad * kColPad; }

int64_t bf16_tiled_elems(int64_t n, int p) {
  return (int64_t)p * row_blocks(n) * k_blocks(n) * 512;
}

int64_t bf16_vtiled_elems(int64_t n, int64_t s, int p) {
  return (int64_t)p * col_blocks(s) * k_blocks(n) * 512;
}

void tile_operator_bf16(const double* Ah, uint16_t* At, int64_t n, int p, hipStream_t st) {
  const int64_t nrb = row_blocks(n), nkb = k_blocks(n);
  const int64_t total = (int64_t)p * nrb * nkb * 64;
  int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(tile_bf16_kernel, dim3(blocks), dim3(256), 0, st, Ah, At, n, p, nrb, nkb);
  TSYLV_LAUNCH_CHECK();
}

// Variants (column blocks, ring depth, phase length, waves, row blocks per
// wave), the autotuner's candidates; the default per s is the best of a
// sweep at n = 4096, p = 32, s = 16 / 32 / 64 and n = 8192, p = 64, s = 128.
// Deeper rings and longer phases (4/4/4/8/2, 4/2/8/8/2) fit in registers but
// measured the same as variant 2 at n = 4096, s = 64, p = 32 (the kernel is
// not short of loads in flight there), and two 4-wave workgroups per CU
// (4/2/2/4/2), 1 % faster alone, 3 % slower inside a solve.  Above s = 64
// the wide kernel with phases of one k block (variant 10) is the default:
// its staging needs 10 fewer registers (245 against 255) and it ran 2 %
// faster than the same kernel with two-block phases (variant 4) at
// n = 8192, s = 128, p = 64, despite a barrier per k block.
template <bool TIO>
void launch_cfg(const Bf16Args& a, int variant, hipStream_t st) {
  static int ncu_cached[64] = {};
  int dev = 0;
  TSYLV_HIP(hipGetDevice(&dev));
  int& ncu = ncu_cached[dev & 63];
  if (ncu == 0) TSYLV_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  switch (variant >= 0 ? variant : bf16_default_variant(a.s)) {
    case 0: launch_wg<1, 4, 8, 8, 2, TIO>(a, ncu, st); break;
    case 1: launch_wg<2, 2, 4, 8, 2, TIO>(a, ncu, st); break;
    case 2: launch_wg<4, 2, 2, 8, 2, TIO>(a, ncu, st); break;
    case 3: launch_wg<4, 8, 8, 8, 1, TIO>(a, ncu, st); break;
    case 4: launch_w32<4, 2, 2, 8, 1, TIO>(a, ncu, st); break;
    case 5: launch_w32<2, 2, 2, 8, 1, TIO>(a, ncu, st); break;
    case 6: launch_w32<4, 2, 2, 4, 2, TIO>(a, ncu, st); break;
    case 7: launch_w32<4, 4, 2, 4, 1, TIO>(a, ncu, st); break;
    case 8: launch_w32<4, 8, 2, 4, 1, TIO>(a, ncu, st); break;
    case 9: launch_w32<2, 4, 2, 8, 1, TIO>(a, ncu, st); break;
    case 10: launch_w32<4, 2, 1, 8, 1, TIO>(a, ncu, st); break;
    default: throw Error(TSYLV_EINVAL, "apply: unknown BF16 variant");
  }
}

void apply_bf16(const uint16_t* At, const uint16_t* Bb, const float* V, uint16_t* Vt,
                float* out, const float* Y, double alpha, double beta, int64_t n, int64_t s,
                int p, hipStream_t st, int variant) {
  if (n <= 0 || s <= 0 || p <= 0) return;
  if (beta != 0.0 && Y == nullptr) throw Error(TSYLV_EINVAL, "apply: beta != 0 needs Y");
  Bf16Args a{};
  a.At = At;
  a.Bb = Bb;
  a.Vt = Vt;
  a.V = V;
  a.out = out;
  a.Y = beta != 0.0 ? Y : nullptr;
  a.alpha = alpha;
  a.beta = beta;
  a.n = n;
  a.s = s;
  a.p = p;
  a.nrb = row_blocks(n);
  a.nkb = k_blocks(n);
  a.ncb = col_blocks(s);
  {
    const int64_t total = (int64_t)p * a.ncb * a.nkb * 64;
    int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(tile_v_bf16_kernel, dim3(blocks), dim3(256), 0, st, V, Vt, n, s, p, a.ncb,
                       a.nkb);
    TSYLV_LAUNCH_CHECK();
  }
  launch_cfg<false>(a, variant, st);
}

void apply_bf16_tiled(const uint16_t* At, const uint16_t* Bb, const bf16t* V, bf16t* out,
                      double alpha, int64_t n, int64_t s, int p, hipStream_t st, int variant) {
  if (n <= 0 || s <= 0 || p <= 0) return;
  if (reinterpret_cast<const void*>(V) == reinterpret_cast<const void*>(out))
    throw Error(TSYLV_EINVAL, "apply: tiled output must not alias the input");
  Bf16Args a{};
  a.At = At;
  a.Bb = Bb;
  a.Vt = reinterpret_cast<const uint16_t*>(V);
  a.outt = reinterpret_cast<uint16_t*>(out);
  a.alpha = alpha;
  a.n = n;
  a.s = s;
  a.p = p;
  a.nrb = row_blocks(n);
  a.nkb = k_blocks(n);
  a.ncb = col_blocks(s);
  launch_cfg<true>(a, variant, st);
}

void tile_scale_bf16(const double* X, bf16t* Xt, double a, int64_t n, int64_t s, int p,
                     hipStream_t st) {
  if (n <= 0 || s <= 0 || p <= 0) return;
  const int64_t ncb = col_blocks(s), nkb = k_blocks(n);
  const int64_t total = (int64_t)p * ncb * nkb * 64;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(tile_scale_bf16_kernel, dim3(blocks), dim3(256), 0, st, X,
                     reinterpret_cast<uint16_t*>(Xt), a, n, s, p, ncb, nkb);
  TSYLV_LAUNCH_CHECK();
}

void untile_update_bf16(const bf16t* V, int64_t ldv, int nv, const double* y, double* X,
                        int64_t n, int64_t s, int p, hipStream_t st) {
  if (nv <= 0 || n <= 0 || s <= 0 || p <= 0) return;
  if (ldv % 8 != 0 || reinterpret_cast<uintptr_t>(V) % 16 != 0)
    throw Error(TSYLV_EINVAL, "untile_update: basis not aligned");
  const int64_t ncb = col_blocks(s), nkb = k_blocks(n);
  const int64_t total = (int64_t)p * ncb * nkb * 64;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(untile_update_bf16_kernel, dim3(blocks), dim3(256), 0, st,
                     reinterpret_cast<const uint16_t*>(V), ldv, nv, y, X, n, s, p, ncb, nkb);
  TSYLV_LAUNCH_CHECK();
}

}  // namespace kern
}  // namespace tsylv
