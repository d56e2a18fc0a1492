// Facewise Sylvester apply with BF16 Fourier slices (FP32 accumulation),
// HBM-bound path of the mixed-precision inner solves.
//
// W_k = Ahat_k V_k - V_k Bhat_k (Algorithm 1 step 2 for eq. (2)).  Both MFMA
// operands are stored in the lane order of v_mfma_f32_16x16x32_bf16, so every
// operand fragment is one coalesced 16-byte load per lane and no LDS or
// barrier is needed:
//   * the operator planes, rounded to BF16 once at setup: plane q, 16-row
//     block rb, 32-deep k block kb form one 1 KB chunk whose lane i + 16 g
//     holds A(16 rb + i, 32 kb + 8 g .. 8 g + 7);
//   * the Krylov vector, rounded to BF16 at the start of every apply into a
//     scratch buffer: plane q, 16-column block cb, k block kb form one chunk
//     whose lane i + 16 g holds V(32 kb + 8 g .. 8 g + 7, 16 cb + i).
// A wave owns R row blocks and CB column blocks of one slice and walks k with
// the next k block's fragments in flight.  The operator (the only large
// stream) is read once from HBM; a slice's V fragments (s n / 8 KB) are shared
// by all its waves through L2, which the XCD-contiguous tile order keeps on
// one XCD.  The small -V_k Bhat_k term is a short extra contraction over s.
#include "kernels.hpp"

namespace tsylv {
namespace kern {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;  // 4 waves, one 16-row block each

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
    const int64_t kb = chunk % nkb, rb = (chunk / nkb) % nrb, q = chunk / (nkb * nrb);
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

struct Bf16Args {
  const uint16_t* At;  // tiled operator planes (nrb x nkb chunks per plane)
  const uint16_t* Bb;  // bf16 planes of Bhat (s x s column-major), or null
  const uint16_t* Vt;  // tiled V planes (ncb x nkb chunks per plane)
  const float* V;
  float* out;
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

__device__ __forceinline__ bf8 ld8(const uint16_t* p) {
  return __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(p));
}

// One wave: row blocks rb0 .. rb0 + R - 1, column blocks cb0 .. cb0 + CB - 1
// of slice k.  All R row blocks and CB column blocks exist in the tiled
// buffers (zero padded), so the main loop has no conditions.
template <int CB, int R, int D, bool CPLX>
__device__ __forceinline__ void bf16_wave(const Bf16Args& a, int k, int64_t rb0, int64_t cb0) {
  int qr, qi;
  slice_planes(a.p, k, qr, qi);
  const int64_t n = a.n, s = a.s, ns = n * s, nkb = a.nkb;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lg = lane >> 4;
  const uint16_t* Ar[R];
  const uint16_t* Ai[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    Ar[r] = a.At + ((int64_t)qr * a.nrb + rb0 + r) * nkb * 512 + lane * 8;
    Ai[r] = CPLX ? a.At + ((int64_t)qi * a.nrb + rb0 + r) * nkb * 512 + lane * 8 : nullptr;
  }
  const uint16_t* Br[CB];
  const uint16_t* Bi[CB];
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    Br[j] = a.Vt + ((int64_t)qr * a.ncb + cb0 + j) * nkb * 512 + lane * 8;
    Bi[j] = CPLX ? a.Vt + ((int64_t)qi * a.ncb + cb0 + j) * nkb * 512 + lane * 8 : nullptr;
  }

  f4 accr[R][CB], acci[R][CB];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      accr[r][j] = f4{0.f, 0.f, 0.f, 0.f};
      acci[r][j] = f4{0.f, 0.f, 0.f, 0.f};
    }

  // Ring of D fragment sets: set u holds k block kb0 + u; after its MFMAs are
  // issued it is refilled with k block kb0 + u + D, so D k blocks of the
  // operator stream are in flight per wave.
  bf8 ar[D][R], ai[D][R], br[D][CB], bi[D][CB];
  auto load = [&](int64_t kb, int u) {
    const int64_t o = kb * 512;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      ar[u][r] = ld8(Ar[r] + o);
      if (CPLX) ai[u][r] = ld8(Ai[r] + o);
    }
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      br[u][j] = ld8(Br[j] + o);
      if (CPLX) bi[u][j] = ld8(Bi[j] + o);
    }
  };
#pragma unroll
  for (int u = 0; u < D; ++u)
    if (u < nkb) load(u, u);
  for (int64_t kb0 = 0; kb0 < nkb; kb0 += D) {
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int64_t kb = kb0 + u;
      if (kb < nkb) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          bf8 mai;
          if (CPLX) mai = neg8(ai[u][r]);
#pragma unroll
          for (int j = 0; j < CB; ++j) {
            accr[r][j] = mma(ar[u][r], br[u][j], accr[r][j]);
            if (CPLX) {
              acci[r][j] = mma(ar[u][r], bi[u][j], acci[r][j]);
              accr[r][j] = mma(mai, bi[u][j], accr[r][j]);
              acci[r][j] = mma(ai[u][r], br[u][j], acci[r][j]);
            }
          }
        }
        if (kb + D < nkb) load(kb + D, u);
      }
    }
  }

  const float* Vr = a.V + qr * ns;
  const float* Vi = CPLX ? a.V + qi * ns : nullptr;
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
          fr[e] = ok ? (uint16_t)(bf16_bits(Vr[row + n * kk]) ^ 0x8000u) : (uint16_t)0;
          if (CPLX) fi[e] = ok ? (uint16_t)(bf16_bits(Vi[row + n * kk]) ^ 0x8000u) : (uint16_t)0;
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

// Workgroup = 4 independent waves on consecutive row groups of one slice.
template <int CB, int R, int D>
__global__ __launch_bounds__(NT) void apply_bf16_kernel(Bf16Args a) {
  const int t = xcd_tile(blockIdx.x, a.total);
  const int ct = t % a.nct;
  const int rt = (t / a.nct) % a.nrt;
  const int k = t / (a.nct * a.nrt);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t rb0 = ((int64_t)rt * (NT / 64) + wave) * R;
  if (rb0 >= (a.n + 15) / 16) return;  // whole wave past the last row
  const int64_t cb0 = (int64_t)ct * CB;
  if ((k == 0) || (2 * k == a.p))
    bf16_wave<CB, R, D, false>(a, k, rb0, cb0);
  else
    bf16_wave<CB, R, D, true>(a, k, rb0, cb0);
}

// Row blocks are padded to a multiple of kRowPad (the largest 4 R) and
// column blocks to a multiple of kColPad (the largest CB).
constexpr int64_t kRowPad = 16, kColPad = 4;

template <int CB, int R, int D>
void launch(Bf16Args a, hipStream_t st) {
  a.nrt = (int)(((a.n + 15) / 16 + 4 * R - 1) / (4 * R));
  a.nct = (int)((a.s + 16 * CB - 1) / (16 * CB));
  a.total = num_slices(a.p) * a.nrt * a.nct;
  hipLaunchKernelGGL((apply_bf16_kernel<CB, R, D>), dim3(a.total), dim3(NT), 0, st, a);
  TSYLV_LAUNCH_CHECK();
}

}  // namespace

static int64_t row_blocks(int64_t n) { return ((n + 15) / 16 + kRowPad - 1) / kRowPad * kRowPad; }
static int64_t col_blocks(int64_t s) { return ((s + 15) / 16 + kColPad - 1) / kColPad * kColPad; }

int64_t bf16_tiled_elems(int64_t n, int p) {
  return (int64_t)p * row_blocks(n) * ((n + 31) / 32) * 512;
}

int64_t bf16_vtiled_elems(int64_t n, int64_t s, int p) {
  return (int64_t)p * col_blocks(s) * ((n + 31) / 32) * 512;
}

void tile_operator_bf16(const double* Ah, uint16_t* At, int64_t n, int p, hipStream_t st) {
  const int64_t nrb = row_blocks(n), nkb = (n + 31) / 32;
  const int64_t total = (int64_t)p * nrb * nkb * 64;
  int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(tile_bf16_kernel, dim3(blocks), dim3(256), 0, st, Ah, At, n, p, nrb, nkb);
  TSYLV_LAUNCH_CHECK();
}

void apply_bf16(const uint16_t* At, const uint16_t* Bb, const float* V, uint16_t* Vt,
                float* out, const float* Y, double alpha, double beta, int64_t n, int64_t s,
                int p, hipStream_t st) {
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
  a.nkb = (n + 31) / 32;
  a.ncb = col_blocks(s);
  {
    const int64_t total = (int64_t)p * a.ncb * a.nkb * 64;
    int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(tile_v_bf16_kernel, dim3(blocks), dim3(256), 0, st, V, Vt, n, s, p, a.ncb,
                       a.nkb);
    TSYLV_LAUNCH_CHECK();
  }
  // (column blocks, row blocks, ring depth) per wave, from a sweep at
  // n = 4096, p = 32 and n = 8192, p = 64
  if (s <= 16)
    launch<1, 1, 2>(a, st);
  else if (s <= 32)
    launch<2, 2, 4>(a, st);
  else
    launch<4, 2, 3>(a, st);
}

}  // namespace kern
}  // namespace tsylv
