// Facewise Sylvester apply with BF16 Fourier slices (FP32 accumulation),
// HBM-bound path of the mixed-precision inner solves.
//
// W_k = Ahat_k V_k - V_k Bhat_k (Algorithm 1 step 2 for eq. (2)) with the
// operator planes rounded to BF16 once at setup and stored pre-tiled in the
// lane order of v_mfma_f32_16x16x32_bf16: plane q, 16-row block rb, 32-deep
// k block kb form one 1 KB chunk whose lane i + 16 g holds the 8 values
// A(16 rb + i, 32 kb + 8 g .. 8 g + 7).  Each wave therefore loads its A
// operand straight from HBM with one coalesced 16-byte load per lane per
// MFMA -- the operator, the only large stream, never goes through LDS --
// while the V_k panels, shared by the 4 waves of a workgroup, are staged
// through LDS in BF16 with k contiguous so a lane's B operand is one 16-byte
// LDS read.  The small -V_k Bhat_k term is a short extra contraction over s
// read directly from global memory.  Tiles are handed out XCD-contiguously
// as in the FP64 kernel.
#include "kernels.hpp"

namespace tsylv {
namespace kern {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;  // 4 waves, one 16-row block each
constexpr int TK = 64;   // k panel staged in LDS (two MFMA k blocks)
constexpr int KP = TK + 8;  // padded LDS row (bf16 elements)

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

struct Bf16Args {
  const uint16_t* At;  // tiled operator planes
  const uint16_t* Bb;  // bf16 planes of Bhat (s x s column-major), or null
  const float* V;
  float* out;
  const float* Y;
  double alpha, beta;
  int64_t n, s;
  int p;
  int64_t nrb, nkb;
  int nrt, nct, total;
};

__device__ __forceinline__ int xcd_tile(int b, int total) {
  const int q = total / 8, r = total % 8;
  const int x = b % 8;
  return x * q + (x < r ? x : r) + b / 8;
}

template <int CB, bool CPLX>
__device__ __forceinline__ void bf16_tile(const Bf16Args& a, int k, int rt, int ct,
                                          uint16_t (*Bs)[16 * CB][KP]) {
  constexpr int TN = 16 * CB;
  constexpr int NB = TK * TN / NT;  // V panel elements per thread and plane
  int qr, qi;
  slice_planes(a.p, k, qr, qi);
  const int64_t n = a.n, s = a.s, ns = n * s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t rb = (int64_t)rt * 4 + wave;  // this wave's 16-row block
  const int64_t c0 = (int64_t)ct * TN;
  const float* Vr = a.V + qr * ns;
  const float* Vi = CPLX ? a.V + qi * ns : nullptr;
  const int64_t chunks_per_plane = a.nrb * a.nkb;
  const uint16_t* Atr = a.At + ((int64_t)qr * chunks_per_plane + rb * a.nkb) * 512 + lane * 8;
  const uint16_t* Ati =
      CPLX ? a.At + ((int64_t)qi * chunks_per_plane + rb * a.nkb) * 512 + lane * 8 : nullptr;
  const bool row_ok = rb < a.nrb;

  f4 accr[CB], acci[CB];
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    accr[j] = f4{0.f, 0.f, 0.f, 0.f};
    acci[j] = f4{0.f, 0.f, 0.f, 0.f};
  }

  float pv_r[NB], pv_i[NB];
  auto load_v = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = tid + NT * u;
      const int kk = idx % TK, col = idx / TK;
      const int64_t gk = k0 + kk, gc = c0 + col;
      const bool ok = gk < n && gc < s;
      pv_r[u] = ok ? Vr[gk + n * gc] : 0.f;
      if (CPLX) pv_i[u] = ok ? Vi[gk + n * gc] : 0.f;
    }
  };
  auto store_v = [&]() {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = tid + NT * u;
      const int kk = idx % TK, col = idx / TK;
      Bs[0][col][kk] = bf16_bits(pv_r[u]);
      if (CPLX) Bs[1][col][kk] = bf16_bits(pv_i[u]);
    }
  };
  auto load_a = [&](const uint16_t* base, int64_t kb) -> bf8 {
    if (!row_ok || kb >= a.nkb) return __builtin_bit_cast(bf8, u16x8{0, 0, 0, 0, 0, 0, 0, 0});
    return __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(base + kb * 512));
  };

  bf8 ar[2], ai[2];
  load_v(0);
  ar[0] = load_a(Atr, 0);
  ar[1] = load_a(Atr, 1);
  if (CPLX) {
    ai[0] = load_a(Ati, 0);
    ai[1] = load_a(Ati, 1);
  }
  for (int64_t k0 = 0; k0 < n; k0 += TK) {
    store_v();
    __syncthreads();
    const bool more = k0 + TK < n;
    if (more) load_v(k0 + TK);
    bf8 nar[2], nai[2];
    if (more) {
      nar[0] = load_a(Atr, k0 / 32 + 2);
      nar[1] = load_a(Atr, k0 / 32 + 3);
      if (CPLX) {
        nai[0] = load_a(Ati, k0 / 32 + 2);
        nai[1] = load_a(Ati, k0 / 32 + 3);
      }
    }
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      const bf8 anr = ar[kc];
      bf8 ani;
      if (CPLX) ani = neg8(ai[kc]);
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        const int col = j * 16 + li;
        const bf8 br = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&Bs[0][col][kc * 32 + 8 * lg]));
        accr[j] = mma(anr, br, accr[j]);
        if (CPLX) {
          const bf8 bi = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&Bs[1][col][kc * 32 + 8 * lg]));
          acci[j] = mma(anr, bi, acci[j]);
          accr[j] = mma(ani, bi, accr[j]);
          acci[j] = mma(ai[kc], br, acci[j]);
        }
      }
    }
    if (more) {
      ar[0] = nar[0];
      ar[1] = nar[1];
      if (CPLX) {
        ai[0] = nai[0];
        ai[1] = nai[1];
      }
    }
    __syncthreads();
  }

  // -V_k Bhat_k: a short contraction over s straight from global memory.
  const int64_t row = 16 * rb + li;
  if (a.Bb) {
    const uint16_t* Br = a.Bb + qr * s * s;
    const uint16_t* Bi = CPLX ? a.Bb + qi * s * s : nullptr;
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
        const int64_t col = c0 + j * 16 + li;
        u16x8 gr, gi;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t kk = k1 + 8 * lg + e;
          const bool ok = col < s && kk < s;
          gr[e] = ok ? Br[kk + s * col] : (uint16_t)0;
          if (CPLX) gi[e] = ok ? Bi[kk + s * col] : (uint16_t)0;
        }
        const bf8 br = __builtin_bit_cast(bf8, gr);
        accr[j] = mma(nvr, br, accr[j]);  // -Vr Br
        if (CPLX) {
          const bf8 bi = __builtin_bit_cast(bf8, gi);
          acci[j] = mma(nvr, bi, acci[j]);  // -Vr Bi
          accr[j] = mma(pvi, bi, accr[j]);  // +Vi Bi
          acci[j] = mma(nvi, br, acci[j]);  // -Vi Br
        }
      }
    }
  }

  // Epilogue (FP32 result layout: element (i, j) in lane j + 16 (i / 4), register i % 4).
  float* Or = a.out + qr * ns;
  float* Oi = CPLX ? a.out + qi * ns : nullptr;
  const float* Yr = a.Y ? a.Y + qr * ns : nullptr;
  const float* Yi = (a.Y && CPLX) ? a.Y + qi * ns : nullptr;
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int64_t col = c0 + j * 16 + li;
    if (col >= s) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rr = 16 * rb + 4 * lg + r;
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

template <int CB>
__global__ __launch_bounds__(NT) void apply_bf16_tiled_kernel(Bf16Args a) {
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][16 * CB][KP];
  const int t = xcd_tile(blockIdx.x, a.total);
  const int ct = t % a.nct;
  const int rt = (t / a.nct) % a.nrt;
  const int k = t / (a.nct * a.nrt);
  if ((k == 0) || (2 * k == a.p))
    bf16_tile<CB, false>(a, k, rt, ct, Bs);
  else
    bf16_tile<CB, true>(a, k, rt, ct, Bs);
}

template <int CB>
void launch(Bf16Args a, hipStream_t st) {
  a.nrt = (int)((a.n + 63) / 64);
  a.nct = (int)((a.s + 16 * CB - 1) / (16 * CB));
  a.total = num_slices(a.p) * a.nrt * a.nct;
  hipLaunchKernelGGL(apply_bf16_tiled_kernel<CB>, dim3(a.total), dim3(NT), 0, st, a);
  TSYLV_LAUNCH_CHECK();
}

}  // namespace

int64_t bf16_tiled_elems(int64_t n, int p) {
  const int64_t nrb = (n + 15) / 16, nkb = (n + 31) / 32;
  return (int64_t)p * nrb * nkb * 512;
}

void tile_operator_bf16(const double* Ah, uint16_t* At, int64_t n, int p, hipStream_t st) {
  const int64_t nrb = (n + 15) / 16, nkb = (n + 31) / 32;
  const int64_t total = (int64_t)p * nrb * nkb * 64;
  int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(tile_bf16_kernel, dim3(blocks), dim3(256), 0, st, Ah, At, n, p, nrb, nkb);
  TSYLV_LAUNCH_CHECK();
}

void apply_bf16(const uint16_t* At, const uint16_t* Bb, const float* V, float* out,
                const float* Y, double alpha, double beta, int64_t n, int64_t s, int p,
                hipStream_t st) {
  if (n <= 0 || s <= 0 || p <= 0) return;
  if (beta != 0.0 && Y == nullptr) throw Error(TSYLV_EINVAL, "apply: beta != 0 needs Y");
  Bf16Args a{};
  a.At = At;
  a.Bb = Bb;
  a.V = V;
  a.out = out;
  a.Y = beta != 0.0 ? Y : nullptr;
  a.alpha = alpha;
  a.beta = beta;
  a.n = n;
  a.s = s;
  a.p = p;
  a.nrb = (n + 15) / 16;
  a.nkb = (n + 31) / 32;
  if (s <= 16)
    launch<1>(a, st);
  else if (s <= 32)
    launch<2>(a, st);
  else
    launch<4>(a, st);
}

}  // namespace kern
}  // namespace tsylv
