// Tube transforms, conversions and the multi-vector (Gram-Schmidt) kernels.
//
// Tube transform: the mode-3 DFT of section 2.1 (fft(A, [], 3)) restricted
// to the conjugate-symmetric half, written as one p x p real matrix applied
// to every tube.  One thread owns one tube: the p values of a tube are
// strided by the slice size E in memory, so a wavefront reads p coalesced
// rows and keeps the whole tube in registers.
//
// Multi-vector kernels: the scalar inner products and updates of tArnoldi
// (Algorithm 2, step 3(b)) on vectors kept in the orthonormal Fourier
// representation, where the inner product of section 2.1 is the plain dot
// product of the stored reals.  Reductions are two-stage and fixed-order
// (wave shuffles, then LDS, then one block per output), so results do not
// depend on timing.
#include "kernels.hpp"

#include <hip/hip_bf16.h>

#include "philox.hpp"

namespace tsylv {
namespace kern {

namespace {

constexpr int kBlock = 256;

// ------------------------------------------------------------------ xform

__global__ void build_xform_kernel(double* M, int p, int kind) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= p * p) return;
  // Row q (plane) and column j (spatial slice) of the forward matrix.
  int q, j;
  if (kind == XF_INVERSE) {
    j = t / p;
    q = t % p;
  } else {
    q = t / p;
    j = t % p;
  }
  int k, part;  // slice and 0 = real part / 1 = imaginary part
  if (q == 0) {
    k = 0;
    part = 0;
  } else if ((p % 2 == 0) && q == p - 1) {
    k = p / 2;
    part = 0;
  } else {
    k = (q + 1) / 2;
    part = (q % 2 == 1) ? 0 : 1;
  }
  int r = (int)(((long long)j * k) % p);
  double c, s;
  if ((4 * r) % p == 0) {
    int quarter = (4 * r) / p;  // angle = quarter * pi/2
    const double cs[4] = {1.0, 0.0, -1.0, 0.0};
    const double sn[4] = {0.0, 1.0, 0.0, -1.0};
    c = cs[quarter];
    s = sn[quarter];
  } else {
    sincospi(2.0 * r / p, &s, &c);
  }
  // DFT kernel exp(-i theta) = cos(theta) - i sin(theta).
  double v = (part == 0) ? c : -s;
  if (kind != XF_OPERATOR) {
    bool real_slice = (k == 0) || (2 * k == p);
    v *= sqrt((real_slice ? 1.0 : 2.0) / p);
  }
  M[t] = v;
}

template <int PMAX>
__device__ __forceinline__ void stage_xform(double* Ms, const double* __restrict__ M, int p) {
  for (int t = threadIdx.x; t < PMAX * PMAX; t += kBlock) {
    int q = t / PMAX, j = t % PMAX;
    Ms[t] = (q < p && j < p) ? M[q * p + j] : 0.0;
  }
  __syncthreads();
}

// out[q E + e] for every q from the tube v (zero past p): one fixed fma
// order, shared by the transforms of stored and of generated tubes.
template <int PMAX>
__device__ __forceinline__ void xform_store(const double* Ms, const double (&v)[PMAX],
                                            double* __restrict__ out, int64_t E, int64_t e,
                                            int p) {
  for (int q = 0; q < p; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < PMAX; ++j) acc = fma(Ms[q * PMAX + j], v[j], acc);
    out[(int64_t)q * E + e] = acc;
  }
}

template <int PMAX>
__global__ __launch_bounds__(kBlock) void tube_xform_kernel(
    const double* __restrict__ in, double* __restrict__ out,
    const double* __restrict__ M, int64_t E, int p) {
  __shared__ double Ms[PMAX * PMAX];
  stage_xform<PMAX>(Ms, M, p);
  int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= E) return;
  double v[PMAX];
#pragma unroll
  for (int j = 0; j < PMAX; ++j) v[j] = (j < p) ? in[(int64_t)j * E + e] : 0.0;
  xform_store<PMAX>(Ms, v, out, E, e, p);
}

// The transform of a generated tensor: each thread draws its tube from the
// counter-based stream in registers, so the spatial tensor is never stored.
template <int PMAX>
__global__ __launch_bounds__(kBlock) void tube_xform_gen_kernel(
    GenTensor g, double* __restrict__ out, const double* __restrict__ M, int64_t E, int p) {
  __shared__ double Ms[PMAX * PMAX];
  stage_xform<PMAX>(Ms, M, p);
  int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= E) return;
  double v[PMAX];
#pragma unroll
  for (int kb = 0; kb < PMAX / 4; ++kb) {
    double x[4] = {0.0, 0.0, 0.0, 0.0};
    if (4 * kb < p) gen_block4(g, e, kb, x);
#pragma unroll
    for (int q = 0; q < 4; ++q) v[4 * kb + q] = (4 * kb + q < p) ? x[q] : 0.0;
  }
  xform_store<PMAX>(Ms, v, out, E, e, p);
}

// The spatial tensor itself: one thread per position e, its tube written
// four slices at a time (each store row coalesced across the wavefront).
__global__ __launch_bounds__(kBlock) void gen_tensor_kernel(GenTensor g, double* __restrict__ out,
                                                            int64_t E, int p) {
  const int64_t nkb = (p + 3) / 4;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < E;
       e += (int64_t)gridDim.x * kBlock) {
    for (int64_t kb = 0; kb < nkb; ++kb) {
      double x[4];
      gen_block4(g, e, kb, x);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (4 * kb + q < p) out[(4 * kb + q) * E + e] = x[q];
    }
  }
}

// Any p: matrix from global memory (cached), tube re-read per output.
__global__ __launch_bounds__(kBlock) void tube_xform_generic_kernel(
    const double* __restrict__ in, double* __restrict__ out,
    const double* __restrict__ M, int64_t E, int p) {
  int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= E) return;
  for (int q = 0; q < p; ++q) {
    double acc = 0.0;
    for (int j = 0; j < p; ++j) acc = fma(M[q * p + j], in[(int64_t)j * E + e], acc);
    out[(int64_t)q * E + e] = acc;
  }
}

// ------------------------------------------------------------- conversion

__global__ void f64_to_f32_kernel(const double* __restrict__ in, float* __restrict__ out,
                                  int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];  // IEEE round to nearest even
}

__global__ void f32_to_f64_kernel(const float* __restrict__ in, double* __restrict__ out,
                                  int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}

// Round a double to bfloat16, nearest even, via float (exact for the
// rounding of the mantissa: the double->float step is itself RNE and then
// the float->bf16 step rounds the remaining bits; double rounding can only
// matter at exact float ties, which we resolve on the double directly).
__device__ inline uint16_t f64_to_bf16_bits(double x) {
  float f = (float)x;
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) {  // inf / nan
    return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  }
  uint32_t lower = u & 0xffffu;
  uint32_t up = u >> 16;
  if (lower > 0x8000u) {
    up += 1;
  } else if (lower == 0x8000u) {
    // exact tie in float: decide with the double value
    double trunc = (double)__uint_as_float(up << 16);
    double next = (double)__uint_as_float((up + 1) << 16);
    double dt = fabs(x - trunc), dn = fabs(next - x);
    if (dn < dt || (dn == dt && (up & 1u))) up += 1;
  }
  return (uint16_t)up;
}

__global__ void f64_to_bf16_kernel(const double* __restrict__ in, uint16_t* __restrict__ out,
                                   int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = f64_to_bf16_bits(in[i]);
}

// Pseudo-random operands for timing (the autotuner): value i is a uniform
// number in [-1, 1) from the splitmix64 finaliser of seed + i, stored as
// FP64, FP32 or BF16 (elem = 8, 4, 2 bytes).
__global__ void fill_random_kernel(void* __restrict__ buf, int64_t count, int elem,
                                   uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    if (elem == 8)
      static_cast<double*>(buf)[i] = u;
    else if (elem == 4)
      static_cast<float*>(buf)[i] = (float)u;
    else
      static_cast<uint16_t*>(buf)[i] = f64_to_bf16_bits(u);
  }
}

// ------------------------------------------------------------ multi-vector

constexpr int kChunk = 4096;  // elements per mdot chunk
constexpr int kEPT = kChunk / kBlock;
constexpr int kVG = 8;  // vectors per mdot block

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// grid: (nchunks, ceil((nv + with_ww) / kVG)).  Vectors of type T, sums in FP64.
template <typename T>
__global__ __launch_bounds__(kBlock) void mdot_kernel(
    const T* __restrict__ V, int64_t ldv, int nv, const T* __restrict__ w,
    int64_t N, double* __restrict__ part, int ldp, int with_ww) {
  const int ncols = nv + with_ww;
  const int g0 = blockIdx.y * kVG;
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  double acc[kVG];
#pragma unroll
  for (int v = 0; v < kVG; ++v) acc[v] = 0.0;
  for (int t = 0; t < kEPT; ++t) {
    int64_t e = base + t * kBlock + threadIdx.x;
    if (e < N) {
      double we = (double)w[e];
#pragma unroll
      for (int v = 0; v < kVG; ++v) {
        int i = g0 + v;
        if (i < nv) acc[v] = fma((double)V[(int64_t)i * ldv + e], we, acc[v]);
        else if (i == nv && with_ww) acc[v] = fma(we, we, acc[v]);
      }
    }
  }
  __shared__ double red[kBlock / 64][kVG];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < kVG; ++v) {
    double r = wave_sum(acc[v]);
    if (lane == 0) red[wid][v] = r;
  }
  __syncthreads();
  if (threadIdx.x < kVG) {
    int i = g0 + threadIdx.x;
    if (i < ncols) {
      double r = 0.0;
      for (int q = 0; q < kBlock / 64; ++q) r += red[q][threadIdx.x];
      part[(int64_t)blockIdx.x * ldp + i] = r;
    }
  }
}

// grid: ncols blocks
__global__ __launch_bounds__(kBlock) void reduce_partials_kernel(
    const double* __restrict__ part, int nchunks, int ldp, double* __restrict__ out) {
  const int col = blockIdx.x;
  double r = 0.0;
  for (int c = threadIdx.x; c < nchunks; c += kBlock) r += part[(int64_t)c * ldp + col];
  __shared__ double red[kBlock / 64];
  r = wave_sum(r);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) t += red[q];
    out[col] = t;
  }
}

constexpr int kMaxUpd = 1024;

// w[e] -= sum_i h[i] V_i[e]; basis of type TB, target of type TW, FP64 arithmetic.
template <typename TB, typename TW>
__global__ __launch_bounds__(kBlock) void mupdate_kernel(
    const TB* __restrict__ V, int64_t ldv, int nv, const double* __restrict__ h,
    TW* __restrict__ w, int64_t N) {
  __shared__ double hs[kMaxUpd];
  for (int i = threadIdx.x; i < nv; i += kBlock) hs[i] = h[i];
  __syncthreads();
  int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= N) return;
  double acc = (double)w[e];
  for (int i = 0; i < nv; ++i) acc = fma(-hs[i], (double)V[(int64_t)i * ldv + e], acc);
  w[e] = (TW)acc;
}

template <typename TI, typename TO>
__global__ void scale_kernel(const TI* __restrict__ x, TO* __restrict__ out, double a, int64_t N) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (TO)(a * (double)x[i]);
}

// ---- fused CGS2 passes over a lazily normalised basis ----------------
// The basis vectors V_i are stored unnormalised; sigma[i] = 1 / ||V_i|| makes
// sigma_i V_i orthonormal.  Every wave works on its own tiles of 16 x EPL
// contiguous elements; within a tile the 64 lanes form 4 groups of 16, and
// group g holds vectors g, g + 4, g + 8, ... (VPW of them), EPL contiguous
// elements of each per lane.  The update w -= sum c_i V_i is summed over the
// groups with two lane shuffles, so waves never wait on each other; a block
// owns kOChunk elements and combines its four waves' partial sums once, at
// the end.  All sums run in FP64 in a fixed order.

constexpr int kOWaves = kBlock / 64;
constexpr int kOGroups = 4;  // vector groups per wave
constexpr int kOChunk = 8192;

// Device view of kern::bf16t: widens exactly to FP64, and is built from an
// FP64 value by rounding to FP32 and then to the nearest-even BF16.
struct OB16 {
  uint16_t bits;
  OB16() = default;
  __device__ explicit OB16(double x) {
    uint32_t u = __float_as_uint((float)x);
    if ((u & 0x7f800000u) == 0x7f800000u) {
      bits = (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));  // inf stays inf, NaN quiet
    } else {
      u += 0x7fffu + ((u >> 16) & 1u);
      bits = (uint16_t)(u >> 16);
    }
  }
  __device__ operator double() const { return (double)__uint_as_float((uint32_t)bits << 16); }
};
static_assert(sizeof(OB16) == sizeof(bf16t), "OB16 is a view of bf16t");
struct alignas(8) OB16x4 {
  OB16 e[4];
};
struct alignas(16) OB16x8 {
  OB16 e[8];
};

// Keeps a loaded value in its register until here (an empty asm the
// compiler cannot see through).
template <typename T>
__device__ __forceinline__ void opin(T& x) {
  asm volatile("" : "+v"(x));
}
template <>
__device__ __forceinline__ void opin(OB16& x) {
  asm volatile("" : "+v"(x.bits));
}

template <typename T, int EPL>
struct OVec;
template <>
struct OVec<OB16, 4> {
  using type = OB16x4;
};
template <>
struct OVec<OB16, 8> {
  using type = OB16x8;
};
template <>
struct OVec<float, 2> {
  using type = float2;
};
template <>
struct OVec<float, 4> {
  using type = float4;
};
template <>
struct OVec<double, 1> {
  using type = double;
};
template <>
struct OVec<double, 2> {
  using type = double2;
};

// Sum over the 16 lanes of a group (fixed xor tree).
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sums of acc[k] into columns cols[k] (< 0 skips k) of `ncols`, the
// columns this lane's group owns; column c's sum r goes to out[pos(c)]
// (skipped when pos(c) < 0) as put(c, r).  One barrier.
template <int NA, typename Pos, typename Put>
__device__ __forceinline__ void oblock_reduce(const double (&acc)[NA], const int (&cols)[NA],
                                              int ncols, Pos pos, Put put,
                                              double* __restrict__ out) {
  constexpr int MAXC = NA * kOGroups;
  __shared__ double red[kOWaves][MAXC];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    const double r = group_sum(acc[k]);
    if ((lane & 15) == 0 && cols[k] >= 0) red[wid][cols[k]] = r;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < ncols; c += kBlock) {
    double r = red[0][c];
#pragma unroll
    for (int q = 1; q < kOWaves; ++q) r += red[q][c];
    const int at = pos(c);
    if (at >= 0) out[at] = put(c, r);
  }
}

// out[col(k)] = sum over the block of acc[k] (times scale[col] if given).
template <int NA>
__device__ __forceinline__ void oblock_store(const double (&acc)[NA], const int (&cols)[NA],
                                             int ncols, const double* __restrict__ scale,
                                             double* __restrict__ out) {
  oblock_reduce<NA>(
      acc, cols, ncols, [](int c) { return c; },
      [scale](int c, double r) { return scale ? r * scale[c] : r; }, out);
}

// Loads this lane's EPL elements of its group's VPW vectors for the tile at
// `off`.  FULL (the whole tile lies below `lim`, a wave-uniform test): every
// load is issued unconditionally so that all are in flight together; slots
// past nv read vector nv - 1 again (cache lines another lane group of the
// wave loads at the same time) and are neutralised by the callers (zero
// coefficient, zero weight).  Otherwise each element is guarded and the
// slots past nv are zero.
template <bool FULL, typename T, int VPW, int EPL>
__device__ __forceinline__ void oload_tile(const T* __restrict__ V, int64_t ldv, int nv, int g,
                                           const T* __restrict__ w, int64_t off, int64_t lim,
                                           T (&v)[VPW][EPL]) {
  using VT = typename OVec<T, EPL>::type;
#pragma unroll
  for (int k = 0; k < VPW; ++k) {
    const int i = g + kOGroups * k;
    if (FULL) {
      const T* src = V + (int64_t)min(i, nv - 1) * ldv;
      const VT t = *reinterpret_cast<const VT*>(src + off);
      const T* tp = reinterpret_cast<const T*>(&t);
#pragma unroll
      for (int l = 0; l < EPL; ++l) v[k][l] = tp[l];
    } else {
#pragma unroll
      for (int l = 0; l < EPL; ++l)
        v[k][l] = (i < nv && off + l < lim) ? V[(int64_t)i * ldv + off + l] : (T)0;
    }
  }
}

template <bool FULL, typename T, int EPL>
__device__ __forceinline__ void oload_w(const T* __restrict__ w, int64_t off, int64_t lim,
                                        T (&v)[EPL]) {
  using VT = typename OVec<T, EPL>::type;
  if (FULL) {
    const VT t = *reinterpret_cast<const VT*>(w + off);
    const T* tp = reinterpret_cast<const T*>(&t);
#pragma unroll
    for (int l = 0; l < EPL; ++l) v[l] = tp[l];
  } else {
#pragma unroll
    for (int l = 0; l < EPL; ++l) v[l] = (off + l < lim) ? w[off + l] : (T)0;
  }
}

template <bool FULL, typename T, int VPW, int EPL>
__device__ __forceinline__ void odots_tile(const T* __restrict__ V, int64_t ldv, int nv, int g,
                                           const T* __restrict__ w, int64_t off, int64_t lim,
                                           double (&acc)[VPW], double& ww) {
  T wv[EPL];
  oload_w<FULL, T, EPL>(w, off, lim, wv);
  T v[VPW][EPL];
  oload_tile<FULL, T, VPW, EPL>(V, ldv, nv, g, w, off, lim, v);
#pragma unroll
  for (int k = 0; k < VPW; ++k)
#pragma unroll
    for (int l = 0; l < EPL; ++l) acc[k] = fma((double)v[k][l], (double)wv[l], acc[k]);
#pragma unroll
  for (int l = 0; l < EPL; ++l) ww = fma((double)wv[l], (double)wv[l], ww);
}

// part[c][i] = sigma_i sum_e V_i[e] w[e] (i < nv), part[c][nv] = sum_e w[e]^2
// over chunk c.
template <typename T, int VPW, int EPL>
__global__ __launch_bounds__(kBlock) void ortho_dots_kernel(
    const T* __restrict__ V, int64_t ldv, int nv, const double* __restrict__ sigma,
    const T* __restrict__ w, int64_t N, double* __restrict__ part, int ldp) {
  constexpr int TE = 16 * EPL;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int g = lane >> 4;
  double acc[VPW], ww = 0.0;
#pragma unroll
  for (int k = 0; k < VPW; ++k) acc[k] = 0.0;
  const int64_t base = (int64_t)blockIdx.x * kOChunk;
  const int64_t end = min(N, base + kOChunk);
  for (int64_t t0 = base + wid * TE; t0 < end; t0 += kOWaves * TE) {
    const int64_t off = t0 + (lane & 15) * EPL;
    if (t0 + TE <= end)
      odots_tile<true, T, VPW, EPL>(V, ldv, nv, g, w, off, end, acc, ww);
    else
      odots_tile<false, T, VPW, EPL>(V, ldv, nv, g, w, off, end, acc, ww);
  }
  double* out = part + (int64_t)blockIdx.x * ldp;
  double all[VPW + 1];
  int cols[VPW + 1];
#pragma unroll
  for (int k = 0; k < VPW; ++k) {
    const int i = g + kOGroups * k;
    // unconditional product: a select on acc would let the compiler drop
    // (and branch around) the loads of the unused slots
    all[k] = acc[k] * ((i < nv) ? sigma[i] : 0.0);
    cols[k] = (i < nv) ? i : -1;
  }
  all[VPW] = ww;  // every group saw the same w; group 0 reports it
  cols[VPW] = (g == 0) ? nv : -1;
  oblock_store<VPW + 1>(all, cols, nv + 1, nullptr, out);
}

template <bool FULL, typename T, int VPW, int EPL>
__device__ __forceinline__ void oupdate_tile(const T* __restrict__ V, int64_t ldv, int nv, int g,
                                             const double (&cs)[VPW], T* __restrict__ w,
                                             int64_t off, int64_t lim, int mode,
                                             double (&acc)[VPW], double& ww) {
  T v[VPW][EPL];
  oload_tile<FULL, T, VPW, EPL>(V, ldv, nv, g, w, off, lim, v);
  double x[EPL];
  {
    T wv[EPL];
    oload_w<FULL, T, EPL>(w, off, lim, wv);
#pragma unroll
    for (int l = 0; l < EPL; ++l) x[l] = (g == 0) ? (double)wv[l] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < VPW; ++k)
#pragma unroll
    for (int l = 0; l < EPL; ++l) x[l] = fma(-cs[k], (double)v[k][l], x[l]);
  T xt[EPL];
#pragma unroll
  for (int l = 0; l < EPL; ++l) {
    // (p0 + p1) + (p2 + p3) in every group: the same bits in all four
    double y = x[l] + __shfl_xor(x[l], 16, 64);
    y += __shfl_xor(y, 32, 64);
    xt[l] = (T)y;
  }
  if (g == 0) {
    if (FULL) {
      using VT = typename OVec<T, EPL>::type;
      VT t;
      T* tp = reinterpret_cast<T*>(&t);
#pragma unroll
      for (int l = 0; l < EPL; ++l) tp[l] = xt[l];
      *reinterpret_cast<VT*>(w + off) = t;
    } else {
#pragma unroll
      for (int l = 0; l < EPL; ++l)
        if (off + l < lim) w[off + l] = xt[l];
    }
  }
  if (mode == 0) {
    // Widen the basis values again here rather than keeping the widened
    // copies from the update live (FP32: half the registers).
#pragma unroll
    for (int k = 0; k < VPW; ++k)
#pragma unroll
      for (int l = 0; l < EPL; ++l) opin(v[k][l]);
#pragma unroll
    for (int k = 0; k < VPW; ++k)
#pragma unroll
      for (int l = 0; l < EPL; ++l) acc[k] = fma((double)v[k][l], (double)xt[l], acc[k]);
  } else {
#pragma unroll
    for (int l = 0; l < EPL; ++l) ww = fma((double)xt[l], (double)xt[l], ww);
  }
}

// w -= sum_i h[i] sigma[i] V_i; then (mode 0) part[c][i] = sigma_i V_i . w for
// the next CGS pass, or (mode 1) part[c][0] = ||w||^2.
template <typename T, int VPW, int EPL>
__global__ __launch_bounds__(kBlock) void ortho_update_kernel(
    const T* __restrict__ V, int64_t ldv, int nv, const double* __restrict__ h,
    const double* __restrict__ sigma, T* __restrict__ w, int64_t N, double* __restrict__ part,
    int ldp, int mode) {
  constexpr int TE = 16 * EPL;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int g = lane >> 4;
  double cs[VPW], acc[VPW];
#pragma unroll
  for (int k = 0; k < VPW; ++k) {
    const int i = g + kOGroups * k;
    cs[k] = (i < nv) ? h[i] * sigma[i] : 0.0;
    acc[k] = 0.0;
  }
  double ww = 0.0;
  const int64_t base = (int64_t)blockIdx.x * kOChunk;
  const int64_t end = min(N, base + kOChunk);
  for (int64_t t0 = base + wid * TE; t0 < end; t0 += kOWaves * TE) {
    const int64_t off = t0 + (lane & 15) * EPL;
    if (t0 + TE <= end)
      oupdate_tile<true, T, VPW, EPL>(V, ldv, nv, g, cs, w, off, end, mode, acc, ww);
    else
      oupdate_tile<false, T, VPW, EPL>(V, ldv, nv, g, cs, w, off, end, mode, acc, ww);
  }
  double* out = part + (int64_t)blockIdx.x * ldp;
  if (mode == 0) {
    double all[VPW];
    int cols[VPW];
#pragma unroll
    for (int k = 0; k < VPW; ++k) {
      const int i = g + kOGroups * k;
      all[k] = acc[k] * ((i < nv) ? sigma[i] : 0.0);
      cols[k] = (i < nv) ? i : -1;
    }
    oblock_store<VPW>(all, cols, nv, nullptr, out);
  } else {
    double all[1] = {ww};
    int cols[1] = {g == 0 ? 0 : -1};
    oblock_store<1>(all, cols, 1, nullptr, out);
  }
}

// ---- delayed reorthogonalisation (one projection sweep + one update sweep
// per Arnoldi step; see the Krylov driver) ---------------------------------

// part[c] = [sigma_i V_i . u (i < nvt), sigma_i V_i . w (i < nvt), u . w,
//            u . u, w . w] over chunk c (2 nvt + 3 values).  One launch
// covers the nv vectors i0 .. i0 + nv - 1 of the nvt (V and sigma point at
// vector i0) and, when `scalars`, the last three values; each vector's sum
// is the same whichever launch covers it (its lane group and element order
// depend on its index only).
template <typename T, int VPW, int EPL>
__global__ __launch_bounds__(kBlock) void ortho_dots2_kernel(
    const T* __restrict__ V, int64_t ldv, int nv, const double* __restrict__ sigma,
    const T* __restrict__ u, const T* __restrict__ w, int64_t N, double* __restrict__ part,
    int ldp, int i0, int nvt, int scalars) {
  constexpr int TE = 16 * EPL;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4;
  double aa[VPW], ab[VPW], uw = 0.0, uu = 0.0, ww = 0.0;
#pragma unroll
  for (int k = 0; k < VPW; ++k) aa[k] = ab[k] = 0.0;
  const int64_t base = (int64_t)blockIdx.x * kOChunk;
  const int64_t end = min(N, base + kOChunk);
  for (int64_t t0 = base + wid * TE; t0 < end; t0 += kOWaves * TE) {
    const int64_t off = t0 + (lane & 15) * EPL;
    T uv[EPL], wv[EPL], v[VPW][EPL];
    if (t0 + TE <= end) {
      oload_w<true, T, EPL>(u, off, end, uv);
      oload_w<true, T, EPL>(w, off, end, wv);
      oload_tile<true, T, VPW, EPL>(V, ldv, nv, g, w, off, end, v);
    } else {
      oload_w<false, T, EPL>(u, off, end, uv);
      oload_w<false, T, EPL>(w, off, end, wv);
      oload_tile<false, T, VPW, EPL>(V, ldv, nv, g, w, off, end, v);
    }
#pragma unroll
    for (int k = 0; k < VPW; ++k)
#pragma unroll
      for (int l = 0; l < EPL; ++l) {
        aa[k] = fma((double)v[k][l], (double)uv[l], aa[k]);
        ab[k] = fma((double)v[k][l], (double)wv[l], ab[k]);
      }
#pragma unroll
    for (int l = 0; l < EPL; ++l) {
      uw = fma((double)uv[l], (double)wv[l], uw);
      uu = fma((double)uv[l], (double)uv[l], uu);
      ww = fma((double)wv[l], (double)wv[l], ww);
    }
  }
  double* out = part + (int64_t)blockIdx.x * ldp;
  double all[2 * VPW + 3];
  int cols[2 * VPW + 3];
#pragma unroll
  for (int k = 0; k < VPW; ++k) {
    const int i = g + kOGroups * k;
    const double sg = (i < nv) ? sigma[i] : 0.0;
    all[k] = aa[k] * sg;
    all[VPW + k] = ab[k] * sg;
    cols[k] = (i < nv) ? i : -1;
    cols[VPW + k] = (i < nv) ? nv + i : -1;
  }
  all[2 * VPW] = uw;  // every group saw the same u and w; group 0 reports
  all[2 * VPW + 1] = uu;
  all[2 * VPW + 2] = ww;
  cols[2 * VPW] = (g == 0) ? 2 * nv : -1;
  cols[2 * VPW + 1] = (g == 0) ? 2 * nv + 1 : -1;
  cols[2 * VPW + 2] = (g == 0) ? 2 * nv + 2 : -1;
  // local column c: V . u of vector c < nv, V . w of vector c - nv < nv, then
  // the three scalars
  oblock_reduce<2 * VPW + 3>(
      all, cols, 2 * nv + 3,
      [=](int c) {
        return c < nv ? i0 + c
                      : (c < 2 * nv ? nvt + i0 + (c - nv) : (scalars ? 2 * nvt + (c - 2 * nv) : -1));
      },
      [](int, double r) { return r; }, out);
}

// coef = [ac (nv), bc (nv), alpha, gamma] (FP64):
//   u <- v = u - sum_i ac_i V_i                       (when u is given)
//   w <- alpha w + sum_i bc_i V_i + gamma v            (gamma only with u)
// Every thread owns EL consecutive elements (one 16-byte access per vector)
// and streams the nv basis vectors over them, eight loads in flight, summing
// in FP64 in index order: no cross-lane sums, and each vector is read once.
template <typename T, int EL>
__global__ __launch_bounds__(kBlock) void ortho_update2_kernel(
    const T* __restrict__ V, int64_t ldv, int nv, const double* __restrict__ coef,
    T* __restrict__ u, T* __restrict__ w, int64_t N) {
  using VT = typename OVec<T, EL>::type;
  constexpr int UN = 8;
  const double alpha = coef[2 * nv], gamma = coef[2 * nv + 1];
  const bool has_u = u != nullptr;
  const int64_t slots = (N + EL - 1) / EL;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < slots;
       t += (int64_t)gridDim.x * kBlock) {
    const int64_t off = t * EL;
    double pa[EL], pb[EL];
#pragma unroll
    for (int l = 0; l < EL; ++l) pa[l] = pb[l] = 0.0;
    T wv[EL], uv[EL], vt[EL], wt[EL];
    if (off + EL <= N) {
      int i = 0;
      for (; i + UN <= nv; i += UN) {
        VT x[UN];
#pragma unroll
        for (int q = 0; q < UN; ++q)
          x[q] = *reinterpret_cast<const VT*>(V + (int64_t)(i + q) * ldv + off);
#pragma unroll
        for (int q = 0; q < UN; ++q) {
          const double ca = coef[i + q], cb = coef[nv + i + q];
          const T* xe = reinterpret_cast<const T*>(&x[q]);
#pragma unroll
          for (int l = 0; l < EL; ++l) {
            pa[l] = fma(ca, (double)xe[l], pa[l]);
            pb[l] = fma(cb, (double)xe[l], pb[l]);
          }
        }
      }
      for (; i < nv; ++i) {
        const VT x = *reinterpret_cast<const VT*>(V + (int64_t)i * ldv + off);
        const double ca = coef[i], cb = coef[nv + i];
        const T* xe = reinterpret_cast<const T*>(&x);
#pragma unroll
        for (int l = 0; l < EL; ++l) {
          pa[l] = fma(ca, (double)xe[l], pa[l]);
          pb[l] = fma(cb, (double)xe[l], pb[l]);
        }
      }
      const VT wx = *reinterpret_cast<const VT*>(w + off);
      const T* we = reinterpret_cast<const T*>(&wx);
#pragma unroll
      for (int l = 0; l < EL; ++l) wv[l] = we[l];
      if (has_u) {
        const VT ux = *reinterpret_cast<const VT*>(u + off);
        const T* ue = reinterpret_cast<const T*>(&ux);
#pragma unroll
        for (int l = 0; l < EL; ++l) uv[l] = ue[l];
      }
    } else {
      for (int i = 0; i < nv; ++i) {
        const double ca = coef[i], cb = coef[nv + i];
#pragma unroll
        for (int l = 0; l < EL; ++l) {
          const double x = off + l < N ? (double)V[(int64_t)i * ldv + off + l] : 0.0;
          pa[l] = fma(ca, x, pa[l]);
          pb[l] = fma(cb, x, pb[l]);
        }
      }
#pragma unroll
      for (int l = 0; l < EL; ++l) {
        wv[l] = off + l < N ? w[off + l] : (T)0;
        uv[l] = (has_u && off + l < N) ? u[off + l] : (T)0;
      }
    }
#pragma unroll
    for (int l = 0; l < EL; ++l) {
      double nw = fma(alpha, (double)wv[l], pb[l]);
      if (has_u) {
        vt[l] = (T)((double)uv[l] - pa[l]);
        nw = fma(gamma, (double)vt[l], nw);
      }
      wt[l] = (T)nw;
    }
    if (off + EL <= N) {
      VT tw;
      T* tp = reinterpret_cast<T*>(&tw);
#pragma unroll
      for (int l = 0; l < EL; ++l) tp[l] = wt[l];
      *reinterpret_cast<VT*>(w + off) = tw;
      if (has_u) {
        VT tv;
        T* tq = reinterpret_cast<T*>(&tv);
#pragma unroll
        for (int l = 0; l < EL; ++l) tq[l] = vt[l];
        *reinterpret_cast<VT*>(u + off) = tv;
      }
    } else {
#pragma unroll
      for (int l = 0; l < EL; ++l)
        if (off + l < N) {
          w[off + l] = wt[l];
          if (has_u) u[off + l] = vt[l];
        }
    }
  }
}

// Device side of one round of the delayed CGS2 process (the arithmetic the
// Krylov driver does on the host between rounds, done here so that a whole
// restart cycle can be enqueued at once).  State: H (column i, entries
// 0..i+1, at H + i ldh), h1p (first projection of the pending column),
// sigma, scal = [||M q_{j-1}||^2, round of a breakdown or -1].  Round 0
// consumes [q_0 . W', ||W'||^2]; round j >= 1 the 2 j + 3 sums of the
// projection sweep (or, in the final round, the j + 1 sums [Q^T u_j,
// ||u_j||^2]) and finalises column j - 1; unless final it writes the
// coefficients of the next update sweep [ac (j), bc (j), alpha, gamma],
// sigma_j and the next h1p.  After a breakdown every later round writes zero
// coefficients (the vectors become zero, never NaN).  One block of 64
// threads; sums in index order.
__global__ __launch_bounds__(64) void dcgs2_round_kernel(const double* __restrict__ res, int j,
                                                         int final_round, int ldh,
                                                         double* __restrict__ H,
                                                         double* __restrict__ h1p,
                                                         double* __restrict__ sigma,
                                                         double* __restrict__ coef,
                                                         double* __restrict__ scal) {
  constexpr double eps = 2.220446049250313e-16;
  // everything the round reads is staged in LDS first (one parallel load),
  // so the sequential part runs on LDS latencies
  __shared__ double Hs[64][65];  // Hs[i][l] = H(l, i), the finished columns i < j
  __shared__ double a[64], b[64], g[65], hp[65], sg[64], sh[8];
  const int t = threadIdx.x;
  if (j == 0) {
    if (t == 0) {
      h1p[0] = res[0];
      scal[0] = res[1];
      scal[1] = -1.0;
      coef[0] = 0.0;
      coef[1] = -res[0] * sigma[0];
      coef[2] = 1.0;
      coef[3] = 0.0;
    }
    return;
  }
  if (scal[1] >= 0.0) {  // the cycle broke down earlier: inert coefficients
    for (int l = t; l < 2 * j + 2; l += 64) coef[l] = 0.0;
    if (t == 0) sigma[j] = 0.0;
    return;
  }
  if (t < j) {
    a[t] = res[t];
    b[t] = final_round ? 0.0 : res[j + t];
    hp[t] = h1p[t];
    sg[t] = sigma[t];
  }
  if (t == 0) {
    sh[0] = final_round ? res[j] : res[2 * j + 1];  // d
    sh[1] = final_round ? 0.0 : res[2 * j];         // c
    sh[2] = final_round ? 0.0 : res[2 * j + 2];     // e
    sh[3] = scal[0];                                // w2prev
  }
  // columns 0..j-2 of H (rows 0..i+1 of column i), eight loads in flight
#pragma unroll 8
  for (int i = 0; i < 62; ++i)
    if (i + 1 < j && t <= i + 1) Hs[i][t] = H[t + (int64_t)ldh * i];
  __syncthreads();
  if (t == 0) {
    double na2 = 0.0;
    for (int l = 0; l < j; ++l) na2 += a[l] * a[l];
    const double nu2 = sh[0] - na2;
    const bool breakdown = !(nu2 > 256.0 * eps * eps * sh[3]);
    const double nu = breakdown ? 0.0 : sqrt(nu2);
    H[j + (int64_t)ldh * (j - 1)] = nu;
    Hs[j - 1][j] = nu;
    sh[4] = nu;
    sh[5] = breakdown ? 1.0 : 0.0;
    if (breakdown) scal[1] = (double)j;
  }
  if (t < j) {
    const double hv = hp[t] + a[t];
    H[t + (int64_t)ldh * (j - 1)] = hv;
    Hs[j - 1][t] = hv;
  }
  __syncthreads();
  const double nu = sh[4];
  if (final_round || sh[5] != 0.0) {
    if (!final_round) {
      for (int l = t; l < 2 * j + 2; l += 64) coef[l] = 0.0;
      if (t == 0) sigma[j] = 0.0;
    }
    return;
  }
  // g = H a over the finished columns 0..j-1 (H(l, i) is zero for l > i + 1)
  if (t <= j) {
    double acc = 0.0;
    for (int i = (t > 0 ? t - 1 : 0); i < j; ++i) acc += Hs[i][t] * a[i];
    g[t] = acc;
  }
  __syncthreads();
  if (t == 0) {
    double ab = 0.0;
    for (int l = 0; l < j; ++l) ab += a[l] * b[l];
    const double qjw = (sh[1] - ab) / nu;  // q_j . W'
    double gw = 0.0, gg = 0.0;
    for (int l = 0; l < j; ++l) gw += g[l] * b[l];
    gw += g[j] * qjw;
    for (int l = 0; l <= j; ++l) gg += g[l] * g[l];
    scal[0] = fmax(0.0, (sh[2] - 2.0 * gw + gg) / (nu * nu));
    sh[6] = qjw;
  }
  __syncthreads();
  if (t < j) {
    const double hn = (b[t] - g[t]) / nu;
    coef[t] = a[t] * sg[t];
    coef[j + t] = -(g[t] / nu + hn) * sg[t];
    h1p[t] = hn;
  } else if (t == j) {
    const double hn = (sh[6] - g[j]) / nu;
    coef[2 * j] = 1.0 / nu;
    coef[2 * j + 1] = -(g[j] / nu + hn) / nu;
    h1p[j] = hn;
    sigma[j] = 1.0 / nu;
  }
}

inline int stream_grid(int64_t count) {
  int64_t b = (count + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

// ------------------------------------------------------------------ launchers

void build_xform(double* M, int p, int kind, hipStream_t st) {
  int tot = p * p;
  hipLaunchKernelGGL(build_xform_kernel, dim3((tot + 255) / 256), dim3(256), 0, st, M, p, kind);
  TSYLV_LAUNCH_CHECK();
}

void tube_xform_f64(const double* in, double* out, const double* M, int64_t E, int p,
                    hipStream_t st) {
  if (E <= 0) return;
  dim3 grid((unsigned)((E + kBlock - 1) / kBlock));
  if (p <= 4)
    hipLaunchKernelGGL(tube_xform_kernel<4>, grid, dim3(kBlock), 0, st, in, out, M, E, p);
  else if (p <= 8)
    hipLaunchKernelGGL(tube_xform_kernel<8>, grid, dim3(kBlock), 0, st, in, out, M, E, p);
  else if (p <= 16)
    hipLaunchKernelGGL(tube_xform_kernel<16>, grid, dim3(kBlock), 0, st, in, out, M, E, p);
  else if (p <= 32)
    hipLaunchKernelGGL(tube_xform_kernel<32>, grid, dim3(kBlock), 0, st, in, out, M, E, p);
  else if (p <= 64)
    hipLaunchKernelGGL(tube_xform_kernel<64>, grid, dim3(kBlock), 0, st, in, out, M, E, p);
  else
    hipLaunchKernelGGL(tube_xform_generic_kernel, grid, dim3(kBlock), 0, st, in, out, M, E, p);
  TSYLV_LAUNCH_CHECK();
}

void tube_xform_gen_f64(const GenTensor& g, double* out, const double* M, int64_t E, int p,
                        hipStream_t st) {
  if (E <= 0) return;
  if (p > kGenXformMaxP) throw Error(TSYLV_EINVAL, "generated transform: p > 64");
  dim3 grid((unsigned)((E + kBlock - 1) / kBlock));
  if (p <= 4)
    hipLaunchKernelGGL(tube_xform_gen_kernel<4>, grid, dim3(kBlock), 0, st, g, out, M, E, p);
  else if (p <= 8)
    hipLaunchKernelGGL(tube_xform_gen_kernel<8>, grid, dim3(kBlock), 0, st, g, out, M, E, p);
  else if (p <= 16)
    hipLaunchKernelGGL(tube_xform_gen_kernel<16>, grid, dim3(kBlock), 0, st, g, out, M, E, p);
  else if (p <= 32)
    hipLaunchKernelGGL(tube_xform_gen_kernel<32>, grid, dim3(kBlock), 0, st, g, out, M, E, p);
  else
    hipLaunchKernelGGL(tube_xform_gen_kernel<64>, grid, dim3(kBlock), 0, st, g, out, M, E, p);
  TSYLV_LAUNCH_CHECK();
}

void gen_tensor_f64(const GenTensor& g, double* out, int64_t E, int p, hipStream_t st) {
  if (E <= 0 || p <= 0) return;
  hipLaunchKernelGGL(gen_tensor_kernel, dim3(stream_grid(E)), dim3(kBlock), 0, st, g, out, E, p);
  TSYLV_LAUNCH_CHECK();
}

void convert_f64_f32(const double* in, float* out, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(stream_grid(count)), dim3(kBlock), 0, st, in, out,
                     count);
  TSYLV_LAUNCH_CHECK();
}

void convert_f32_f64(const float* in, double* out, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(f32_to_f64_kernel, dim3(stream_grid(count)), dim3(kBlock), 0, st, in, out,
                     count);
  TSYLV_LAUNCH_CHECK();
}

void convert_f64_bf16(const double* in, uint16_t* out, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(f64_to_bf16_kernel, dim3(stream_grid(count)), dim3(kBlock), 0, st, in, out,
                     count);
  TSYLV_LAUNCH_CHECK();
}

void fill_random(void* buf, int64_t count, int elem, uint64_t seed, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(fill_random_kernel, dim3(stream_grid(count)), dim3(kBlock), 0, st, buf,
                     count, elem, seed);
  TSYLV_LAUNCH_CHECK();
}

int mdot_chunks(int64_t N) { return (int)((N + kChunk - 1) / kChunk); }

template <typename T>
static void mdot_any(const T* V, int64_t ldv, int nv, const T* w, int64_t N, double* part,
                     int ldp, int with_ww, hipStream_t st) {
  int ncols = nv + (with_ww ? 1 : 0);
  if (ncols == 0 || N <= 0) return;
  if (ncols > ldp) throw Error(TSYLV_EINVAL, "mdot: partial row too short");
  dim3 grid(mdot_chunks(N), (ncols + kVG - 1) / kVG);
  hipLaunchKernelGGL(mdot_kernel<T>, grid, dim3(kBlock), 0, st, V, ldv, nv, w, N, part, ldp,
                     with_ww ? 1 : 0);
  TSYLV_LAUNCH_CHECK();
}

void mdot_partial(const double* V, int64_t ldv, int nv, const double* w, int64_t N,
                  double* part, int ldp, int with_ww, hipStream_t st) {
  mdot_any<double>(V, ldv, nv, w, N, part, ldp, with_ww, st);
}

void mdot_partial(const float* V, int64_t ldv, int nv, const float* w, int64_t N, double* part,
                  int ldp, int with_ww, hipStream_t st) {
  mdot_any<float>(V, ldv, nv, w, N, part, ldp, with_ww, st);
}

void reduce_partials(const double* part, int nchunks, int ldp, int ncols, double* out,
                     hipStream_t st) {
  if (ncols == 0) return;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(ncols), dim3(kBlock), 0, st, part, nchunks,
                     ldp, out);
  TSYLV_LAUNCH_CHECK();
}

template <typename TB, typename TW>
static void mupdate_any(const TB* V, int64_t ldv, int nv, const double* h, TW* w, int64_t N,
                        hipStream_t st) {
  if (nv == 0 || N <= 0) return;
  if (nv > kMaxUpd) throw Error(TSYLV_EINVAL, "mupdate: too many vectors");
  dim3 grid((unsigned)((N + kBlock - 1) / kBlock));
  hipLaunchKernelGGL((mupdate_kernel<TB, TW>), grid, dim3(kBlock), 0, st, V, ldv, nv, h, w, N);
  TSYLV_LAUNCH_CHECK();
}

void mupdate(const double* V, int64_t ldv, int nv, const double* h, double* w, int64_t N,
             hipStream_t st) {
  mupdate_any<double, double>(V, ldv, nv, h, w, N, st);
}

void mupdate(const float* V, int64_t ldv, int nv, const double* h, float* w, int64_t N,
             hipStream_t st) {
  mupdate_any<float, float>(V, ldv, nv, h, w, N, st);
}

void mupdate(const float* V, int64_t ldv, int nv, const double* h, double* w, int64_t N,
             hipStream_t st) {
  mupdate_any<float, double>(V, ldv, nv, h, w, N, st);
}

void dcgs2_round(const double* res, int j, bool final_round, int ldh, double* H, double* h1p,
                 double* sigma, double* coef, double* scal, hipStream_t st) {
  if (j < 0 || j > 63) throw Error(TSYLV_EINVAL, "dcgs2_round: round out of range");
  hipLaunchKernelGGL(dcgs2_round_kernel, dim3(1), dim3(64), 0, st, res, j, final_round ? 1 : 0,
                     ldh, H, h1p, sigma, coef, scal);
  TSYLV_LAUNCH_CHECK();
}

int ortho_chunks(int64_t N) { return (int)((N + kOChunk - 1) / kOChunk); }

int ortho_max_vectors(bool) { return 16 * kOGroups; }

// elements per lane: 16-byte accesses for FP64 and FP32 (measured faster than
// 8-byte FP32 accesses despite the extra registers), 8-byte ones for BF16
// (four values per lane keep the register count of the FP32 kernels)
template <typename T>
constexpr int ortho_epl() {
  return sizeof(T) == 8 ? 2 : 4;
}

template <typename T>
static void ortho_check(const T* V, int64_t ldv, const T* w) {
  constexpr int EPL = ortho_epl<T>();
  constexpr uintptr_t align = sizeof(T) * EPL;
  if ((reinterpret_cast<uintptr_t>(V) | reinterpret_cast<uintptr_t>(w)) % align != 0 ||
      ldv % EPL != 0)
    throw Error(TSYLV_EINVAL, "ortho: basis not aligned");
}

template <typename T, int VPW>
static void ortho_dots_t(const T* V, int64_t ldv, int nv, const double* sigma, const T* w,
                         int64_t N, double* part, int ldp, hipStream_t st) {
  hipLaunchKernelGGL((ortho_dots_kernel<T, VPW, ortho_epl<T>()>), dim3(ortho_chunks(N)),
                     dim3(kBlock), 0, st, V, ldv, nv, sigma, w, N, part, ldp);
  TSYLV_LAUNCH_CHECK();
}

template <typename T, int VPW>
static void ortho_update_t(const T* V, int64_t ldv, int nv, const double* h, const double* sigma,
                           T* w, int64_t N, double* part, int ldp, int mode, hipStream_t st) {
  hipLaunchKernelGGL((ortho_update_kernel<T, VPW, ortho_epl<T>()>), dim3(ortho_chunks(N)),
                     dim3(kBlock), 0, st, V, ldv, nv, h, sigma, w, N, part, ldp, mode);
  TSYLV_LAUNCH_CHECK();
}

// vectors per lane group for nv basis vectors
static int ortho_vpw(int nv) {
  static const int sizes[] = {1, 2, 3, 4, 6, 8, 10, 12, 14, 16};
  const int need = (nv + kOGroups - 1) / kOGroups;
  for (int v : sizes)
    if (need <= v) return v;
  throw Error(TSYLV_EINVAL, "ortho: too many basis vectors");
}

#define TSYLV_OVPW_CASES(F) \
  F(1) F(2) F(3) F(4) F(6) F(8) F(10) F(12) F(14) F(16)

template <typename T>
static void ortho_dots_any(const T* V, int64_t ldv, int nv, const double* sigma, const T* w,
                           int64_t N, double* part, int ldp, hipStream_t st) {
  if (nv < 1 || nv + 1 > ldp) throw Error(TSYLV_EINVAL, "ortho: bad vector count");
  if (N <= 0) return;
  ortho_check(V, ldv, w);
  switch (ortho_vpw(nv)) {
#define F(K) \
  case K: ortho_dots_t<T, K>(V, ldv, nv, sigma, w, N, part, ldp, st); break;
    TSYLV_OVPW_CASES(F)
#undef F
  }
}

template <typename T>
static void ortho_update_any(const T* V, int64_t ldv, int nv, const double* h,
                             const double* sigma, T* w, int64_t N, double* part, int ldp,
                             int mode, hipStream_t st) {
  if (nv < 1 || nv > ldp) throw Error(TSYLV_EINVAL, "ortho: bad vector count");
  if (N <= 0) return;
  ortho_check(V, ldv, (const T*)w);
  switch (ortho_vpw(nv)) {
#define F(K) \
  case K: ortho_update_t<T, K>(V, ldv, nv, h, sigma, w, N, part, ldp, mode, st); break;
    TSYLV_OVPW_CASES(F)
#undef F
  }
}

void ortho_dots(const double* V, int64_t ldv, int nv, const double* sigma, const double* w,
                int64_t N, double* part, int ldp, hipStream_t st) {
  ortho_dots_any<double>(V, ldv, nv, sigma, w, N, part, ldp, st);
}
void ortho_dots(const float* V, int64_t ldv, int nv, const double* sigma, const float* w,
                int64_t N, double* part, int ldp, hipStream_t st) {
  ortho_dots_any<float>(V, ldv, nv, sigma, w, N, part, ldp, st);
}
void ortho_update(const double* V, int64_t ldv, int nv, const double* h, const double* sigma,
                  double* w, int64_t N, double* part, int ldp, int mode, hipStream_t st) {
  ortho_update_any<double>(V, ldv, nv, h, sigma, w, N, part, ldp, mode, st);
}
void ortho_update(const float* V, int64_t ldv, int nv, const double* h, const double* sigma,
                  float* w, int64_t N, double* part, int ldp, int mode, hipStream_t st) {
  ortho_update_any<float>(V, ldv, nv, h, sigma, w, N, part, ldp, mode, st);
}

void ortho_dots(const bf16t* V, int64_t ldv, int nv, const double* sigma, const bf16t* w,
                int64_t N, double* part, int ldp, hipStream_t st) {
  ortho_dots_any<OB16>(reinterpret_cast<const OB16*>(V), ldv, nv, sigma,
                       reinterpret_cast<const OB16*>(w), N, part, ldp, st);
}
void ortho_update(const bf16t* V, int64_t ldv, int nv, const double* h, const double* sigma,
                  bf16t* w, int64_t N, double* part, int ldp, int mode, hipStream_t st) {
  ortho_update_any<OB16>(reinterpret_cast<const OB16*>(V), ldv, nv, h, sigma,
                         reinterpret_cast<OB16*>(w), N, part, ldp, mode, st);
}

template <typename T>
static void ortho_dots2_part(const T* V, int64_t ldv, int nv, const double* sigma, const T* u,
                             const T* w, int64_t N, double* part, int ldp, int i0, int nvt,
                             bool scalars, hipStream_t st) {
  const dim3 grid(ortho_chunks(N)), block(kBlock);
  constexpr int EPL = ortho_epl<T>();
  const T* Vi = V + (int64_t)i0 * ldv;
  const double* si = sigma + i0;
  const int sc = scalars ? 1 : 0;
  switch (ortho_vpw(nv)) {
#define F(K)                                                                               \
  case K:                                                                                  \
    hipLaunchKernelGGL((ortho_dots2_kernel<T, K, EPL>), grid, block, 0, st, Vi, ldv, nv, si, \
                       u, w, N, part, ldp, i0, nvt, sc);                                   \
    break;
    TSYLV_OVPW_CASES(F)
#undef F
  }
  TSYLV_LAUNCH_CHECK();
}

// Above ortho_dots2_split<T>() vectors the sweep is two launches (that many
// vectors with the scalars, then the rest): one launch over all of them
// would need more than 168 VGPRs (the FP64 sums of 2 VPW vectors per lane
// and their widened values), two waves per SIMD and too few loads in
// flight (3.9 against 5.7 TB/s for BF16 vectors at n s p = 6.7e7); the
// split re-reads u and w once more and computes the same bits.  BF16 vectors
// reach that at VPW = 10 (193 VGPRs), FP32 and FP64 ones at VPW = 12.
template <typename T>
constexpr int ortho_dots2_split() {
  return sizeof(T) == 2 ? 8 * kOGroups : 10 * kOGroups;
}

template <typename T>
static void ortho_dots2_any(const T* V, int64_t ldv, int nv, const double* sigma, const T* u,
                            const T* w, int64_t N, double* part, int ldp, hipStream_t st) {
  if (nv < 1 || 2 * nv + 3 > ldp) throw Error(TSYLV_EINVAL, "ortho: bad vector count");
  if (N <= 0) return;
  ortho_check(V, ldv, w);
  ortho_check(V, ldv, u);
  constexpr int split = ortho_dots2_split<T>();
  if (nv <= split) {
    ortho_dots2_part(V, ldv, nv, sigma, u, w, N, part, ldp, 0, nv, true, st);
    return;
  }
  ortho_dots2_part(V, ldv, split, sigma, u, w, N, part, ldp, 0, nv, true, st);
  ortho_dots2_part(V, ldv, nv - split, sigma, u, w, N, part, ldp, split, nv, false, st);
}

template <typename T>
static void ortho_update2_any(const T* V, int64_t ldv, int nv, const double* coef, T* u, T* w,
                              int64_t N, hipStream_t st) {
  if (nv < 1) throw Error(TSYLV_EINVAL, "ortho: bad vector count");
  if (N <= 0) return;
  constexpr int EL = 16 / (int)sizeof(T);  // one 16-byte access per vector and thread
  if ((reinterpret_cast<uintptr_t>(V) | reinterpret_cast<uintptr_t>(w) |
       reinterpret_cast<uintptr_t>(u)) % 16 != 0 || ldv % EL != 0)
    throw Error(TSYLV_EINVAL, "ortho: basis not aligned");
  const int64_t slots = (N + EL - 1) / EL;
  const int blocks = (int)std::min<int64_t>((slots + kBlock - 1) / kBlock, 16384);
  hipLaunchKernelGGL((ortho_update2_kernel<T, EL>), dim3(blocks), dim3(kBlock), 0, st, V, ldv, nv,
                     coef, u, w, N);
  TSYLV_LAUNCH_CHECK();
}

void ortho_dots2(const double* V, int64_t ldv, int nv, const double* sigma, const double* u,
                 const double* w, int64_t N, double* part, int ldp, hipStream_t st) {
  ortho_dots2_any<double>(V, ldv, nv, sigma, u, w, N, part, ldp, st);
}
void ortho_dots2(const float* V, int64_t ldv, int nv, const double* sigma, const float* u,
                 const float* w, int64_t N, double* part, int ldp, hipStream_t st) {
  ortho_dots2_any<float>(V, ldv, nv, sigma, u, w, N, part, ldp, st);
}
void ortho_update2(const double* V, int64_t ldv, int nv, const double* coef, double* u, double* w,
                   int64_t N, hipStream_t st) {
  ortho_update2_any<double>(V, ldv, nv, coef, u, w, N, st);
}
void ortho_update2(const float* V, int64_t ldv, int nv, const double* coef, float* u, float* w,
                   int64_t N, hipStream_t st) {
  ortho_update2_any<float>(V, ldv, nv, coef, u, w, N, st);
}
void ortho_dots2(const bf16t* V, int64_t ldv, int nv, const double* sigma, const bf16t* u,
                 const bf16t* w, int64_t N, double* part, int ldp, hipStream_t st) {
  ortho_dots2_any<OB16>(reinterpret_cast<const OB16*>(V), ldv, nv, sigma,
                        reinterpret_cast<const OB16*>(u), reinterpret_cast<const OB16*>(w), N,
                        part, ldp, st);
}
void ortho_update2(const bf16t* V, int64_t ldv, int nv, const double* coef, bf16t* u, bf16t* w,
                   int64_t N, hipStream_t st) {
  ortho_update2_any<OB16>(reinterpret_cast<const OB16*>(V), ldv, nv, coef,
                          reinterpret_cast<OB16*>(u), reinterpret_cast<OB16*>(w), N, st);
}

template <typename TI, typename TO>
static void scale_any(const TI* x, TO* out, double a, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL((scale_kernel<TI, TO>), dim3(stream_grid(N)), dim3(kBlock), 0, st, x, out,
                     a, N);
  TSYLV_LAUNCH_CHECK();
}

void scale(const double* x, double* out, double a, int64_t N, hipStream_t st) {
  scale_any<double, double>(x, out, a, N, st);
}
void scale(const float* x, float* out, double a, int64_t N, hipStream_t st) {
  scale_any<float, float>(x, out, a, N, st);
}
void scale(const double* x, float* out, double a, int64_t N, hipStream_t st) {
  scale_any<double, float>(x, out, a, N, st);
}

}  // namespace kern
}  // namespace tsylv
