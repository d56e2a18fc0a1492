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
__global__ __launch_bounds__(kBlock) void tube_xform_kernel(
    const double* __restrict__ in, double* __restrict__ out,
    const double* __restrict__ M, int64_t E, int p) {
  __shared__ double Ms[PMAX * PMAX];
  for (int t = threadIdx.x; t < PMAX * PMAX; t += kBlock) {
    int q = t / PMAX, j = t % PMAX;
    Ms[t] = (q < p && j < p) ? M[q * p + j] : 0.0;
  }
  __syncthreads();
  int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= E) return;
  double v[PMAX];
#pragma unroll
  for (int j = 0; j < PMAX; ++j) v[j] = (j < p) ? in[(int64_t)j * E + e] : 0.0;
  for (int q = 0; q < p; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < PMAX; ++j) acc = fma(Ms[q * PMAX + j], v[j], acc);
    out[(int64_t)q * E + e] = acc;
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
