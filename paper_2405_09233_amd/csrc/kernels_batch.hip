// Vector kernels of the batched lockstep tGMRES (Algorithm 3 with the
// Arnoldi process of Algorithm 2, classical Gram-Schmidt applied twice, for
// many independent instances at once).
//
// Work items are chunks of kBatchChunk elements of one instance's vectors;
// the grid covers the chunks of every instance, a block finds its instance
// by binary search over the instances' first chunk, and instances that are
// not stepping return at once.  Each thread owns 32 elements of its chunk
// (coalesced: element base + 256 q + thread).  Dot products reduce within a
// wave by shuffles, across the four waves in a fixed order, and across the
// chunks of an instance in chunk order (batch_reduce), so an instance's
// numbers do not depend on the rest of the batch.  The second Gram-Schmidt
// pass is taken only when the first one cancelled more than 1 - 1/sqrt(2) of
// ||W|| (the criterion of Daniel, Gragg, Kaufman and Stewart, Math. Comp.
// 1976); otherwise ||W|| after the pass follows from Pythagoras, and the
// step reads the basis twice instead of four times.  The small per-instance
// arithmetic (the Givens rotations of section 3.3, the restart test of
// Algorithm 3, the triangular solve for y) runs in one wave per instance.
#include "kernels.hpp"

namespace tsylv {
namespace kern {

namespace {

constexpr int kBT = 256;
constexpr int kQ = (int)(kBatchChunk / kBT);
static_assert(kQ * kBT == kBatchChunk, "chunk split");

__device__ __forceinline__ int find_chunk_item(const BatchItem* items, int count, int c) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].chunk0 <= c) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ bool stepping(const BatchState& S) { return S.active != 0; }

// part[c][l] = V_l . x over chunk c (MODE STEP: x = W, l <= j; WNORM: W . W;
// RESID: V_0 . V_0; CNORM: Zc . Zc).  The mode is a template parameter: a
// runtime four-way choice of the vector was compiled into a wrong pointer
// selection (CNORM read W), so every mode-dependent choice here is made at
// compile time.
template <int MODE>
__global__ __launch_bounds__(kBT) void batch_dots_kernel(const BatchItem* __restrict__ items,
                                                         int count,
                                                         const BatchState* __restrict__ st,
                                                         const int* __restrict__ jp,
                                                         double* __restrict__ part, int ldp) {
  const int c = blockIdx.x;
  const int i = find_chunk_item(items, count, c);
  const BatchItem& it = items[i];
  bool on;
  if constexpr (MODE == BM_STEP)
    on = st[i].active != 0;
  else if constexpr (MODE == BM_PASS2 || MODE == BM_WNORM)
    on = st[i].active != 0 && st[i].reorth != 0;
  else if constexpr (MODE == BM_RESID)
    on = st[i].done == 0;
  else
    on = true;
  if (!on) return;
  const double* x;
  int nv = 1;  // columns: V_l . x for l < nv - (STEP ? 1 : 0), STEP adds x . x
  if constexpr (MODE == BM_STEP) {
    x = it.W;
    nv = *jp + 2;
  } else if constexpr (MODE == BM_PASS2) {
    x = it.W;
    nv = *jp + 1;
  } else if constexpr (MODE == BM_WNORM) {
    x = it.W;
  } else if constexpr (MODE == BM_RESID) {
    x = it.V;
  } else {
    x = it.Zc;
  }
  const int64_t base = (int64_t)(c - it.chunk0) * kBatchChunk;
  const int64_t end = it.N < base + kBatchChunk ? it.N : base + kBatchChunk;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double xv[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int64_t e = base + q * kBT + tid;
    xv[q] = e < end ? x[e] : 0.0;
  }
  __shared__ double red[kBT / 64][kBatchMaxM + 2];
  const int nbasis = (MODE == BM_STEP) ? nv - 1 : ((MODE == BM_PASS2) ? nv : 0);
  for (int l = 0; l < nv; ++l) {
    const double* v = (l < nbasis) ? it.V + (int64_t)l * it.ldv : x;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int64_t e = base + q * kBT + tid;
      if (e < end) acc = fma(v[e], xv[q], acc);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) red[wave][l] = acc;
  }
  __syncthreads();
  if (tid < nv)
    part[(int64_t)c * ldp + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

// One wave per instance: sums its chunks' partials in chunk order, then
//   STEP / PASS2: H(0:j, j) = (or +=) h, coef = h (the pass's coefficients);
//   WNORM: ||W||, H(j+1, j), the Givens update of section 3.3 and the stop
//          test (estimate, breakdown, end of cycle);
//   RESID / RESID0: beta = ||R||, the restart test of Algorithm 3 (RESID
//          counts a finished cycle), and g, coef for the new cycle;
//   CNORM: ||C||.
template <int MODE>
__global__ __launch_bounds__(64) void batch_reduce_kernel(const BatchItem* __restrict__ items,
                                                          BatchState* __restrict__ st,
                                                          const int* __restrict__ jp,
                                                          const double* __restrict__ part, int ldp,
                                                          int m, double tol, int max_cycles) {
  const int i = blockIdx.x;
  const BatchItem& it = items[i];
  BatchState& S = st[i];
  constexpr bool kResid = MODE == BM_RESID || MODE == BM_RESID0;
  constexpr bool kGs = MODE == BM_STEP || MODE == BM_PASS2;
  bool on;
  if constexpr (MODE == BM_STEP || MODE == BM_WNORM)
    on = S.active != 0;
  else if constexpr (MODE == BM_PASS2)
    on = S.active != 0 && S.reorth != 0;
  else if constexpr (kResid)
    on = S.done == 0;
  else
    on = true;
  if (!on) return;
  const int j = *jp;
  const int nv = (MODE == BM_STEP) ? j + 2 : ((MODE == BM_PASS2) ? j + 1 : 1);
  const int lane = threadIdx.x;
  __shared__ double sums[kBatchMaxM + 2];
  if (lane < nv) {
    double acc = 0.0;
    for (int q = 0; q < it.nchunks; ++q) acc += part[(int64_t)(it.chunk0 + q) * ldp + lane];
    sums[lane] = acc;
  }
  __syncthreads();
  const int ldh = m + 1;
  if constexpr (kGs) {
    if (lane <= j) {
      double* h = it.H + (int64_t)j * ldh;
      h[lane] = (MODE == BM_STEP) ? sums[lane] : h[lane] + sums[lane];
      it.coef[lane] = sums[lane];
    }
    if (MODE == BM_STEP && lane == 0) {
      // ||W - V h||^2 = ||W||^2 - ||h||^2 when V is orthonormal
      const double ww = sums[j + 1];
      double hh = 0.0;
      for (int l = 0; l <= j; ++l) hh += sums[l] * sums[l];
      const double rem = ww - hh;
      S.mv2 = ww;
      if (rem > 0.5 * ww) {
        S.reorth = 0;
        S.hn = sqrt(rem);
      } else {
        S.reorth = 1;
      }
    }
    return;
  }
  if (lane != 0) return;
  if constexpr (MODE == BM_CNORM) {
    S.cnorm = sqrt(sums[0]);
    return;
  }
  if constexpr (MODE == BM_WNORM) {
    double* h = it.H + (int64_t)j * ldh;
    const double hn = S.reorth ? sqrt(sums[0]) : S.hn;
    const double mv2 = S.mv2;
    h[j + 1] = hn;
    for (int l = 0; l < j; ++l) {
      const double a = h[l], b = h[l + 1];
      h[l] = it.cs[l] * a + it.sn[l] * b;
      h[l + 1] = -it.sn[l] * a + it.cs[l] * b;
    }
    const double a = h[j], b = h[j + 1];
    const double r = hypot(a, b);
    const double c = r > 0.0 ? a / r : 1.0, s = r > 0.0 ? b / r : 0.0;
    it.cs[j] = c;
    it.sn[j] = s;
    h[j] = r;
    h[j + 1] = 0.0;
    const double gj = it.g[j];
    it.g[j] = c * gj;
    it.g[j + 1] = -s * gj;
    const double est = fabs(it.g[j + 1]);
    S.hn = hn;
    S.est = est;
    S.jdone = j + 1;
    S.steps += 1;
    const bool breakdown = hn <= 16.0 * 2.220446049250313e-16 * sqrt(mv2);
    if (est <= tol * S.cnorm || breakdown || j + 1 >= m) S.active = 0;
    return;
  }
  // restart test on the true residual R = C - M(X), stored in V_0
  const double beta = sqrt(sums[0]);
  S.beta = beta;
  S.est = beta;
  if constexpr (MODE == BM_RESID) S.cycles += 1;
  const double relres = S.cnorm > 0.0 ? beta / S.cnorm : (beta > 0.0 ? INFINITY : 0.0);
  S.jdone = 0;
  if (relres <= tol) {
    S.done = 1;
    S.active = 0;
    S.status = TSYLV_OK;
  } else if (S.cycles >= max_cycles) {
    S.done = 1;
    S.active = 0;
    S.status = TSYLV_NOT_CONVERGED;
  } else {
    S.active = 1;
    it.g[0] = beta;
    for (int l = 1; l <= m; ++l) it.g[l] = 0.0;
    it.coef[0] = 1.0 / beta;
  }
}

// STEP: W -= sum_{l <= j} coef_l V_l;  XUPDATE: Zx += sum_{l < jdone} y_l V_l.
template <int MODE>
__global__ __launch_bounds__(kBT) void batch_update_kernel(const BatchItem* __restrict__ items,
                                                           int count,
                                                           const BatchState* __restrict__ st,
                                                           const int* __restrict__ jp) {
  const int c = blockIdx.x;
  const int i = find_chunk_item(items, count, c);
  const BatchItem& it = items[i];
  const BatchState& S = st[i];
  constexpr bool kStep = MODE == BM_STEP || MODE == BM_PASS2;
  const bool on = (MODE == BM_STEP)    ? S.active != 0
                  : (MODE == BM_PASS2) ? (S.active != 0 && S.reorth != 0)
                                       : (S.done == 0 && S.jdone > 0);
  if (!on) return;
  const int nv = kStep ? *jp + 1 : S.jdone;
  const double* cf;
  double* x;
  if constexpr (kStep) {
    cf = it.coef;
    x = it.W;
  } else {
    cf = it.y;
    x = it.Zx;
  }
  constexpr double sg = kStep ? -1.0 : 1.0;
  const int64_t base = (int64_t)(c - it.chunk0) * kBatchChunk;
  const int64_t end = it.N < base + kBatchChunk ? it.N : base + kBatchChunk;
  const int tid = threadIdx.x;
  double acc[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int64_t e = base + q * kBT + tid;
    acc[q] = e < end ? x[e] : 0.0;
  }
  for (int l = 0; l < nv; ++l) {
    const double* v = it.V + (int64_t)l * it.ldv;
    const double a = sg * cf[l];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int64_t e = base + q * kBT + tid;
      if (e < end) acc[q] = fma(a, v[e], acc[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int64_t e = base + q * kBT + tid;
    if (e < end) x[e] = acc[q];
  }
}

// STEP: V_{j+1} = W / ||W|| (instances still stepping);
// RESID: V_0 *= 1 / beta (instances starting a cycle).
template <int MODE>
__global__ __launch_bounds__(kBT) void batch_scale_kernel(const BatchItem* __restrict__ items,
                                                          int count,
                                                          const BatchState* __restrict__ st,
                                                          const int* __restrict__ jp) {
  const int c = blockIdx.x;
  const int i = find_chunk_item(items, count, c);
  const BatchItem& it = items[i];
  const BatchState& S = st[i];
  if (S.active == 0) return;
  const double* x;
  double* y;
  double a;
  if constexpr (MODE == BM_STEP) {
    x = it.W;
    y = it.V + (int64_t)(*jp + 1) * it.ldv;
    a = 1.0 / S.hn;
  } else {
    x = it.V;
    y = it.V;
    a = it.coef[0];
  }
  const int64_t base = (int64_t)(c - it.chunk0) * kBatchChunk;
  const int64_t end = it.N < base + kBatchChunk ? it.N : base + kBatchChunk;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int64_t e = base + q * kBT + threadIdx.x;
    if (e < end) y[e] = a * x[e];
  }
}

// y = R^{-1} g over the jdone steps of the cycle (R: the rotated H).
__global__ __launch_bounds__(64) void batch_backsub_kernel(const BatchItem* __restrict__ items,
                                                           const BatchState* __restrict__ st,
                                                           int m) {
  const int i = blockIdx.x;
  const BatchState& S = st[i];
  if (threadIdx.x != 0 || S.done || S.jdone <= 0) return;
  const BatchItem& it = items[i];
  const int k = S.jdone, ldh = m + 1;
  for (int r = k - 1; r >= 0; --r) {
    double acc = it.g[r];
    for (int c = r + 1; c < k; ++c) acc -= it.H[r + (int64_t)c * ldh] * it.y[c];
    const double d = it.H[r + (int64_t)r * ldh];
    it.y[r] = d != 0.0 ? acc / d : 0.0;
  }
}

__global__ void batch_set_j_kernel(int* jp, int v) {
  if (threadIdx.x == 0) *jp = v;
}

__global__ void batch_advance_kernel(int* jp) {
  if (threadIdx.x == 0) *jp += 1;
}

}  // namespace

void batch_dots(const BatchItem* items, int count, int total_chunks, const BatchState* st,
                const int* jp, double* part, int ldp, int mode, hipStream_t s) {
  if (total_chunks <= 0) return;
  const dim3 g(total_chunks), b(kBT);
  switch (mode) {
    case BM_STEP:
      klaunch(batch_dots_kernel<BM_STEP>, g, b, 0, s, items, count, st, jp, part, ldp);
      break;
    case BM_PASS2:
      klaunch(batch_dots_kernel<BM_PASS2>, g, b, 0, s, items, count, st, jp, part, ldp);
      break;
    case BM_WNORM:
      klaunch(batch_dots_kernel<BM_WNORM>, g, b, 0, s, items, count, st, jp, part, ldp);
      break;
    case BM_RESID:
      klaunch(batch_dots_kernel<BM_RESID>, g, b, 0, s, items, count, st, jp, part, ldp);
      break;
    case BM_CNORM:
      klaunch(batch_dots_kernel<BM_CNORM>, g, b, 0, s, items, count, st, jp, part, ldp);
      break;
    default:
      throw Error(TSYLV_EINVAL, "batch_dots: mode");
  }
  TSYLV_LAUNCH_CHECK();
}

void batch_reduce(const BatchItem* items, int count, BatchState* st, const int* jp,
                  const double* part, int ldp, int mode, int m, double tol, int max_cycles,
                  hipStream_t s) {
  if (count <= 0) return;
  const dim3 g(count), b(64);
  switch (mode) {
#define TSYLV_REDUCE_CASE(M)                                                                  \
  case M:                                                                                     \
    klaunch(batch_reduce_kernel<M>, g, b, 0, s, items, st, jp, part, ldp, m, tol, \
                       max_cycles);                                                           \
    break;
    TSYLV_REDUCE_CASE(BM_STEP)
    TSYLV_REDUCE_CASE(BM_PASS2)
    TSYLV_REDUCE_CASE(BM_WNORM)
    TSYLV_REDUCE_CASE(BM_RESID)
    TSYLV_REDUCE_CASE(BM_RESID0)
    TSYLV_REDUCE_CASE(BM_CNORM)
#undef TSYLV_REDUCE_CASE
    default:
      throw Error(TSYLV_EINVAL, "batch_reduce: mode");
  }
  TSYLV_LAUNCH_CHECK();
}

void batch_update(const BatchItem* items, int count, int total_chunks, const BatchState* st,
                  const int* jp, int mode, hipStream_t s) {
  if (total_chunks <= 0) return;
  const dim3 g(total_chunks), b(kBT);
  if (mode == BM_STEP)
    klaunch(batch_update_kernel<BM_STEP>, g, b, 0, s, items, count, st, jp);
  else if (mode == BM_PASS2)
    klaunch(batch_update_kernel<BM_PASS2>, g, b, 0, s, items, count, st, jp);
  else if (mode == BM_XUPDATE)
    klaunch(batch_update_kernel<BM_XUPDATE>, g, b, 0, s, items, count, st, jp);
  else
    throw Error(TSYLV_EINVAL, "batch_update: mode");
  TSYLV_LAUNCH_CHECK();
}

void batch_scale(const BatchItem* items, int count, int total_chunks, const BatchState* st,
                 const int* jp, int mode, hipStream_t s) {
  if (total_chunks <= 0) return;
  const dim3 g(total_chunks), b(kBT);
  if (mode == BM_STEP)
    klaunch(batch_scale_kernel<BM_STEP>, g, b, 0, s, items, count, st, jp);
  else if (mode == BM_RESID)
    klaunch(batch_scale_kernel<BM_RESID>, g, b, 0, s, items, count, st, jp);
  else
    throw Error(TSYLV_EINVAL, "batch_scale: mode");
  TSYLV_LAUNCH_CHECK();
}

void batch_backsub(const BatchItem* items, int count, const BatchState* st, int m,
                   hipStream_t s) {
  if (count <= 0) return;
  klaunch(batch_backsub_kernel, dim3(count), dim3(64), 0, s, items, st, m);
  TSYLV_LAUNCH_CHECK();
}

void batch_set_j(int* jp, int value, hipStream_t s) {
  klaunch(batch_set_j_kernel, dim3(1), dim3(64), 0, s, jp, value);
  TSYLV_LAUNCH_CHECK();
}

void batch_advance(int* jp, hipStream_t s) {
  klaunch(batch_advance_kernel, dim3(1), dim3(64), 0, s, jp);
  TSYLV_LAUNCH_CHECK();
}

}  // namespace kern
}  // namespace tsylv
