// Internal definitions shared by the HIP kernels and the C++ drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <tuple>
#include <utility>

#include "../../include/tsylv.h"

namespace tsylv {

// Error carried from deep inside a driver to the C-ABI boundary, where it is
// turned into a status code.
struct Error : public std::runtime_error {
  int status;
  Error(int st, const std::string& msg) : std::runtime_error(msg), status(st) {}
};

#define TSYLV_HIP(call)                                                        \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      throw ::tsylv::Error(TSYLV_EHIP, std::string(#call) + ": " +             \
                                           hipGetErrorString(e_));            \
  } while (0)

#define TSYLV_LAUNCH_CHECK() TSYLV_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// Fourier half-spectrum plane layout.
//
// A real tensor with p frontal slices has a mode-3 DFT that is conjugate
// symmetric (Fhat_{p-k} = conj(Fhat_k)), so slices k = 0 .. floor(p/2) carry
// all of it.  Slice 0 and, for even p, slice p/2 are real; the others are
// complex.  We store them as exactly p real "planes", each a rows x cols
// column-major matrix:
//     plane 0              Re(slice 0)
//     planes 2k-1, 2k      Re(slice k), Im(slice k)     1 <= k < p/2
//     plane p-1            Re(slice p/2)                (p even only)
// so a Fourier tensor has the same number of reals as the spatial one.
// ---------------------------------------------------------------------------
__host__ __device__ inline int num_slices(int p) { return p / 2 + 1; }

__host__ __device__ inline void slice_planes(int p, int k, int& qr, int& qi) {
  if (k == 0) {
    qr = 0;
    qi = -1;
  } else if (2 * k == p) {
    qr = p - 1;
    qi = -1;
  } else {
    qr = 2 * k - 1;
    qi = 2 * k;
  }
}

// Transform kinds for the p x p tube-transform matrix (see build_xform).
enum XformKind {
  XF_OPERATOR = 0,  // unscaled DFT planes (for A and B)
  XF_FORWARD = 1,   // orthonormal real DFT (vectors: spatial -> planes)
  XF_INVERSE = 2    // its transpose (planes -> spatial)
};

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Kernel launches that can be recorded into a graph instead of enqueued.
// While a GraphRecorder is installed on the calling thread, klaunch adds a
// kernel node behind the previous one (the nodes form a chain, the order of
// the launches) and enqueues nothing; otherwise it launches on `st`.  A
// graph built this way involves no stream capture, so work that other
// threads issue meanwhile (on the legacy default stream, say) cannot
// invalidate it.
struct GraphRecorder {
  hipGraph_t graph = nullptr;
  hipGraphNode_t last = nullptr;
};
GraphRecorder*& graph_recorder();  // the calling thread's recorder (or null)

template <typename Tuple, size_t... I>
inline void kparam_ptrs(Tuple& t, void** out, std::index_sequence<I...>) {
  ((out[I] = static_cast<void*>(&std::get<I>(t))), ...);
}

template <typename... P, typename... A>
inline void klaunch(void (*kernel)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t st,
                    A&&... args) {
  GraphRecorder* r = graph_recorder();
  if (!r) {
    hipLaunchKernelGGL(kernel, grid, block, lds, st, std::forward<A>(args)...);
    return;
  }
  std::tuple<P...> vals(std::forward<A>(args)...);
  void* ptrs[sizeof...(P) + 1];
  kparam_ptrs(vals, ptrs, std::index_sequence_for<P...>{});
  hipKernelNodeParams np{};
  np.func = reinterpret_cast<void*>(kernel);
  np.gridDim = grid;
  np.blockDim = block;
  np.sharedMemBytes = (unsigned)lds;
  np.kernelParams = ptrs;
  np.extra = nullptr;
  hipGraphNode_t node = nullptr;
  TSYLV_HIP(hipGraphAddKernelNode(&node, r->graph, r->last ? &r->last : nullptr,
                                  r->last ? 1 : 0, &np));
  r->last = node;
}

}  // namespace tsylv
