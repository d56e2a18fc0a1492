// A resumable tGMRES / tFOM solve (Algorithm 3, optionally inside FP64
// iterative refinement).  The synchronous entry points and the serving loop
// drive the same object, so a solve computes the same bits whether it runs
// alone or next to others:
//     while (!t.done()) { t.enqueue(); <synchronise t's stream>; t.complete(); }
// enqueue() puts the next phase's kernels on the task's stream; complete()
// reads the small results back (FP64 Givens / LU on the host) and picks the
// next phase.
#pragma once

#include <chrono>
#include <memory>
#include <vector>

#include "runtime.hpp"

namespace tsylv {

struct KrylovState;  // device buffers and host bookkeeping (solver_krylov.cpp)

class KrylovTask {
 public:
  // Validated arguments; the workspace is taken from `arena` here (throws
  // TSYLV_ENOMEM if it does not fit).  `pinned` must hold pinned_doubles(o)
  // doubles of page-locked host memory owned by the caller.  With `gen`
  // non-null, A, B and C are ignored and the synthetic instance of seed
  // *gen is drawn on the device inside the setup transforms (p <= 64).
  KrylovTask(Ctx& ctx, hipStream_t st, bool profile, double* pinned, int method, int64_t n,
             int64_t s, int64_t p, const double* A, const double* B, const double* C, double* X,
             const tsylv_opts& o, const uint64_t* gen = nullptr);
  ~KrylovTask();
  KrylovTask(const KrylovTask&) = delete;
  KrylovTask& operator=(const KrylovTask&) = delete;

  static size_t pinned_doubles(const tsylv_opts& o);

  void enqueue();
  void complete();
  bool done() const;
  int status() const;
  const tsylv_info& info() const;
  hipStream_t stream() const;

 private:
  std::unique_ptr<KrylovState> s_;
};

}  // namespace tsylv
