// Context, HBM arena and pinned host staging.
#pragma once

#include <array>
#include <map>
#include <string>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace tsylv {

// First-fit allocator over the caller's device buffer.  Every workspace of
// the library comes from here: the arena size is the HBM budget.  Offsets
// are 256-byte aligned.  Thread-safe.
class Arena {
 public:
  Arena() = default;
  void init(char* base, size_t bytes);
  // Returns nullptr when no free block is large enough.
  void* alloc(size_t bytes);
  void free(void* ptr);
  // Usable bytes: the buffer minus the skew that aligns its first block.
  size_t capacity() const { return usable_; }
  size_t in_use() const;
  size_t largest_free() const;

 private:
  char* base_ = nullptr;
  size_t size_ = 0;
  size_t usable_ = 0;
  std::map<size_t, size_t> free_;  // offset -> size
  std::map<size_t, size_t> used_;  // offset -> size
  mutable std::mutex mu_;
};

// Bump allocator on top of one arena block: the workspace of one solve.
class Workspace {
 public:
  Workspace(Arena& arena, size_t bytes);
  ~Workspace();
  Workspace(const Workspace&) = delete;
  Workspace& operator=(const Workspace&) = delete;
  template <typename T>
  T* take(int64_t count) {
    size_t b = (size_t)round_up((int64_t)(count * sizeof(T)), 256);
    if (used_ + b > bytes_) throw Error(TSYLV_ENOMEM, "workspace plan exceeded");
    T* p = reinterpret_cast<T*>(base_ + used_);
    used_ += b;
    return p;
  }
  static size_t bytes_for(int64_t count, size_t elem) {
    return (size_t)round_up((int64_t)(count * elem), 256);
  }

 private:
  Arena& arena_;
  char* base_ = nullptr;
  size_t bytes_ = 0;
  size_t used_ = 0;
};

// Bump allocator over a device buffer the caller provides (no arena): the
// scratch of the allocation-free entry points.
class Carve {
 public:
  Carve(char* base, size_t bytes) : base_(base), bytes_(bytes) {}
  template <typename T>
  T* take(int64_t count) {
    size_t b = (size_t)round_up((int64_t)(count * sizeof(T)), 256);
    if (used_ + b > bytes_) throw Error(TSYLV_ENOMEM, "scratch plan exceeded");
    T* p = reinterpret_cast<T*>(base_ + used_);
    used_ += b;
    return p;
  }

 private:
  char* base_;
  size_t bytes_;
  size_t used_ = 0;
};

struct Scheduler;  // serving loop (serve.cpp)

// HIP-event timing of kernel families (tsylv_profile).
class Profiler {
 public:
  ~Profiler();
  // mask: bit k times family k (0 stops timing)
  void enable(unsigned mask);
  bool on() const { return mask_ != 0; }
  bool on(int kid) const { return (mask_ >> kid) & 1u; }
  void begin(int kid, hipStream_t st);
  void end(int kid, hipStream_t st);
  void read(int kid, int64_t& launches, double& ms);

 private:
  void fold();  // sync on the recorded events and accumulate
  unsigned mask_ = 0;
  std::vector<hipEvent_t> pool_;
  size_t next_ = 0;
  struct Pending { int kid; hipEvent_t a, b; };
  std::vector<Pending> pending_;
  hipEvent_t cur_start_[TSYLV_K_COUNT] = {};
  int64_t launches_[TSYLV_K_COUNT] = {};
  double ms_[TSYLV_K_COUNT] = {};
};

// Tile choices of the facewise apply per (precision, n, s, p), filled by
// the autotuner (tune.cpp) or set by the caller; thread-safe.  get() returns
// -1 (the default for s) for a shape with no entry.
class TuneTable {
 public:
  int get(int prec, int64_t n, int64_t s, int64_t p) const;
  void set(int prec, int64_t n, int64_t s, int64_t p, int variant);  // -1 erases
  size_t size() const;
  // Text form: a header line, then one "prec n s p variant" line per entry.
  std::string serialize() const;
  void parse(const std::string& text);  // validates everything before it adds

 private:
  std::map<std::array<int64_t, 4>, int> m_;
  mutable std::mutex mu_;
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool owns_arena = false;
  void* arena_ptr = nullptr;
  Arena arena;
  // pinned host staging for small device->host results
  double* pinned = nullptr;
  size_t pinned_count = 0;
  Scheduler* sched = nullptr;  // created by the first tsylv_submit
  std::mutex sched_mu;
  std::mutex sync_mu;  // serialises synchronous calls on the context
  Profiler prof;
  TuneTable tune;

  // pinned host staging of the batch's stream executor (created on first
  // use, kept until the context is destroyed)
  double* task_pinned = nullptr;
  size_t task_pinned_count = 0;

  double* host_buffer(size_t count);  // grows the pinned buffer as needed
  double* task_buffer(size_t count);
  void sync() { TSYLV_HIP(hipStreamSynchronize(stream)); }
};

// Brackets kernel launches on stream `st` with profiling events when
// profiling is on and `enabled` (the serving loop's tasks never time).
struct ProfScope {
  Ctx& c;
  int kid;
  hipStream_t st;
  bool on;
  ProfScope(Ctx& ctx, int k, hipStream_t s, bool enabled = true)
      : c(ctx), kid(k), st(s), on(enabled && ctx.prof.on(k)) {
    if (on) c.prof.begin(kid, st);
  }
  ~ProfScope() {
    if (on) c.prof.end(kid, st);
  }
};

}  // namespace tsylv
