#include "runtime.hpp"

namespace tsylv {

GraphRecorder*& graph_recorder() {
  static thread_local GraphRecorder* r = nullptr;
  return r;
}

void Arena::init(char* base, size_t bytes) {
  std::lock_guard<std::mutex> g(mu_);
  base_ = base;
  size_ = bytes;
  free_.clear();
  used_.clear();
  // keep the first block 256-byte aligned
  size_t skew = (size_t)((256 - ((uintptr_t)base % 256)) % 256);
  usable_ = bytes > skew ? bytes - skew : 0;
  if (usable_ > 0) free_[skew] = usable_;
}

void* Arena::alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (size_t)round_up((int64_t)bytes, 256);
  std::lock_guard<std::mutex> g(mu_);
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= bytes) {
      size_t off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > bytes) free_[off + bytes] = sz - bytes;
      used_[off] = bytes;
      return base_ + off;
    }
  }
  return nullptr;
}

void Arena::free(void* ptr) {
  if (!ptr) return;
  std::lock_guard<std::mutex> g(mu_);
  size_t off = (size_t)((char*)ptr - base_);
  auto it = used_.find(off);
  if (it == used_.end()) return;
  size_t sz = it->second;
  used_.erase(it);
  auto nx = free_.lower_bound(off);
  if (nx != free_.end() && off + sz == nx->first) {  // merge with next
    sz += nx->second;
    nx = free_.erase(nx);
  }
  if (nx != free_.begin()) {  // merge with previous
    auto pv = std::prev(nx);
    if (pv->first + pv->second == off) {
      pv->second += sz;
      return;
    }
  }
  free_[off] = sz;
}

size_t Arena::in_use() const {
  std::lock_guard<std::mutex> g(mu_);
  size_t t = 0;
  for (auto& kv : used_) t += kv.second;
  return t;
}

size_t Arena::largest_free() const {
  std::lock_guard<std::mutex> g(mu_);
  size_t m = 0;
  for (auto& kv : free_) m = kv.second > m ? kv.second : m;
  return m;
}

Workspace::Workspace(Arena& arena, size_t bytes) : arena_(arena), bytes_(bytes) {
  base_ = static_cast<char*>(arena_.alloc(bytes));
  if (!base_) throw Error(TSYLV_ENOMEM, "arena too small for the workspace");
}

Workspace::~Workspace() { arena_.free(base_); }

double* Ctx::task_buffer(size_t count) {
  if (count > task_pinned_count) {
    if (task_pinned) TSYLV_HIP(hipHostFree(task_pinned));
    task_pinned = nullptr;
    task_pinned_count = 0;
    void* h = nullptr;
    TSYLV_HIP(hipHostMalloc(&h, count * sizeof(double), hipHostMallocDefault));
    task_pinned = static_cast<double*>(h);
    task_pinned_count = count;
  }
  return task_pinned;
}

double* Ctx::host_buffer(size_t count) {
  if (count > pinned_count)
    throw Error(TSYLV_EINVAL, "host staging buffer too small (restart length too large)");
  return pinned;
}

Profiler::~Profiler() {
  for (auto e : pool_) (void)hipEventDestroy(e);
}

void Profiler::enable(unsigned mask) {
  const bool on = mask != 0;
  if (on) {
    if (pool_.empty()) {
      pool_.resize(8192);
      for (auto& e : pool_) TSYLV_HIP(hipEventCreate(&e));
    }
    pending_.clear();
    next_ = 0;
    for (int k = 0; k < TSYLV_K_COUNT; ++k) {
      launches_[k] = 0;
      ms_[k] = 0.0;
    }
  } else {
    fold();
  }
  mask_ = mask;
}

void Profiler::fold() {
  if (pending_.empty()) {
    next_ = 0;
    return;
  }
  TSYLV_HIP(hipEventSynchronize(pending_.back().b));
  for (auto& pe : pending_) {
    float ms = 0.0f;
    TSYLV_HIP(hipEventElapsedTime(&ms, pe.a, pe.b));
    ms_[pe.kid] += ms;
    launches_[pe.kid] += 1;
  }
  pending_.clear();
  next_ = 0;
}

void Profiler::begin(int kid, hipStream_t st) {
  if (next_ + 2 > pool_.size()) fold();
  hipEvent_t a = pool_[next_++];
  TSYLV_HIP(hipEventRecord(a, st));
  cur_start_[kid] = a;
}

void Profiler::end(int kid, hipStream_t st) {
  hipEvent_t b = pool_[next_++];
  TSYLV_HIP(hipEventRecord(b, st));
  pending_.push_back({kid, cur_start_[kid], b});
}

void Profiler::read(int kid, int64_t& launches, double& ms) {
  fold();
  launches = launches_[kid];
  ms = ms_[kid];
}

}  // namespace tsylv
