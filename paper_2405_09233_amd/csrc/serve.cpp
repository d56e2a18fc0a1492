// Serving loop behind tsylv_submit / tsylv_poll: continuous batching of
// tGMRES / tFOM solves (project addition, not in the paper).
//
// A scheduler thread owns up to kSlots active solves, each a KrylovTask on its
// own HIP stream (default priority).  It loops:
//   1. admit queued requests in FIFO order while a slot is free and the
//      request's workspace fits in the arena (the HBM budget);
//   2. for every active solve: if no phase is in flight, enqueue its next
//      phase; if its stream has finished the phase (hipStreamQuery), run the
//      host step (Givens, LU, restart test) and enqueue the next phase at
//      once -- each solve advances at its own pace, not in lock step with
//      the slowest;
//   3. retire finished solves, freeing their slot and workspace.
// A request therefore joins while others are mid-solve and its work overlaps
// theirs.  Each solve runs exactly the kernels and host arithmetic of a
// synchronous call (the same KrylovTask; reductions are fixed-order), so its
// result is bitwise the same alone or in a mix.
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "krylov_task.hpp"
#include "runtime.hpp"
#include "serve.hpp"
#include "solvers.hpp"

namespace tsylv {

namespace {
constexpr int kSlots = 8;
// KrylovTask::pinned_doubles for m <= 1000 (a device-driven cycle, m <= 63,
// needs at most 7 * 65 + 2 + 65 * 64 + 2 of them)
constexpr size_t kPinnedPerSlot = 7 * (1000 + 2) + 2;
}  // namespace

struct Scheduler {
  Ctx& ctx;
  std::vector<hipStream_t> streams;
  double* pinned = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  struct Queued {
    uint64_t ticket;
    tsylv_request r;
  };
  std::deque<Queued> queue;
  struct Record {
    int status;
    tsylv_info info;
  };
  std::unordered_map<uint64_t, Record> done;
  uint64_t next_ticket = 1;
  bool stopping = false;

  struct Active {
    uint64_t ticket;
    int slot;
    std::unique_ptr<KrylovTask> task;
    int error = 0;
    bool in_flight = false;  // a phase is enqueued and not yet completed
  };
  std::vector<Active> active;
  std::vector<int> free_slots;

  explicit Scheduler(Ctx& c) : ctx(c) {
    streams.resize(kSlots, nullptr);
    for (int i = 0; i < kSlots; ++i) {
      TSYLV_HIP(hipStreamCreateWithFlags(&streams[i], hipStreamNonBlocking));
      free_slots.push_back(kSlots - 1 - i);
    }
    void* hp = nullptr;
    TSYLV_HIP(hipHostMalloc(&hp, kSlots * kPinnedPerSlot * sizeof(double), hipHostMallocDefault));
    pinned = static_cast<double*>(hp);
    th = std::thread([this]() { run(); });
  }

  ~Scheduler() {
    {
      std::lock_guard<std::mutex> g(mu);
      stopping = true;
      for (auto& q : queue) {
        tsylv_info inf{};
        inf.status = TSYLV_ECANCELLED;
        done[q.ticket] = {TSYLV_ECANCELLED, inf};
      }
      queue.clear();
    }
    cv.notify_all();
    if (th.joinable()) th.join();
    for (auto s : streams) (void)hipStreamDestroy(s);
    if (pinned) (void)hipHostFree(pinned);
  }

  void finish(uint64_t ticket, int status, const tsylv_info* inf) {
    tsylv_info i{};
    if (inf) i = *inf;
    i.status = status;
    std::lock_guard<std::mutex> g(mu);
    done[ticket] = {status, i};
  }

  // Admits queued requests (FIFO) while slots and arena memory allow.
  void admit() {
    std::unique_lock<std::mutex> lk(mu);
    while (!queue.empty() && !free_slots.empty()) {
      Queued q = queue.front();
      const size_t need = krylov_workspace_bytes(q.r.method, q.r.n, q.r.s, q.r.p, q.r.opts);
      if (need > ctx.arena.capacity()) {  // can never fit
        queue.pop_front();
        tsylv_info inf{};
        inf.status = TSYLV_ENOMEM;
        done[q.ticket] = {TSYLV_ENOMEM, inf};
        continue;
      }
      if (need > ctx.arena.largest_free()) break;  // wait for memory, keep FIFO order
      queue.pop_front();
      const int slot = free_slots.back();
      free_slots.pop_back();
      lk.unlock();
      Active a{q.ticket, slot, nullptr, 0};
      try {
        if (KrylovTask::pinned_doubles(q.r.opts) > kPinnedPerSlot)
          throw Error(TSYLV_EINVAL, "serve: restart length too large");
        a.task.reset(new KrylovTask(ctx, streams[slot], false, pinned + slot * kPinnedPerSlot,
                                    q.r.method, q.r.n, q.r.s, q.r.p, q.r.A, q.r.B, q.r.C, q.r.X,
                                    q.r.opts, q.r.A ? nullptr : &q.r.gen_seed));
      } catch (const Error& e) {
        if (e.status == TSYLV_ENOMEM) {  // fragmentation: retry later, at the head
          lk.lock();
          queue.push_front(q);
          free_slots.push_back(slot);
          break;
        }
        a.error = e.status;
      } catch (...) {
        a.error = TSYLV_EHIP;
      }
      active.push_back(std::move(a));
      lk.lock();
    }
  }

  void run() {
    (void)hipSetDevice(ctx.device);
    for (;;) {
      admit();
      {
        std::unique_lock<std::mutex> lk(mu);
        if (active.empty()) {
          if (stopping && queue.empty()) return;
          cv.wait(lk, [&]() { return stopping || !queue.empty(); });
          continue;
        }
      }
      bool progressed = false;
      for (auto& a : active) {
        if (a.error || !a.task) continue;
        try {
          if (a.in_flight) {
            const hipError_t q = hipStreamQuery(a.task->stream());
            if (q == hipErrorNotReady) continue;
            TSYLV_HIP(q);
            a.in_flight = false;
            a.task->complete();
            progressed = true;
          }
          if (!a.task->done()) {
            a.task->enqueue();
            a.in_flight = true;
            progressed = true;
          }
        } catch (const Error& e) {
          a.error = e.status;
        } catch (...) {
          a.error = TSYLV_EHIP;
        }
      }
      if (!progressed) std::this_thread::yield();
      // retire finished and failed solves; their workspace returns to the arena
      for (size_t i = 0; i < active.size();) {
        Active& a = active[i];
        const bool fin = a.error || (a.task && a.task->done());
        if (!fin) {
          ++i;
          continue;
        }
        if (a.error) {
          if (a.task) (void)hipStreamSynchronize(a.task->stream());
          finish(a.ticket, a.error, nullptr);
        } else {
          finish(a.ticket, a.task->status(), &a.task->info());
        }
        a.task.reset();
        {
          std::lock_guard<std::mutex> g(mu);
          free_slots.push_back(a.slot);
        }
        active.erase(active.begin() + (long)i);
      }
    }
  }
};

Scheduler* scheduler_create(Ctx& ctx) { return new Scheduler(ctx); }

void scheduler_destroy(Scheduler* s) { delete s; }

uint64_t scheduler_submit(Scheduler* s, const tsylv_request& r) {
  uint64_t t;
  {
    std::lock_guard<std::mutex> g(s->mu);
    t = s->next_ticket++;
    s->queue.push_back({t, r});
  }
  s->cv.notify_all();
  return t;
}

int scheduler_poll(Scheduler* s, uint64_t ticket, tsylv_info* info) {
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->done.find(ticket);
  if (it != s->done.end()) {
    if (info) *info = it->second.info;
    return it->second.status;
  }
  if (ticket == 0 || ticket >= s->next_ticket) return TSYLV_EINVAL;
  if (info) {
    *info = tsylv_info{};
    info->status = TSYLV_PENDING;
  }
  return TSYLV_PENDING;
}

}  // namespace tsylv
