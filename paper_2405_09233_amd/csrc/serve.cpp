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
// theirs.  tsylv_submit records an event on the context stream; the slot's
// stream waits on it before the request's first kernel, so work the caller
// enqueued on that stream before submitting (filling A, B, C or X0) is
// finished when the solve reads its inputs.  Each solve runs exactly the
// kernels and host arithmetic of a synchronous call (the same KrylovTask;
// reductions are fixed-order), so its result is bitwise the same alone or in
// a mix.
//
// Requests of method GMRES_BATCHED, and tGMRES requests small enough for the
// single-workgroup solve, that wait at the head of the queue with equal
// options are admitted together, up to kMaxBatch of them and as many as
// the arena holds, as one batch (batch.cpp, without its stream executor)
// that takes one slot and runs on a worker thread on the slot's stream:
// instances that fit one workgroup in one launch, the others in lockstep,
// the lockstep step replayed from a graph of kernel nodes recorded on the
// worker (no stream capture, so the caller's concurrent work on the legacy
// default stream cannot interfere); the scheduler posts every result of the
// batch when the worker ends.  An instance's result in a batch is bitwise
// its batch-of-one result (graph or eager: the same kernels).
#include <atomic>
#include <cstdlib>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "krylov_task.hpp"
#include "runtime.hpp"
#include "sched_policy.hpp"
#include "serve.hpp"
#include "solvers.hpp"

namespace tsylv {

namespace {
constexpr int kSlots = 8;
// KrylovTask::pinned_doubles for m <= 1000 (a device-driven cycle, m <= 63,
// needs at most 7 * 65 + 2 + 65 * 64 + 2 of them)
constexpr size_t kPinnedPerSlot = 7 * (1000 + 2) + 2;
constexpr int kMaxBatch = 512;

bool same_batch_opts(const tsylv_opts& a, const tsylv_opts& b) {
  return a.m == b.m && a.tol == b.tol && a.max_cycles == b.max_cycles &&
         a.x0_given == b.x0_given;
}

// Requests that join batches: GMRES_BATCHED ones, and tGMRES requests whose
// instance a batch solves whole in one workgroup (the same kernel as their
// single solve, so the same bits, with many instances per launch).
bool batch_request(const tsylv_request& r) {
  if (r.method == TSYLV_METHOD_GMRES_BATCHED) return true;
  return r.method == TSYLV_METHOD_GMRES && !r.opts.refine && r.opts.m <= kern::kBatchMaxM &&
         batch_solves_whole(tsylv_problem{r.n, r.s, r.p, r.A, r.B, r.C, r.X}, r.opts);
}

// A batch of requests (GMRES_BATCHED, small tGMRES), run by a worker thread.
struct BatchJob {
  std::vector<uint64_t> tickets;
  std::vector<tsylv_request> reqs;
  std::vector<hipEvent_t> ready;  // the requests' submit events
  std::vector<tsylv_problem> probs;
  std::vector<const uint64_t*> gens;
  std::vector<tsylv_info> infos;
  // The batch's workspace, reserved from the context's arena when the batch
  // is admitted (so that batches admitted one after another cannot count on
  // the same free memory before their workers allocate), carved by `sub`.
  void* block = nullptr;
  Arena sub;
  std::thread th;
  std::atomic<bool> finished{false};
  int error = 0;  // an error of the whole batch
};
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
    hipEvent_t ready;  // recorded on the context stream at submit
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
    hipEvent_t ready = nullptr;  // the submit event (destroyed at retirement)
    bool in_flight = false;  // a phase is enqueued and not yet completed
    std::unique_ptr<BatchJob> job;  // a batch instead of one task
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
        if (q.ready) (void)hipEventDestroy(q.ready);
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

  // Admits queued requests while slots and arena memory allow, as the
  // admission policy (sched_policy.hpp) decides.
  void admit() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      // the batched requests at the head as problems, for the batch sizes
      std::vector<tsylv_problem> probs;
      for (size_t i = 0; i < queue.size() && (int)i < kMaxBatch && batch_request(queue[i].r);
           ++i) {
        const tsylv_request& r = queue[i].r;
        probs.push_back(tsylv_problem{r.n, r.s, r.p, r.A, r.B, r.C, r.X});
      }
      policy::QueueView v;
      v.size = queue.size();
      v.batched = [&](size_t i) { return batch_request(queue[i].r); };
      v.batchable = [&](size_t i, size_t j) {
        return same_batch_opts(queue[i].r.opts, queue[j].r.opts);
      };
      v.need_single = [&](size_t i) {
        const tsylv_request& r = queue[i].r;
        return krylov_workspace_bytes(r.method, r.n, r.s, r.p, r.opts);
      };
      v.need_batch = [&](size_t k) {
        return served_batch_bytes((int)k, probs.data(), queue.front().r.opts);
      };
      const policy::Decision d = policy::next_admission(
          v, free_slots.size(), ctx.arena.largest_free(), ctx.arena.capacity(), kMaxBatch);
      if (d.kind == policy::Kind::Wait) return;
      if (d.kind == policy::Kind::Reject) {
        tsylv_info inf{};
        inf.status = TSYLV_ENOMEM;
        done[queue.front().ticket] = {TSYLV_ENOMEM, inf};
        if (queue.front().ready) (void)hipEventDestroy(queue.front().ready);
        queue.pop_front();
        continue;
      }
      if (d.kind == policy::Kind::Batch) {
        if (!start_batch(lk, d.count, probs)) return;  // memory taken meanwhile: wait
        continue;
      }
      Queued q = queue.front();
      queue.pop_front();
      const int slot = free_slots.back();
      free_slots.pop_back();
      lk.unlock();
      Active a{q.ticket, slot, nullptr, 0};
      a.ready = q.ready;
      try {
        if (KrylovTask::pinned_doubles(q.r.opts) > kPinnedPerSlot)
          throw Error(TSYLV_EINVAL, "serve: restart length too large");
        // the caller's work on the context stream before submit comes first
        // (the task's constructor already enqueues the setup transforms)
        if (a.ready) TSYLV_HIP(hipStreamWaitEvent(streams[slot], a.ready, 0));
        a.task.reset(new KrylovTask(ctx, streams[slot], false, pinned + slot * kPinnedPerSlot,
                                    q.r.method, q.r.n, q.r.s, q.r.p, q.r.A, q.r.B, q.r.C, q.r.X,
                                    q.r.opts, q.r.A ? nullptr : &q.r.gen_seed));
      } catch (const Error& e) {
        // Fragmentation or a synchronous call holding arena memory: retry
        // later, at the head, while other solves run (they return memory);
        // with none active nothing would change, so the request fails.
        if (e.status == TSYLV_ENOMEM && !active.empty()) {
          a.task.reset();
          lk.lock();
          queue.push_front(q);
          free_slots.push_back(slot);
          return;
        }
        a.error = e.status;
      } catch (...) {
        a.error = TSYLV_EHIP;
      }
      active.push_back(std::move(a));
      lk.lock();
    }
  }

  // The first `count` requests of the queue (batched, with equal options;
  // probs their problems) become one batch on a free slot, its workspace
  // reserved at once.  Called with mu held (lk); returns with it held;
  // false (nothing started) when the reservation fails.
  bool start_batch(std::unique_lock<std::mutex>& lk, size_t count,
                   const std::vector<tsylv_problem>& probs) {
    const tsylv_opts o = queue.front().r.opts;
    const size_t need = served_batch_bytes((int)count, probs.data(), o);
    void* block = ctx.arena.alloc(need);
    if (!block) return false;
    std::unique_ptr<BatchJob> job(new BatchJob());
    job->block = block;
    job->sub.init(static_cast<char*>(block), need);
    for (size_t i = 0; i < count; ++i) {
      const tsylv_request& r = queue.front().r;
      job->tickets.push_back(queue.front().ticket);
      job->reqs.push_back(r);
      job->ready.push_back(queue.front().ready);
      job->probs.push_back(tsylv_problem{r.n, r.s, r.p, r.A, r.B, r.C, r.X});
      queue.pop_front();
    }
    job->infos.resize(count);
    for (size_t i = 0; i < count; ++i)
      job->gens.push_back(job->reqs[i].A ? nullptr : &job->reqs[i].gen_seed);
    const int slot = free_slots.back();
    free_slots.pop_back();
    lk.unlock();
    BatchJob* jp = job.get();
    hipStream_t st = streams[slot];
    jp->th = std::thread([this, jp, st, o]() {
      try {
        TSYLV_HIP(hipSetDevice(ctx.device));
        for (hipEvent_t e : jp->ready)
          if (e) TSYLV_HIP(hipStreamWaitEvent(st, e, 0));
        // the step replayed from a recorded graph (TSYLV_BATCH_GRAPH=0: eager)
        const char* g = std::getenv("TSYLV_BATCH_GRAPH");
        gmres_batch(ctx, st, (int)jp->probs.size(), jp->probs.data(), jp->gens.data(), o,
                    jp->infos.data(), !(g && g[0] == '0'), /*no_streams=*/true, &jp->sub);
      } catch (const Error& e) {
        jp->error = e.status;
      } catch (...) {
        jp->error = TSYLV_EHIP;
      }
      jp->finished.store(true);
    });
    Active a{jp->tickets[0], slot, nullptr, 0};
    a.job = std::move(job);
    active.push_back(std::move(a));
    lk.lock();
    return true;
  }

  // A finished batch: every result posted (an arena shortfall puts the
  // requests back at the head of the queue instead).
  void retire_batch(Active& a) {
    BatchJob& j = *a.job;
    if (j.th.joinable()) j.th.join();
    (void)hipStreamSynchronize(streams[a.slot]);
    ctx.arena.free(j.block);
    j.block = nullptr;
    if (j.error == TSYLV_ENOMEM && active.size() > 1) {  // others hold memory: retry
      std::lock_guard<std::mutex> g(mu);
      if (!stopping) {
        for (size_t i = j.tickets.size(); i-- > 0;)
          queue.push_front({j.tickets[i], j.reqs[i], j.ready[i]});
        return;
      }
    }
    for (hipEvent_t e : j.ready)
      if (e) (void)hipEventDestroy(e);
    for (size_t i = 0; i < j.tickets.size(); ++i) {
      if (j.error)
        finish(j.tickets[i], j.error, nullptr);
      else
        finish(j.tickets[i], j.infos[i].status, &j.infos[i]);
    }
  }

  void run() {
    (void)hipSetDevice(ctx.device);
    int idle_passes = 0;
    for (;;) {
      admit();
      {
        std::unique_lock<std::mutex> lk(mu);
        if (active.empty()) {
          if (stopping && queue.empty()) return;
          if (queue.empty())
            cv.wait(lk, [&]() { return stopping || !queue.empty(); });
          else  // the head waits for memory held outside the loop: back off
            cv.wait_for(lk, std::chrono::microseconds(200));
          continue;
        }
      }
      bool progressed = false;
      for (auto& a : active) {
        if (a.job) continue;
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
      // nothing ready: yield, and after a while of nothing back off briefly
      // (a phase takes tens of microseconds at least) instead of spinning
      if (progressed) {
        idle_passes = 0;
      } else if (++idle_passes < 256) {
        std::this_thread::yield();
      } else {
        std::this_thread::sleep_for(std::chrono::microseconds(20));
      }
      // retire finished and failed solves; their workspace returns to the arena
      for (size_t i = 0; i < active.size();) {
        Active& a = active[i];
        if (a.job) {
          if (!a.job->finished.load()) {
            ++i;
            continue;
          }
          retire_batch(a);
          {
            std::lock_guard<std::mutex> g(mu);
            free_slots.push_back(a.slot);
          }
          active.erase(active.begin() + (long)i);
          continue;
        }
        const bool fin = a.error || (a.task && a.task->done());
        if (!fin) {
          ++i;
          continue;
        }
        if (a.error) {
          (void)hipStreamSynchronize(streams[a.slot]);
          finish(a.ticket, a.error, nullptr);
        } else {
          finish(a.ticket, a.task->status(), &a.task->info());
        }
        a.task.reset();
        if (a.ready) (void)hipEventDestroy(a.ready);
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
  hipEvent_t ev = nullptr;
  TSYLV_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  const hipError_t er = hipEventRecord(ev, s->ctx.stream);
  if (er != hipSuccess) {
    (void)hipEventDestroy(ev);
    TSYLV_HIP(er);
  }
  uint64_t t;
  {
    std::lock_guard<std::mutex> g(s->mu);
    t = s->next_ticket++;
    s->queue.push_back({t, r, ev});
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
