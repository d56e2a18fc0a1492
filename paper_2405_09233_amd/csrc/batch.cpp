// Batched lockstep tGMRES(m) over many independent instances (a project
// addition for workloads of many uneven solves; the method per instance is
// Algorithm 3 with the Arnoldi process of Algorithm 2 -- classical
// Gram-Schmidt applied twice -- and the Givens least-squares update of
// section 3.3).
//
// Every instance keeps its Fourier-domain state (operator planes, basis,
// Hessenberg matrix, rotations) on the device.  One Arnoldi step of the whole
// batch is a fixed sequence of launches, each covering every instance:
//   apply (one launch per tile variant present)  W = M(V_j)
//   dots / reduce / update                       W -= V (V^T W), and ||W||^2
//   dots / reduce / update, where needed         the same again (second pass)
//   dots / reduce                                ||W|| (second-pass instances),
//                                                Givens, stop test
//   scale                                        V_{j+1} = W / ||W||
//   advance                                      j += 1 (device counter)
// Since j lives in device memory, the step is recorded once as a HIP graph
// (kernel nodes added directly, no stream capture) and replayed m times per
// cycle; the host reads the instances' flags every
// kCheckEvery steps to end a cycle early when no instance is stepping.  At
// a cycle's end: y = R^{-1} g, X += V y, the true residual R = C - M(X), and
// the restart test of Algorithm 3 -- again one launch each for the batch.
// The batch can be split into up to kGroups groups of balanced apply work,
// each with its own tables, stream and graph, so that the applies of one
// group could run beside the Gram-Schmidt sweeps of another; an instance's
// arithmetic is the same in any group.  Measured with four groups: no gain
// on 64 instances of n up to 2048 (each group's apply grid already fills
// the GPU) and slower small batches (more launches), so one group is used.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <thread>
#include <vector>

#include "kernels.hpp"
#include "krylov_task.hpp"
#include "runtime.hpp"
#include "solvers.hpp"

namespace tsylv {

namespace {

constexpr int kCheckEvery = 8;
constexpr int kVariants = 3;
// the apply tile variants a batch uses (the FP64 defaults by s), by slot
constexpr int kVariantIds[kVariants] = {9, 1, 2};

int variant_slot(int v) {
  for (int k = 0; k < kVariants; ++k)
    if (kVariantIds[k] == v) return k;
  throw Error(TSYLV_EINVAL, "batch: tile variant without a slot");
}
constexpr int kGroups = 1;  // independent lockstep groups per batch (see above)

struct BatchPlan {
  int count = 0, m = 0;
  int total_chunks = 0;
  int ldp = 0;
  int ntiles[kVariants] = {0, 0, 0};
  std::vector<kern::BatchApplyRef> refs[kVariants];
};

int64_t chunks_of(int64_t N) { return (N + kern::kBatchChunk - 1) / kern::kBatchChunk; }

size_t instance_bytes(int64_t n, int64_t s, int64_t p, int m) {
  const int64_t N = n * s * p;
  const int64_t ldv = (N + 63) / 64 * 64;
  return setup_bytes(n, s, p) + Workspace::bytes_for((m + 1) * ldv, 8) +
         Workspace::bytes_for(N, 8) + Workspace::bytes_for((int64_t)(m + 1) * m, 8) +
         5 * Workspace::bytes_for(m + 1, 8);
}

}  // namespace

size_t lockstep_workspace_bytes(int count, const tsylv_problem* probs,
                                       const tsylv_opts& o) {
  if (count <= 0) return 0;
  size_t b = 0;
  int64_t chunks = 0;
  for (int i = 0; i < count; ++i) {
    b += instance_bytes(probs[i].n, probs[i].s, probs[i].p, o.m);
    chunks += chunks_of(probs[i].n * probs[i].s * probs[i].p);
  }
  b += Workspace::bytes_for((int64_t)count, sizeof(kern::BatchItem)) +
       Workspace::bytes_for((int64_t)count, sizeof(kern::BatchState)) +
       Workspace::bytes_for(chunks * (o.m + 3), 8) +
       kVariants * Workspace::bytes_for((int64_t)count, sizeof(kern::BatchApplyRef)) +
       Workspace::bytes_for(1, sizeof(int));
  // each group rounds its own seven tables up to 256 bytes
  b += (size_t)std::min(kGroups, count) * (kVariants + 4) * 256;
  return b;
}

namespace {

// One lockstep group: its own tables, reduction buffer, step counter,
// stream and captured step.  The groups of a batch are independent, so
// their launches overlap on the device (the MFMA-bound applies of one group
// beside the HBM-bound Gram-Schmidt sweeps of another).
struct Group {
  std::vector<int> ids;                 // instances (indices into the batch)
  std::vector<kern::BatchItem> items;
  BatchPlan plan;
  kern::BatchItem* d_items = nullptr;
  kern::BatchState* d_state = nullptr;
  double* d_part = nullptr;
  kern::BatchApplyRef* d_refs[kVariants] = {nullptr, nullptr, nullptr};
  int* d_j = nullptr;
  hipStream_t stream = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<kern::BatchState> flags;
  bool live = true;      // some instance not done
  bool stepping = true;  // some instance stepping in the current cycle
};

}  // namespace

static int gmres_lockstep(Ctx& ctx, Arena& arena, hipStream_t st, int count,
                          const tsylv_problem* probs, const uint64_t* const* gens,
                          const tsylv_opts& o, tsylv_info* infos, bool use_graph) {
  const auto t0 = std::chrono::steady_clock::now();
  const int m = o.m;

  // ---- groups: up to kGroups, balanced by apply work (n^2 s p) ----
  const int ngroups = std::min(kGroups, count);
  std::vector<Group> groups(ngroups);
  {
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    auto work = [&](int i) { return (double)probs[i].n * probs[i].n * probs[i].s * probs[i].p; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
    std::vector<double> load(ngroups, 0.0);
    for (int i : order) {
      int g = 0;
      for (int h = 1; h < ngroups; ++h)
        if (load[h] < load[g]) g = h;
      load[g] += work(i);
      groups[g].ids.push_back(i);
    }
    for (auto& G : groups) std::sort(G.ids.begin(), G.ids.end());
  }

  // ---- workspace and per-instance setup (Algorithm 1 step 1) ----
  Workspace ws(arena, lockstep_workspace_bytes(count, probs, o));
  // on any exit, let every stream drain before the workspace returns to the
  // arena, then release the groups' streams and graphs
  struct Drain {
    hipStream_t s;
    std::vector<Group>* gs;
    ~Drain() {
      (void)hipStreamSynchronize(s);
      for (auto& G : *gs) {
        if (G.stream) (void)hipStreamSynchronize(G.stream);
        if (G.exec) (void)hipGraphExecDestroy(G.exec);
        if (G.stream) (void)hipStreamDestroy(G.stream);
      }
    }
  } drain{st, &groups};
  std::vector<Setup> setups(count);
  std::vector<kern::BatchItem> all(count);
  for (int i = 0; i < count; ++i) {
    const tsylv_problem& q = probs[i];
    const int64_t N = q.n * q.s * q.p;
    const int64_t ldv = (N + 63) / 64 * 64;
    Setup S = setup_fourier(ctx, st, false, ws, q.n, q.s, q.p, q.A, q.B, q.C, q.X,
                            o.x0_given != 0, gens ? gens[i] : nullptr);
    setups[i] = S;
    kern::BatchItem& it = all[i];
    it.Ah = S.Ah;
    it.Bh = S.Bh;
    it.Zc = S.Zc;
    it.Zx = S.Zx;
    it.V = ws.take<double>((m + 1) * ldv);
    it.W = ws.take<double>(N);
    it.H = ws.take<double>((int64_t)(m + 1) * m);
    it.cs = ws.take<double>(m + 1);
    it.sn = ws.take<double>(m + 1);
    it.g = ws.take<double>(m + 1);
    it.y = ws.take<double>(m + 1);
    it.coef = ws.take<double>(m + 1);
    it.n = q.n;
    it.s = q.s;
    it.N = N;
    it.ldv = ldv;
    it.p = (int)q.p;
  }
  for (auto& G : groups) {
    const int gc = (int)G.ids.size();
    G.plan.count = gc;
    G.plan.m = m;
    G.plan.ldp = m + 3;
    int64_t chunk0 = 0;
    for (int k = 0; k < gc; ++k) {
      const tsylv_problem& q = probs[G.ids[k]];
      kern::BatchItem it = all[G.ids[k]];
      it.chunk0 = (int)chunk0;
      it.nchunks = (int)chunks_of(it.N);
      chunk0 += it.nchunks;
      G.items.push_back(it);
      const int vid = kern::batch_apply_variant(q.s), v = variant_slot(vid);
      kern::BatchApplyRef r;
      r.item = k;
      r.tile0 = G.plan.ntiles[v];
      G.plan.ntiles[v] += kern::batch_apply_tiles(vid, q.n, q.s, (int)q.p, &r.nrt, &r.nct);
      G.plan.refs[v].push_back(r);
    }
    G.plan.total_chunks = (int)chunk0;
    G.d_items = ws.take<kern::BatchItem>(gc);
    G.d_state = ws.take<kern::BatchState>(gc);
    G.d_part = ws.take<double>((int64_t)G.plan.total_chunks * G.plan.ldp);
    for (int v = 0; v < kVariants; ++v) G.d_refs[v] = ws.take<kern::BatchApplyRef>(gc);
    G.d_j = ws.take<int>(1);
    G.flags.assign(gc, kern::BatchState{});
  }
  // The tables live in pageable host vectors: copied on the group's stream,
  // which then waits for them (never through the legacy default stream,
  // which another thread's graph capture would make fail); the group's
  // stream first waits for the setups on st.
  TSYLV_HIP(hipStreamSynchronize(st));
  for (auto& G : groups) {
    const int gc = (int)G.ids.size();
    TSYLV_HIP(hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking));
    TSYLV_HIP(hipMemcpyAsync(G.d_items, G.items.data(), sizeof(kern::BatchItem) * gc,
                             hipMemcpyHostToDevice, G.stream));
    TSYLV_HIP(hipMemcpyAsync(G.d_state, G.flags.data(), sizeof(kern::BatchState) * gc,
                             hipMemcpyHostToDevice, G.stream));
    for (int v = 0; v < kVariants; ++v)
      if (!G.plan.refs[v].empty())
        TSYLV_HIP(hipMemcpyAsync(G.d_refs[v], G.plan.refs[v].data(),
                                 sizeof(kern::BatchApplyRef) * G.plan.refs[v].size(),
                                 hipMemcpyHostToDevice, G.stream));
    TSYLV_HIP(hipStreamSynchronize(G.stream));
  }

  auto apply_all = [&](Group& G, int mode, hipStream_t s) {
    for (int v = 0; v < kVariants; ++v)
      if (!G.plan.refs[v].empty())
        kern::batch_apply(G.d_items, G.d_refs[v], (int)G.plan.refs[v].size(), G.plan.ntiles[v],
                          kVariantIds[v], G.d_state, G.d_j, mode, s);
  };
  auto residual = [&](Group& G, int reduce_mode, hipStream_t s) {
    const int gc = G.plan.count;
    apply_all(G, kern::BM_RESID, s);
    kern::batch_dots(G.d_items, gc, G.plan.total_chunks, G.d_state, G.d_j, G.d_part, G.plan.ldp,
                     kern::BM_RESID, s);
    kern::batch_reduce(G.d_items, gc, G.d_state, G.d_j, G.d_part, G.plan.ldp, reduce_mode, m,
                       o.tol, o.max_cycles, s);
    kern::batch_scale(G.d_items, gc, G.plan.total_chunks, G.d_state, G.d_j, kern::BM_RESID, s);
  };
  auto step = [&](Group& G, hipStream_t s) {
    const int gc = G.plan.count;
    apply_all(G, kern::BM_STEP, s);
    for (int pass = 0; pass < 2; ++pass) {
      // the second pass runs only for the instances whose first pass cancelled
      const int md = pass == 0 ? kern::BM_STEP : kern::BM_PASS2;
      kern::batch_dots(G.d_items, gc, G.plan.total_chunks, G.d_state, G.d_j, G.d_part,
                       G.plan.ldp, md, s);
      kern::batch_reduce(G.d_items, gc, G.d_state, G.d_j, G.d_part, G.plan.ldp, md, m, o.tol,
                         o.max_cycles, s);
      kern::batch_update(G.d_items, gc, G.plan.total_chunks, G.d_state, G.d_j, md, s);
    }
    kern::batch_dots(G.d_items, gc, G.plan.total_chunks, G.d_state, G.d_j, G.d_part, G.plan.ldp,
                     kern::BM_WNORM, s);
    kern::batch_reduce(G.d_items, gc, G.d_state, G.d_j, G.d_part, G.plan.ldp, kern::BM_WNORM, m,
                       o.tol, o.max_cycles, s);
    kern::batch_scale(G.d_items, gc, G.plan.total_chunks, G.d_state, G.d_j, kern::BM_STEP, s);
    kern::batch_advance(G.d_j, s);
  };
  auto read_state = [&](Group& G) {
    TSYLV_HIP(hipMemcpyAsync(G.flags.data(), G.d_state, sizeof(kern::BatchState) * G.plan.count,
                             hipMemcpyDeviceToHost, G.stream));
    TSYLV_HIP(hipStreamSynchronize(G.stream));
    G.live = G.stepping = false;
    for (auto& f : G.flags) {
      G.live = G.live || !f.done;
      G.stepping = G.stepping || f.active;
    }
  };

  // ||C|| and the initial residual (X0 = 0 or the given X0), per group
  for (auto& G : groups) {
    kern::batch_set_j(G.d_j, 0, G.stream);
    kern::batch_dots(G.d_items, G.plan.count, G.plan.total_chunks, G.d_state, G.d_j, G.d_part,
                     G.plan.ldp, kern::BM_CNORM, G.stream);
    kern::batch_reduce(G.d_items, G.plan.count, G.d_state, G.d_j, G.d_part, G.plan.ldp,
                       kern::BM_CNORM, m, o.tol, o.max_cycles, G.stream);
    residual(G, kern::BM_RESID0, G.stream);
  }

  // each group's step as a graph of kernel nodes, recorded (not captured
  // from a stream: nothing another thread does meanwhile can invalidate it)
  // and replayed on the group's stream
  if (use_graph) {
    for (auto& G : groups) {
      hipGraph_t graph = nullptr;
      TSYLV_HIP(hipGraphCreate(&graph, 0));
      GraphRecorder rec{graph, nullptr};
      graph_recorder() = &rec;
      try {
        step(G, G.stream);
      } catch (...) {
        graph_recorder() = nullptr;
        (void)hipGraphDestroy(graph);
        throw;
      }
      graph_recorder() = nullptr;
      const hipError_t e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      TSYLV_HIP(e);
    }
  }

  for (auto& G : groups) read_state(G);
  for (int cycle = 0; cycle < o.max_cycles; ++cycle) {
    bool any = false;
    for (auto& G : groups) {
      G.stepping = G.live;
      if (G.live) {
        kern::batch_set_j(G.d_j, 0, G.stream);
        any = true;
      }
    }
    if (!any) break;
    for (int j = 0; j < m; ++j) {
      for (auto& G : groups) {
        if (!G.stepping) continue;
        if (use_graph)
          TSYLV_HIP(hipGraphLaunch(G.exec, G.stream));
        else
          step(G, G.stream);
      }
      if ((j + 1) % kCheckEvery == 0 && j + 1 < m) {
        bool more = false;
        for (auto& G : groups)
          if (G.stepping) {
            read_state(G);
            more = more || G.stepping;
          }
        if (!more) break;
      }
    }
    for (auto& G : groups) {
      if (!G.live) continue;
      kern::batch_backsub(G.d_items, G.plan.count, G.d_state, m, G.stream);
      kern::batch_update(G.d_items, G.plan.count, G.plan.total_chunks, G.d_state, G.d_j,
                         kern::BM_XUPDATE, G.stream);
      residual(G, kern::BM_RESID, G.stream);
    }
    for (auto& G : groups)
      if (G.live) read_state(G);
  }

  // ---- Algorithm 1 step 3: X = inverse transform of the planes ----
  for (auto& G : groups) TSYLV_HIP(hipStreamSynchronize(G.stream));
  for (int i = 0; i < count; ++i)
    kern::tube_xform_f64(all[i].Zx, probs[i].X, setups[i].xf_inv, probs[i].n * probs[i].s,
                         (int)probs[i].p, st);
  TSYLV_HIP(hipStreamSynchronize(st));
  for (auto& G : groups) read_state(G);
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = TSYLV_OK;
  for (auto& G : groups)
    for (size_t k = 0; k < G.ids.size(); ++k) {
      const kern::BatchState& S = G.flags[k];
      tsylv_info& inf = infos[G.ids[k]];
      std::memset(&inf, 0, sizeof(inf));
      inf.status = S.done ? S.status : TSYLV_NOT_CONVERGED;
      inf.steps = S.steps;
      inf.cycles = S.cycles;
      inf.outer = 0;
      inf.relres_true = S.cnorm > 0.0 ? S.beta / S.cnorm : 0.0;
      inf.relres_est = inf.relres_true;
      inf.seconds = secs;
      if (inf.status != TSYLV_OK) worst = TSYLV_NOT_CONVERGED;
    }
  return worst;
}

// ---------------------------------------------------------------------------
// Which executor serves an instance.  The lockstep kernels win where each
// solve is launch- and synchronisation-bound (many small instances: 6x the
// serving loop at n <= 256, s <= 16, p <= 8); for large instances one
// lockstep step alternates an MFMA-bound apply of everything with HBM-bound
// sweeps of everything, and independent solves on several streams, which
// overlap the apply of one instance with the sweeps of another, are faster
// (1.6x on n up to 2048, s up to 128).  Refined solves (FP32 / BF16 inner
// cycles) always take the stream executor.  The choice depends on the
// instance alone, so its result does not depend on the rest of the batch.
// ---------------------------------------------------------------------------

namespace {

constexpr int64_t kLockstepMaxElems = int64_t(1) << 18;  // n s p of a lockstep instance
constexpr int kTaskStreams = 8;

bool lockstep_instance(const tsylv_problem& q, const tsylv_opts& o) {
  return !o.refine && q.n * q.s * q.p <= kLockstepMaxElems;
}

int xform_blocks(int64_t E) {
  return (int)((E + kern::kBatchXformBlock - 1) / kern::kBatchXformBlock);
}

// Instances small enough for a whole solve in one workgroup (the single
// solve's criterion, kern::tiny_krylov_fits; TSYLV_KRYLOV_TINY=0 turns it
// off here too) are solved by one launch for all of them.
bool tiny_instance(const tsylv_problem& q, const tsylv_opts& o) {
  if (o.refine) return false;
  const char* f = std::getenv("TSYLV_KRYLOV_TINY");
  if (f && f[0] == '0') return false;
  return kern::tiny_krylov_fits(q.n, q.s, q.p, o.m);
}

size_t tiny_batch_bytes(int count, const tsylv_problem* probs, const tsylv_opts& o) {
  if (count <= 0) return 0;
  // (per instance: its Fourier setup, which bounds what the shared
  // transform matrices and X0 planes take; at most four forward and one
  // inverse transform descriptor)
  size_t b = Workspace::bytes_for((int64_t)count, sizeof(kern::TinyJob)) +
             Workspace::bytes_for((int64_t)count * kern::kTinyRecord, 8) +
             Workspace::bytes_for(5 * (int64_t)count, sizeof(kern::XformDesc)) +
             Workspace::bytes_for(5 * (int64_t)count + 2, sizeof(int));
  for (int i = 0; i < count; ++i) {
    const int64_t N = probs[i].n * probs[i].s * probs[i].p;
    b += setup_bytes(probs[i].n, probs[i].s, probs[i].p) +
         Workspace::bytes_for((int64_t)(o.m + 1) * N, 8) +
         Workspace::bytes_for((int64_t)o.m * o.m, 8);
  }
  return b;
}

// The single-workgroup executor: every instance's setup transforms, one
// launch that runs each instance's whole restarted tGMRES(m) in a
// workgroup of its own (Algorithm 3 on the device, kern::tiny_krylov_batch),
// the inverse transforms, one copy of the result records.  It runs on a
// stream of its own, ordered after the caller's stream, beside the lockstep
// executor (whose instances fill the rest of the GPU); finish() waits for
// it.  An instance's arithmetic is that of its single solve (tsylv_gmres
// takes the same kernel for it), in any batch.
class TinyExec {
 public:
  TinyExec(Ctx& ctx, Arena& arena, hipStream_t parent, int count, const tsylv_problem* probs,
           const uint64_t* const* gens, const tsylv_opts& o)
      : ws_(arena, tiny_batch_bytes(count, probs, o)), count_(count) {
    TSYLV_HIP(hipStreamCreateWithFlags(&own_.s, hipStreamNonBlocking));
    TSYLV_HIP(hipEventCreateWithFlags(&own_.ready, hipEventDisableTiming));
    s_ = own_.s;
    ready_ = own_.ready;
    TSYLV_HIP(hipEventRecord(ready_, parent));
    TSYLV_HIP(hipStreamWaitEvent(s_, ready_, 0));
    jobs_.resize(count);
    rec_ = ws_.take<double>((int64_t)count * kern::kTinyRecord);
    size_t lds = 0;
    for (int i = 0; i < count; ++i)
      lds = std::max(lds, kern::tiny_krylov_lds(probs[i].n, probs[i].s, probs[i].p, o.m));
    // Algorithm 1 step 1 for every stored instance in one launch (with one
    // set of transform matrices per distinct p and one zero fill of their
    // X0 planes), Algorithm 1 step 3 for every X in another; an instance
    // whose tensors are generated takes the single solve's setup.
    const bool x0 = o.x0_given != 0;
    struct Mats {
      double *op, *fwd, *inv;
    };
    std::map<int64_t, Mats> mats;
    auto mats_of = [&](int64_t p) {
      auto it = mats.find(p);
      if (it != mats.end()) return it->second;
      const Mats M{ws_.take<double>(p * p), ws_.take<double>(p * p), ws_.take<double>(p * p)};
      kern::build_xform(M.op, (int)p, XF_OPERATOR, s_);
      kern::build_xform(M.fwd, (int)p, XF_FORWARD, s_);
      kern::build_xform(M.inv, (int)p, XF_INVERSE, s_);
      mats.emplace(p, M);
      return M;
    };
    int64_t zx_total = 0;
    for (int i = 0; i < count; ++i)
      if (!(gens && gens[i])) zx_total += probs[i].n * probs[i].s * probs[i].p;
    double* zx = ws_.take<double>(zx_total);
    if (zx_total > 0 && !x0)
      TSYLV_HIP(hipMemsetAsync(zx, 0, zx_total * sizeof(double), s_));
    std::vector<kern::XformDesc> fwd, inv;
    for (int i = 0; i < count; ++i) {
      const tsylv_problem& q = probs[i];
      const int64_t N = q.n * q.s * q.p;
      kern::TinyJob& j = jobs_[i];
      const double* xf_inv;
      if (gens && gens[i]) {
        const Setup S = setup_fourier(ctx, s_, false, ws_, q.n, q.s, q.p, q.A, q.B, q.C, q.X,
                                      x0, gens[i]);
        j.Ah = S.Ah;
        j.Bh = S.Bh;
        j.Zc = S.Zc;
        j.Zx = S.Zx;
        xf_inv = S.xf_inv;
      } else {
        const Mats M = mats_of(q.p);
        double* Ah = ws_.take<double>(q.p * q.n * q.n);
        double* Bh = ws_.take<double>(q.p * q.s * q.s);
        double* Zc = ws_.take<double>(N);
        j.Ah = Ah;
        j.Bh = Bh;
        j.Zc = Zc;
        j.Zx = zx;
        zx += N;
        fwd.push_back({q.A, Ah, M.op, q.n * q.n, (int)q.p});
        fwd.push_back({q.B, Bh, M.op, q.s * q.s, (int)q.p});
        fwd.push_back({q.C, Zc, M.fwd, q.n * q.s, (int)q.p});
        if (x0) fwd.push_back({q.X, j.Zx, M.fwd, q.n * q.s, (int)q.p});
        xf_inv = M.inv;
      }
      inv.push_back({j.Zx, q.X, xf_inv, q.n * q.s, (int)q.p});
      j.Vg = ws_.take<double>((int64_t)(o.m + 1) * N);
      j.Rg = ws_.take<double>((int64_t)o.m * o.m);
      j.hist = nullptr;
      j.hist_cap = 0;
      j.out = rec_ + (int64_t)i * kern::kTinyRecord;
      j.tol = o.tol;
      j.n = (int)q.n;
      j.s = (int)q.s;
      j.p = (int)q.p;
      j.m = o.m;
      j.max_cycles = std::max(o.max_cycles, 0);
      j.fom = 0;
      j.x0_given = x0 ? 1 : 0;
      j.lslots = kern::tiny_krylov_slots(q.n, q.s, q.p, o.m, lds);
    }
    // descriptor tables: the forward ones, then the inverse ones with block
    // offsets of their own (host copies stay members until the stream has
    // been waited for)
    descs_ = fwd;
    descs_.insert(descs_.end(), inv.begin(), inv.end());
    bfirst_.assign(descs_.size() + 2, 0);
    const size_t nf = fwd.size();
    for (size_t d = 0; d < nf; ++d) bfirst_[d + 1] = bfirst_[d] + xform_blocks(fwd[d].E);
    for (size_t d = 0; d < inv.size(); ++d)
      bfirst_[nf + 2 + d] = bfirst_[nf + 1 + d] + xform_blocks(inv[d].E);
    kern::TinyJob* d_jobs = ws_.take<kern::TinyJob>(count);
    kern::XformDesc* d_desc = ws_.take<kern::XformDesc>((int64_t)descs_.size());
    int* d_bf = ws_.take<int>((int64_t)bfirst_.size());
    TSYLV_HIP(hipMemcpyAsync(d_jobs, jobs_.data(), sizeof(kern::TinyJob) * count,
                             hipMemcpyHostToDevice, s_));
    TSYLV_HIP(hipMemcpyAsync(d_desc, descs_.data(), sizeof(kern::XformDesc) * descs_.size(),
                             hipMemcpyHostToDevice, s_));
    TSYLV_HIP(hipMemcpyAsync(d_bf, bfirst_.data(), sizeof(int) * bfirst_.size(),
                             hipMemcpyHostToDevice, s_));
    kern::batch_xform(d_desc, d_bf, (int)nf, bfirst_[nf], s_);
    kern::tiny_krylov_batch(d_jobs, count, lds, s_);
    kern::batch_xform(d_desc + nf, d_bf + nf + 1, (int)inv.size(), bfirst_.back(), s_);
  }
  TinyExec(const TinyExec&) = delete;
  TinyExec& operator=(const TinyExec&) = delete;

  // Waits for the launch; the records to infos (in the batch's order) and
  // the caller's stream ordered after this executor's work.  Returns
  // TSYLV_OK or TSYLV_NOT_CONVERGED (some instance did not converge).
  int finish(hipStream_t parent, tsylv_info* infos) {
    std::vector<double> h((size_t)count_ * kern::kTinyRecord);
    TSYLV_HIP(hipMemcpyAsync(h.data(), rec_, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                             s_));
    TSYLV_HIP(hipStreamSynchronize(s_));
    TSYLV_HIP(hipEventRecord(ready_, s_));
    TSYLV_HIP(hipStreamWaitEvent(parent, ready_, 0));
    int worst = TSYLV_OK;
    for (int i = 0; i < count_; ++i) {
      const double* r = h.data() + (size_t)i * kern::kTinyRecord;
      tsylv_info& in = infos[i];
      in = tsylv_info{};
      in.status = (int)r[0];
      in.steps = (int)r[1];
      in.cycles = (int)r[2];
      in.relres_true = r[3];
      in.relres_est = r[4];
      in.fom_fallback = (int)r[5];
      if (in.status != TSYLV_OK) worst = TSYLV_NOT_CONVERGED;
    }
    return worst;
  }

 private:
  // The stream and event, waited for and released before the workspace is
  // returned to the arena (members go in reverse order, also when the
  // constructor throws after work was enqueued).
  struct OwnStream {
    hipStream_t s = nullptr;
    hipEvent_t ready = nullptr;
    OwnStream() = default;
    OwnStream(const OwnStream&) = delete;
    OwnStream& operator=(const OwnStream&) = delete;
    ~OwnStream() {
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
      if (ready) (void)hipEventDestroy(ready);
    }
  };
  Workspace ws_;
  OwnStream own_;
  int count_;
  hipStream_t s_ = nullptr;
  hipEvent_t ready_ = nullptr;
  std::vector<kern::TinyJob> jobs_;
  std::vector<kern::XformDesc> descs_;
  std::vector<int> bfirst_;
  double* rec_ = nullptr;
};

// Up to kTaskStreams solves at a time, each a KrylovTask (the synchronous
// solve's object) on its own stream, advanced as its stream finishes a
// phase; admitted in order while the arena holds their workspaces.
int run_tasks(Ctx& ctx, hipStream_t st, const std::vector<int>& ids, const tsylv_problem* probs,
              const uint64_t* const* gens, const tsylv_opts& o, tsylv_info* infos) {
  const size_t per_slot = KrylovTask::pinned_doubles(o);
  double* pinned = ctx.task_buffer(kTaskStreams * per_slot);
  struct Slot {
    hipStream_t s = nullptr;
    std::unique_ptr<KrylovTask> t;
    int idx = -1;
    bool in_flight = false;
  };
  std::vector<Slot> slots(kTaskStreams);
  hipEvent_t ready = nullptr;
  struct Cleanup {
    std::vector<Slot>& sl;
    hipEvent_t& ev;
    ~Cleanup() {
      for (auto& x : sl) {
        if (x.s) (void)hipStreamSynchronize(x.s);
        x.t.reset();
        if (x.s) (void)hipStreamDestroy(x.s);
      }
      if (ev) (void)hipEventDestroy(ev);
    }
  } cleanup{slots, ready};
  TSYLV_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  TSYLV_HIP(hipEventRecord(ready, st));  // the caller's work on st comes first
  for (auto& x : slots) {
    TSYLV_HIP(hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking));
    TSYLV_HIP(hipStreamWaitEvent(x.s, ready, 0));
  }
  size_t next = 0;
  int active = 0, idle = 0;
  while (next < ids.size() || active > 0) {
    // admit
    for (int k = 0; k < kTaskStreams && next < ids.size(); ++k) {
      Slot& x = slots[k];
      if (x.t) continue;
      const int i = ids[next];
      const tsylv_problem& q = probs[i];
      try {
        x.t.reset(new KrylovTask(ctx, x.s, false, pinned + (size_t)k * per_slot,
                                 TSYLV_METHOD_GMRES, q.n, q.s, q.p, q.A, q.B, q.C, q.X, o,
                                 gens ? gens[i] : nullptr));
      } catch (const Error& e) {
        if (e.status == TSYLV_ENOMEM && active > 0) break;  // wait for memory
        std::memset(&infos[i], 0, sizeof(tsylv_info));
        infos[i].status = e.status;
        ++next;
        continue;
      }
      x.idx = i;
      x.in_flight = false;
      ++active;
      ++next;
    }
    // advance
    bool progressed = false;
    for (auto& x : slots) {
      if (!x.t) continue;
      try {
        if (x.in_flight) {
          const hipError_t qe = hipStreamQuery(x.s);
          if (qe == hipErrorNotReady) continue;
          TSYLV_HIP(qe);
          x.in_flight = false;
          x.t->complete();
          progressed = true;
        }
        if (!x.t->done()) {
          x.t->enqueue();
          x.in_flight = true;
          progressed = true;
          continue;
        }
        infos[x.idx] = x.t->info();
        infos[x.idx].status = x.t->status();
      } catch (const Error& e) {
        (void)hipStreamSynchronize(x.s);
        std::memset(&infos[x.idx], 0, sizeof(tsylv_info));
        infos[x.idx].status = e.status;
      }
      x.t.reset();
      x.idx = -1;
      --active;
      progressed = true;
    }
    if (progressed)
      idle = 0;
    else if (++idle > 256)
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    else
      std::this_thread::yield();
  }
  int worst = TSYLV_OK;
  for (int i : ids)
    if (infos[i].status != TSYLV_OK) worst = TSYLV_NOT_CONVERGED;
  return worst;
}

}  // namespace

size_t batch_workspace_bytes(int count, const tsylv_problem* probs, const tsylv_opts& o) {
  std::vector<tsylv_problem> lock, tiny;
  std::vector<size_t> task_bytes;
  for (int i = 0; i < count; ++i) {
    if (tiny_instance(probs[i], o))
      tiny.push_back(probs[i]);
    else if (lockstep_instance(probs[i], o))
      lock.push_back(probs[i]);
    else
      task_bytes.push_back(
          krylov_workspace_bytes(TSYLV_METHOD_GMRES, probs[i].n, probs[i].s, probs[i].p, o));
  }
  // the stream executor runs first, up to kTaskStreams workspaces at once;
  // the lockstep batch after it, then the single-workgroup one
  std::sort(task_bytes.begin(), task_bytes.end(), std::greater<size_t>());
  size_t tb = 0;
  for (size_t k = 0; k < task_bytes.size() && k < (size_t)kTaskStreams; ++k) tb += task_bytes[k];
  // then the lockstep and single-workgroup executors side by side
  return std::max(tb, lockstep_workspace_bytes((int)lock.size(), lock.data(), o) +
                          tiny_batch_bytes((int)tiny.size(), tiny.data(), o));
}

bool batch_solves_whole(const tsylv_problem& q, const tsylv_opts& o) {
  return tiny_instance(q, o);
}

size_t served_batch_bytes(int count, const tsylv_problem* probs, const tsylv_opts& o) {
  std::vector<tsylv_problem> lock, tiny;
  for (int i = 0; i < count; ++i) (tiny_instance(probs[i], o) ? tiny : lock).push_back(probs[i]);
  return lockstep_workspace_bytes((int)lock.size(), lock.data(), o) +
         tiny_batch_bytes((int)tiny.size(), tiny.data(), o);
}

int gmres_batch(Ctx& ctx, hipStream_t st, int count, const tsylv_problem* probs,
                const uint64_t* const* gens, const tsylv_opts& o, tsylv_info* infos,
                bool use_graph, bool no_streams, Arena* arena) {
  const auto t0 = std::chrono::steady_clock::now();
  Arena& ar = arena ? *arena : ctx.arena;
  std::vector<int> lock, tasks, tiny;
  for (int i = 0; i < count; ++i) {
    if (tiny_instance(probs[i], o))
      tiny.push_back(i);
    else
      (no_streams || lockstep_instance(probs[i], o) ? lock : tasks).push_back(i);
  }
  int worst = TSYLV_OK;
  if (!tasks.empty() && run_tasks(ctx, st, tasks, probs, gens, o, infos) != TSYLV_OK)
    worst = TSYLV_NOT_CONVERGED;
  // the single-workgroup executor launches first and runs beside the
  // lockstep batch
  std::vector<tsylv_problem> tp;
  std::vector<const uint64_t*> tg;
  for (int i : tiny) {
    tp.push_back(probs[i]);
    tg.push_back(gens ? gens[i] : nullptr);
  }
  std::unique_ptr<TinyExec> tex;
  if (!tiny.empty())
    tex.reset(
        new TinyExec(ctx, ar, st, (int)tiny.size(), tp.data(), gens ? tg.data() : nullptr, o));
  if (!lock.empty()) {
    std::vector<tsylv_problem> lp;
    std::vector<const uint64_t*> lg;
    for (int i : lock) {
      lp.push_back(probs[i]);
      lg.push_back(gens ? gens[i] : nullptr);
    }
    std::vector<tsylv_info> li(lock.size());
    if (gmres_lockstep(ctx, ar, st, (int)lock.size(), lp.data(), gens ? lg.data() : nullptr, o,
                       li.data(), use_graph) != TSYLV_OK)
      worst = TSYLV_NOT_CONVERGED;
    for (size_t k = 0; k < lock.size(); ++k) infos[lock[k]] = li[k];
  }
  if (tex) {
    std::vector<tsylv_info> ti(tiny.size());
    if (tex->finish(st, ti.data()) != TSYLV_OK) worst = TSYLV_NOT_CONVERGED;
    for (size_t k = 0; k < tiny.size(); ++k) infos[tiny[k]] = ti[k];
  }
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int i = 0; i < count; ++i) infos[i].seconds = secs;
  return worst;
}

}  // namespace tsylv
