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
// Since j lives in device memory, the step is captured once as a HIP graph
// and replayed m times per cycle; the host reads the instances' flags every
// kCheckEvery steps to end a cycle early when no instance is stepping.  At
// a cycle's end: y = R^{-1} g, X += V y, the true residual R = C - M(X), and
// the restart test of Algorithm 3 -- again one launch each for the batch.
#include <chrono>
#include <cstring>
#include <memory>
#include <vector>

#include "kernels.hpp"
#include "runtime.hpp"
#include "solvers.hpp"

namespace tsylv {

namespace {

constexpr int kCheckEvery = 8;
constexpr int kVariants = 3;

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

size_t batch_workspace_bytes(int count, const tsylv_problem* probs, const tsylv_opts& o) {
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
  return b;
}

int gmres_batch(Ctx& ctx, int count, const tsylv_problem* probs, const tsylv_opts& o,
                tsylv_info* infos, bool use_graph) {
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = ctx.stream;
  const int m = o.m;
  BatchPlan plan;
  plan.count = count;
  plan.m = m;
  plan.ldp = m + 3;

  // ---- workspace and per-instance setup (Algorithm 1 step 1) ----
  Workspace ws(ctx.arena, batch_workspace_bytes(count, probs, o));
  // on any exit, let the stream drain before the workspace returns to the arena
  struct SyncOnExit {
    hipStream_t s;
    ~SyncOnExit() { (void)hipStreamSynchronize(s); }
  } drain{st};
  std::vector<kern::BatchItem> items(count);
  std::vector<Setup> setups(count);
  int64_t chunk0 = 0;
  for (int i = 0; i < count; ++i) {
    const tsylv_problem& q = probs[i];
    const int64_t N = q.n * q.s * q.p;
    const int64_t ldv = (N + 63) / 64 * 64;
    Setup S = setup_fourier(ctx, st, false, ws, q.n, q.s, q.p, q.A, q.B, q.C, q.X,
                            o.x0_given != 0);
    setups[i] = S;
    kern::BatchItem& it = items[i];
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
    it.chunk0 = (int)chunk0;
    it.nchunks = (int)chunks_of(N);
    chunk0 += it.nchunks;
    const int v = kern::batch_apply_variant(q.s);
    kern::BatchApplyRef r;
    r.item = i;
    r.tile0 = plan.ntiles[v];
    plan.ntiles[v] += kern::batch_apply_tiles(v, q.n, q.s, (int)q.p, &r.nrt, &r.nct);
    plan.refs[v].push_back(r);
  }
  plan.total_chunks = (int)chunk0;
  kern::BatchItem* d_items = ws.take<kern::BatchItem>(count);
  kern::BatchState* d_state = ws.take<kern::BatchState>(count);
  double* d_part = ws.take<double>((int64_t)plan.total_chunks * plan.ldp);
  kern::BatchApplyRef* d_refs[kVariants];
  for (int v = 0; v < kVariants; ++v) d_refs[v] = ws.take<kern::BatchApplyRef>(count);
  int* d_j = ws.take<int>(1);
  std::vector<kern::BatchState> hstate(count);
  std::memset(hstate.data(), 0, sizeof(kern::BatchState) * count);
  // The tables live in pageable host vectors: blocking copies once the
  // stream is idle (the setups above are done), then the batch's kernels.
  TSYLV_HIP(hipStreamSynchronize(st));
  TSYLV_HIP(hipMemcpy(d_items, items.data(), sizeof(kern::BatchItem) * count,
                      hipMemcpyHostToDevice));
  TSYLV_HIP(hipMemcpy(d_state, hstate.data(), sizeof(kern::BatchState) * count,
                      hipMemcpyHostToDevice));
  for (int v = 0; v < kVariants; ++v)
    if (!plan.refs[v].empty())
      TSYLV_HIP(hipMemcpy(d_refs[v], plan.refs[v].data(),
                          sizeof(kern::BatchApplyRef) * plan.refs[v].size(),
                          hipMemcpyHostToDevice));
  kern::batch_set_j(d_j, 0, st);

  auto apply_all = [&](int mode, hipStream_t s) {
    for (int v = 0; v < kVariants; ++v)
      if (!plan.refs[v].empty())
        kern::batch_apply(d_items, d_refs[v], (int)plan.refs[v].size(), plan.ntiles[v], v,
                          d_state, d_j, mode, s);
  };
  auto residual = [&](int reduce_mode, hipStream_t s) {
    apply_all(kern::BM_RESID, s);
    kern::batch_dots(d_items, count, plan.total_chunks, d_state, d_j, d_part, plan.ldp,
                     kern::BM_RESID, s);
    kern::batch_reduce(d_items, count, d_state, d_j, d_part, plan.ldp, reduce_mode, m, o.tol,
                       o.max_cycles, s);
    kern::batch_scale(d_items, count, plan.total_chunks, d_state, d_j, kern::BM_RESID, s);
  };
  auto step = [&](hipStream_t s) {
    apply_all(kern::BM_STEP, s);
    for (int pass = 0; pass < 2; ++pass) {
      // the second pass runs only for the instances whose first pass cancelled
      const int md = pass == 0 ? kern::BM_STEP : kern::BM_PASS2;
      kern::batch_dots(d_items, count, plan.total_chunks, d_state, d_j, d_part, plan.ldp, md, s);
      kern::batch_reduce(d_items, count, d_state, d_j, d_part, plan.ldp, md, m, o.tol,
                         o.max_cycles, s);
      kern::batch_update(d_items, count, plan.total_chunks, d_state, d_j, md, s);
    }
    kern::batch_dots(d_items, count, plan.total_chunks, d_state, d_j, d_part, plan.ldp,
                     kern::BM_WNORM, s);
    kern::batch_reduce(d_items, count, d_state, d_j, d_part, plan.ldp, kern::BM_WNORM, m, o.tol,
                       o.max_cycles, s);
    kern::batch_scale(d_items, count, plan.total_chunks, d_state, d_j, kern::BM_STEP, s);
    kern::batch_advance(d_j, s);
  };

  // ||C|| and the initial residual (X0 = 0 or the given X0)
  kern::batch_dots(d_items, count, plan.total_chunks, d_state, d_j, d_part, plan.ldp,
                   kern::BM_CNORM, st);
  kern::batch_reduce(d_items, count, d_state, d_j, d_part, plan.ldp, kern::BM_CNORM, m, o.tol,
                     o.max_cycles, st);
  residual(kern::BM_RESID0, st);

  // one step as a graph, captured on a private stream and replayed on ours
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  struct Cleanup {
    hipGraphExec_t* e;
    hipStream_t* c;
    ~Cleanup() {
      if (*e) (void)hipGraphExecDestroy(*e);
      if (*c) (void)hipStreamDestroy(*c);
    }
  } cleanup{&exec, &cap};
  if (use_graph) {
    TSYLV_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    TSYLV_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    try {
      step(cap);
    } catch (...) {
      (void)hipStreamEndCapture(cap, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    TSYLV_HIP(hipStreamEndCapture(cap, &graph));
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    TSYLV_HIP(e);
  }

  std::vector<kern::BatchState> flags(count);
  kern::BatchState* h_flags = flags.data();
  auto read_state = [&]() {
    TSYLV_HIP(hipStreamSynchronize(st));
    TSYLV_HIP(hipMemcpy(h_flags, d_state, sizeof(kern::BatchState) * count,
                        hipMemcpyDeviceToHost));
  };
  read_state();
  for (int cycle = 0; cycle < o.max_cycles; ++cycle) {
    int live = 0;
    for (int i = 0; i < count; ++i) live += h_flags[i].done ? 0 : 1;
    if (live == 0) break;
    kern::batch_set_j(d_j, 0, st);
    for (int j = 0; j < m; ++j) {
      if (use_graph)
        TSYLV_HIP(hipGraphLaunch(exec, st));
      else
        step(st);
      if ((j + 1) % kCheckEvery == 0 && j + 1 < m) {
        read_state();
        int stepping = 0;
        for (int i = 0; i < count; ++i) stepping += h_flags[i].active;
        if (stepping == 0) break;
      }
    }
    kern::batch_backsub(d_items, count, d_state, m, st);
    kern::batch_update(d_items, count, plan.total_chunks, d_state, d_j, kern::BM_XUPDATE, st);
    residual(kern::BM_RESID, st);
    read_state();
  }

  // ---- Algorithm 1 step 3: X = inverse transform of the planes ----
  for (int i = 0; i < count; ++i)
    kern::tube_xform_f64(items[i].Zx, probs[i].X, setups[i].xf_inv, probs[i].n * probs[i].s,
                         (int)probs[i].p, st);
  read_state();
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = TSYLV_OK;
  for (int i = 0; i < count; ++i) {
    const kern::BatchState& S = h_flags[i];
    tsylv_info& inf = infos[i];
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

}  // namespace tsylv
