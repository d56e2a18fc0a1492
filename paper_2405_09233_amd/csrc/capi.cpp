// extern "C" boundary: argument checks, context handling, error mapping.
#include <cstdlib>
#include <cstring>
#include <new>

#include "kernels.hpp"
#include "runtime.hpp"
#include "serve.hpp"
#include "solvers.hpp"

using namespace tsylv;

struct tsylv_ctx {
  Ctx c;
};

namespace {

constexpr size_t kPinned = 1 << 16;  // doubles of pinned host staging

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    return e.status;
  } catch (const std::bad_alloc&) {
    return TSYLV_ENOMEM;
  } catch (...) {
    return TSYLV_EHIP;
  }
}

// A size query that never throws (0 on any failure).
template <typename F>
size_t guarded_size(F&& f) {
  try {
    return f();
  } catch (...) {
    return 0;
  }
}

bool dims_ok(int64_t n, int64_t s, int64_t p) {
  return n > 0 && s > 0 && p > 0 && n <= (int64_t(1) << 20) && s <= (int64_t(1) << 20) &&
         p <= 4096;
}

bool opts_ok(const tsylv_opts& o) {
  bool ok = o.m >= 1 && o.m <= 1000 && o.max_cycles >= 0 && o.tol >= 0.0 &&
            (o.prec == TSYLV_FP64 || o.prec == TSYLV_FP32 || o.prec == TSYLV_BF16);
  if (o.refine)
    ok = ok && o.prec != TSYLV_FP64 && o.inner_m >= 1 && o.inner_m <= 1000 && o.max_outer >= 0 &&
         o.inner_tol > 0.0 && o.inner_tol < 1.0;
  else
    ok = ok && o.prec == TSYLV_FP64;
  return ok;
}

bool tbs_dims_ok(int64_t n, int64_t s) {
  return n >= 1 && s >= 1 && n <= kern::tbs_max_size() && s <= kern::tbs_max_size();
}

void set_device(const tsylv_ctx* ctx) { TSYLV_HIP(hipSetDevice(ctx->c.device)); }

// Early rejection: the info record (if any) still carries the status.
int reject(tsylv_info* info, int status) {
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = status;
  }
  return status;
}

}  // namespace

extern "C" {

void tsylv_default_opts(int method, tsylv_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->m = (method == TSYLV_METHOD_TBA) ? 10 : 30;
  o->max_cycles = 500;
  o->tol = 1e-8;
  o->x0_given = 0;
  o->prec = TSYLV_FP64;
  o->refine = 0;
  o->inner_m = 40;
  o->inner_tol = 1e-4;
  o->max_outer = 500;
  o->res_hist = nullptr;
  o->res_hist_cap = 0;
}

int tsylv_create(tsylv_ctx** out, int device, void* hip_stream, void* arena, size_t arena_bytes) {
  if (!out || arena_bytes == 0) return TSYLV_EINVAL;
  *out = nullptr;
  return guarded([&]() {
    int ndev = 0;
    TSYLV_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return (int)TSYLV_EINVAL;
    TSYLV_HIP(hipSetDevice(device));
    auto* ctx = new tsylv_ctx();
    ctx->c.device = device;
    ctx->c.stream = static_cast<hipStream_t>(hip_stream);
    if (arena == nullptr) {
      void* p = nullptr;
      hipError_t e = hipMalloc(&p, arena_bytes);
      if (e != hipSuccess) {
        delete ctx;
        return (int)TSYLV_ENOMEM;
      }
      ctx->c.owns_arena = true;
      arena = p;
    }
    ctx->c.arena_ptr = arena;
    ctx->c.arena.init(static_cast<char*>(arena), arena_bytes);
    void* hp = nullptr;
    if (hipHostMalloc(&hp, kPinned * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      if (ctx->c.owns_arena) (void)hipFree(ctx->c.arena_ptr);
      delete ctx;
      return (int)TSYLV_ENOMEM;
    }
    ctx->c.pinned = static_cast<double*>(hp);
    ctx->c.pinned_count = kPinned;
    *out = ctx;
    return (int)TSYLV_OK;
  });
}

int tsylv_destroy(tsylv_ctx* ctx) {
  if (!ctx) return TSYLV_EINVAL;
  return guarded([&]() {
    set_device(ctx);
    {
      std::lock_guard<std::mutex> g(ctx->c.sched_mu);
      if (ctx->c.sched) scheduler_destroy(ctx->c.sched);
      ctx->c.sched = nullptr;
    }
    (void)hipStreamSynchronize(ctx->c.stream);
    if (ctx->c.pinned) (void)hipHostFree(ctx->c.pinned);
    if (ctx->c.task_pinned) (void)hipHostFree(ctx->c.task_pinned);
    if (ctx->c.owns_arena) (void)hipFree(ctx->c.arena_ptr);
    delete ctx;
    return (int)TSYLV_OK;
  });
}

size_t tsylv_workspace_bytes(int method, int64_t n, int64_t s, int64_t p, const tsylv_opts* opts) {
  if (!dims_ok(n, s, p)) return 0;
  tsylv_opts o;
  tsylv_default_opts(method < 0 ? 0 : method, &o);
  if (opts) o = *opts;
  if (method == -1) return apply_workspace_bytes(n, s, p);
  if (method == TSYLV_METHOD_GMRES || method == TSYLV_METHOD_FOM)
    return krylov_workspace_bytes(method, n, s, p, o);
  if (method == TSYLV_METHOD_TBS)  // beyond 64: the tGMRES that stands in for it
    return tbs_dims_ok(n, s) ? krylov_workspace_bytes(method, n, s, p, o)
                             : krylov_workspace_bytes(TSYLV_METHOD_GMRES, n, s, p,
                                                      tbs_fallback_opts(o.tol));
  if (method == TSYLV_METHOD_TBA) {
    if (n < 2 * s) return 0;
    int m = o.m;
    if ((int64_t)(m + 1) * s > n) m = (int)(n / s) - 1;
    return tba_workspace_bytes(n, s, p, m);
  }
  return 0;
}

int tsylv_apply(tsylv_ctx* ctx, int64_t n, int64_t s, int64_t p, const double* A, const double* B,
                const double* X, double* Y, int prec) {
  if (!ctx || !A || !B || !X || !Y || !dims_ok(n, s, p)) return TSYLV_EINVAL;
  if (prec != TSYLV_FP64 && prec != TSYLV_FP32 && prec != TSYLV_BF16) return TSYLV_EINVAL;
  return guarded([&]() {
    std::lock_guard<std::mutex> g(ctx->c.sync_mu);
    set_device(ctx);
    return apply_spatial(ctx->c, n, s, p, A, B, X, Y, prec);
  });
}

static int krylov_entry(int method, tsylv_ctx* ctx, int64_t n, int64_t s, int64_t p,
                        const double* A, const double* B, const double* C, double* X,
                        const tsylv_opts* opts, tsylv_info* info) {
  if (!ctx || !A || !B || !C || !X || !dims_ok(n, s, p)) return reject(info, TSYLV_EINVAL);
  tsylv_opts o;
  tsylv_default_opts(method, &o);
  if (opts) o = *opts;
  if (!opts_ok(o)) return reject(info, TSYLV_EINVAL);
  tsylv_info local;
  std::memset(&local, 0, sizeof(local));
  tsylv_info& inf = info ? *info : local;
  std::memset(&inf, 0, sizeof(inf));
  int st = guarded([&]() {
    std::lock_guard<std::mutex> g(ctx->c.sync_mu);
    set_device(ctx);
    return krylov_solve(ctx->c, method, n, s, p, A, B, C, X, o, inf);
  });
  inf.status = st;
  return st;
}

int tsylv_fom(tsylv_ctx* ctx, int64_t n, int64_t s, int64_t p, const double* A, const double* B,
              const double* C, double* X, const tsylv_opts* opts, tsylv_info* info) {
  return krylov_entry(TSYLV_METHOD_FOM, ctx, n, s, p, A, B, C, X, opts, info);
}

int tsylv_gmres(tsylv_ctx* ctx, int64_t n, int64_t s, int64_t p, const double* A,
                const double* B, const double* C, double* X, const tsylv_opts* opts,
                tsylv_info* info) {
  return krylov_entry(TSYLV_METHOD_GMRES, ctx, n, s, p, A, B, C, X, opts, info);
}

int tsylv_tbs(tsylv_ctx* ctx, int64_t n, int64_t s, int64_t p, const double* A, const double* B,
              const double* C, double* X, const tsylv_opts* opts, tsylv_info* info) {
  tsylv_opts o;
  tsylv_default_opts(TSYLV_METHOD_TBS, &o);
  if (opts) o.tol = opts->tol;  // the direct solve reads the tolerance only
  if (!tbs_dims_ok(n, s)) {
    // beyond the direct solve's size limit: tGMRES to the same tolerance
    if (!dims_ok(n, s, p)) return reject(info, TSYLV_EINVAL);
    const tsylv_opts g = tbs_fallback_opts(o.tol);
    return krylov_entry(TSYLV_METHOD_GMRES, ctx, n, s, p, A, B, C, X, &g, info);
  }
  return krylov_entry(TSYLV_METHOD_TBS, ctx, n, s, p, A, B, C, X, &o, info);
}

int tsylv_tba(tsylv_ctx* ctx, int64_t n, int64_t s, int64_t p, const double* A, const double* B,
              const double* C, double* X, const tsylv_opts* opts, tsylv_info* info) {
  if (!ctx || !A || !B || !C || !X || !dims_ok(n, s, p) || n < 2 * s)
    return reject(info, TSYLV_EINVAL);
  tsylv_opts o;
  tsylv_default_opts(TSYLV_METHOD_TBA, &o);
  if (opts) o = *opts;
  if (!opts_ok(o) || o.refine) return reject(info, TSYLV_EINVAL);
  tsylv_info local;
  std::memset(&local, 0, sizeof(local));
  tsylv_info& inf = info ? *info : local;
  std::memset(&inf, 0, sizeof(inf));
  int st = guarded([&]() {
    std::lock_guard<std::mutex> g(ctx->c.sync_mu);
    set_device(ctx);
    return tba_solve(ctx->c, n, s, p, A, B, C, X, o, inf);
  });
  inf.status = st;
  return st;
}

static bool batch_ok(int count, const tsylv_problem* probs, const tsylv_opts& o) {
  if (count < 1 || count > 65536 || !probs) return false;
  if (o.m < 1 || o.m > kern::kBatchMaxM || !opts_ok(o) || o.res_hist || o.x0_given > 1)
    return false;
  int64_t chunks = 0;
  for (int i = 0; i < count; ++i) {
    const tsylv_problem& q = probs[i];
    if (!q.A || !q.B || !q.C || !q.X || !dims_ok(q.n, q.s, q.p)) return false;
    chunks += (q.n * q.s * q.p + kern::kBatchChunk - 1) / kern::kBatchChunk;
  }
  return chunks < (int64_t(1) << 30);
}

size_t tsylv_batch_workspace_bytes(int count, const tsylv_problem* probs, const tsylv_opts* opts) {
  tsylv_opts o;
  tsylv_default_opts(TSYLV_METHOD_GMRES, &o);
  if (opts) o = *opts;
  if (!batch_ok(count, probs, o)) return 0;
  return batch_workspace_bytes(count, probs, o);
}

int tsylv_gmres_batch(tsylv_ctx* ctx, int count, const tsylv_problem* probs,
                      const tsylv_opts* opts, tsylv_info* infos) {
  if (!ctx || !infos) return TSYLV_EINVAL;
  tsylv_opts o;
  tsylv_default_opts(TSYLV_METHOD_GMRES, &o);
  if (opts) o = *opts;
  if (!batch_ok(count, probs, o)) return TSYLV_EINVAL;
  const char* g = std::getenv("TSYLV_BATCH_GRAPH");
  const bool use_graph = !(g && g[0] == '0');
  return guarded([&]() {
    std::lock_guard<std::mutex> lk(ctx->c.sync_mu);
    set_device(ctx);
    return gmres_batch(ctx->c, ctx->c.stream, count, probs, nullptr, o, infos, use_graph);
  });
}

size_t tsylv_tbs_batch_workspace_bytes(int count, const tsylv_problem* probs) {
  if (count < 1 || count > (1 << 20) || !probs) return 0;
  return guarded_size([&]() { return tbs_batch_workspace_bytes(count, probs); });
}

int tsylv_tbs_batch(tsylv_ctx* ctx, int count, const tsylv_problem* probs, const tsylv_opts* opts,
                    tsylv_info* infos) {
  if (!ctx || !infos || !probs || count < 1 || count > (1 << 20)) return TSYLV_EINVAL;
  if (tbs_batch_workspace_bytes(count, probs) == 0) return TSYLV_EINVAL;
  tsylv_opts o;
  tsylv_default_opts(TSYLV_METHOD_TBS, &o);
  if (opts) o.tol = opts->tol;
  if (!(o.tol >= 0.0)) return TSYLV_EINVAL;
  return guarded([&]() {
    std::lock_guard<std::mutex> lk(ctx->c.sync_mu);
    set_device(ctx);
    return tbs_batch(ctx->c, count, probs, o, infos);
  });
}

int tsylv_generate(tsylv_ctx* ctx, uint64_t seed, int64_t n, int64_t s, int64_t p, double* A,
                   double* B, double* C) {
  if (!ctx || !dims_ok(n, s, p)) return TSYLV_EINVAL;
  return guarded([&]() {
    std::lock_guard<std::mutex> g(ctx->c.sync_mu);
    set_device(ctx);
    hipStream_t st = ctx->c.stream;
    if (A) kern::gen_tensor_f64(gen_instance(seed, 0, n, s, p), A, n * n, (int)p, st);
    if (B) kern::gen_tensor_f64(gen_instance(seed, 1, n, s, p), B, s * s, (int)p, st);
    if (C) kern::gen_tensor_f64(gen_instance(seed, 2, n, s, p), C, n * s, (int)p, st);
    ctx->c.sync();
    return (int)TSYLV_OK;
  });
}

int tsylv_submit(tsylv_ctx* ctx, const tsylv_request* req, uint64_t* ticket) {
  if (!ctx || !req || !ticket) return TSYLV_EINVAL;
  tsylv_request r = *req;
  // AUTO: the direct solve for small FP64 instances, tGMRES otherwise
  if (r.method == TSYLV_METHOD_AUTO)
    r.method = (tbs_dims_ok(r.n, r.s) && !r.opts.refine && r.opts.prec == TSYLV_FP64)
                   ? TSYLV_METHOD_TBS
                   : TSYLV_METHOD_GMRES;
  const bool given = r.A && r.B && r.C, generated = !r.A && !r.B && !r.C;
  if (!(given || generated) || !r.X || !dims_ok(r.n, r.s, r.p)) return TSYLV_EINVAL;
  if (generated && r.p > kern::kGenXformMaxP) return TSYLV_EINVAL;
  if (r.method != TSYLV_METHOD_GMRES && r.method != TSYLV_METHOD_FOM &&
      r.method != TSYLV_METHOD_TBS && r.method != TSYLV_METHOD_GMRES_BATCHED)
    return TSYLV_EINVAL;
  if (r.method == TSYLV_METHOD_GMRES_BATCHED &&
      (r.opts.refine || r.opts.m > kern::kBatchMaxM || r.opts.x0_given))
    return TSYLV_EINVAL;
  if (r.method == TSYLV_METHOD_TBS && r.opts.refine) return TSYLV_EINVAL;
  if (r.method == TSYLV_METHOD_TBS && !tbs_dims_ok(r.n, r.s)) {
    // beyond the direct solve's size limit: tGMRES to the same tolerance
    r.method = TSYLV_METHOD_GMRES;
    r.opts = tbs_fallback_opts(r.opts.tol);
  }
  if (!opts_ok(r.opts)) return TSYLV_EINVAL;
  if (r.opts.res_hist) return TSYLV_EINVAL;  // no host history buffers across threads
  return guarded([&]() {
    std::lock_guard<std::mutex> g(ctx->c.sched_mu);
    if (!ctx->c.sched) {
      set_device(ctx);
      ctx->c.sched = scheduler_create(ctx->c);
    }
    *ticket = scheduler_submit(ctx->c.sched, r);
    return (int)TSYLV_OK;
  });
}

int tsylv_poll(tsylv_ctx* ctx, uint64_t ticket, tsylv_info* info) {
  if (!ctx) return TSYLV_EINVAL;
  return guarded([&]() {
    std::lock_guard<std::mutex> g(ctx->c.sched_mu);
    if (!ctx->c.sched) return (int)TSYLV_EINVAL;
    return scheduler_poll(ctx->c.sched, ticket, info);
  });
}

int tsylv_profile(tsylv_ctx* ctx, int enable) {
  if (!ctx) return TSYLV_EINVAL;
  return guarded([&]() {
    std::lock_guard<std::mutex> g(ctx->c.sync_mu);
    set_device(ctx);
    ctx->c.prof.enable(enable != 0 ? (1u << TSYLV_K_COUNT) - 1u : 0u);
    return (int)TSYLV_OK;
  });
}

int tsylv_profile_families(tsylv_ctx* ctx, unsigned mask) {
  if (!ctx || (mask >> TSYLV_K_COUNT) != 0) return TSYLV_EINVAL;
  return guarded([&]() {
    std::lock_guard<std::mutex> g(ctx->c.sync_mu);
    set_device(ctx);
    ctx->c.prof.enable(mask);
    return (int)TSYLV_OK;
  });
}

int tsylv_apply_variants(int prec) {
  if (prec != TSYLV_FP64 && prec != TSYLV_FP32 && prec != TSYLV_BF16) return TSYLV_EINVAL;
  return kern::apply_variant_count(prec);
}

int tsylv_apply_default_variant(int prec, int64_t n, int64_t s) {
  if ((prec != TSYLV_FP64 && prec != TSYLV_FP32 && prec != TSYLV_BF16) || n < 1 || s < 1)
    return TSYLV_EINVAL;
  return kern::apply_default_variant(prec, n, s);
}

int tsylv_autotune(tsylv_ctx* ctx, int64_t n, int64_t s, int64_t p, int prec, int reps,
                   int* best, float* ms, int ms_cap) {
  if (!ctx || !dims_ok(n, s, p) || tsylv_apply_variants(prec) < 0 || reps < 1 || reps > 1000 ||
      ms_cap < 0)
    return TSYLV_EINVAL;
  return guarded([&]() {
    std::lock_guard<std::mutex> g(ctx->c.sync_mu);
    set_device(ctx);
    autotune(ctx->c, n, s, p, prec, reps, best, ms, ms_cap);
    return (int)TSYLV_OK;
  });
}

int tsylv_tune_set(tsylv_ctx* ctx, int prec, int64_t n, int64_t s, int64_t p, int variant) {
  if (!ctx || !dims_ok(n, s, p)) return TSYLV_EINVAL;
  return guarded([&]() {
    ctx->c.tune.set(prec, n, s, p, variant);
    return (int)TSYLV_OK;
  });
}

int tsylv_tune_get(tsylv_ctx* ctx, int prec, int64_t n, int64_t s, int64_t p, int* variant) {
  if (!ctx || !variant || tsylv_apply_variants(prec) < 0) return TSYLV_EINVAL;
  *variant = ctx->c.tune.get(prec, n, s, p);
  return TSYLV_OK;
}

int tsylv_tune_save(tsylv_ctx* ctx, const char* path) {
  if (!ctx || !path) return TSYLV_EINVAL;
  return guarded([&]() {
    tune_save(ctx->c, path);
    return (int)TSYLV_OK;
  });
}

int tsylv_tune_load(tsylv_ctx* ctx, const char* path) {
  if (!ctx || !path) return TSYLV_EINVAL;
  return guarded([&]() {
    tune_load(ctx->c, path);
    return (int)TSYLV_OK;
  });
}

int tsylv_profile_read(tsylv_ctx* ctx, int kernel_id, tsylv_kstat* out) {
  if (!ctx || !out || kernel_id < 0 || kernel_id >= TSYLV_K_COUNT) return TSYLV_EINVAL;
  return guarded([&]() {
    std::lock_guard<std::mutex> g(ctx->c.sync_mu);
    set_device(ctx);
    ctx->c.prof.read(kernel_id, out->launches, out->total_ms);
    return (int)TSYLV_OK;
  });
}

const char* tsylv_strerror(int status) {
  switch (status) {
    case TSYLV_OK: return "ok";
    case TSYLV_NOT_CONVERGED: return "not converged (X holds the last iterate)";
    case TSYLV_PENDING: return "pending";
    case TSYLV_EINVAL: return "invalid argument";
    case TSYLV_ENOMEM: return "arena too small";
    case TSYLV_EBREAKDOWN:
      return "breakdown: non-invertible tube in Normalization, or a Schur iteration that did "
             "not converge";
    case TSYLV_ESINGULAR: return "singular (projected) problem";
    case TSYLV_EHIP: return "HIP runtime error";
    case TSYLV_ECANCELLED: return "cancelled";
    case TSYLV_ESCRATCH:
      return "sizes exceed the static scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}

}  // extern "C"
