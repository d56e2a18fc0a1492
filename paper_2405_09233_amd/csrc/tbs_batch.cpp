// t-Bartels-Stewart (section 4: Algorithm 4, t-Schur, and Algorithm 5) for a
// batch of small independent instances in one pass: the forward transforms
// of every A, B and C in one launch, the slice solves of every instance in
// one launch (one wavefront per (instance, Fourier slice)), the FP64
// residual in the Fourier planes and its per-instance norms in two more, the
// inverse transforms of every X in one, and one synchronisation.  Each
// instance's arithmetic is that of its own solve: the kernels read only its
// tables, and its norms are summed in slice order.  Instances beyond the
// direct solve's size limit (n or s above 64) are solved by tGMRES instead
// (the batched tGMRES executors, after the direct pass).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <map>
#include <vector>

#include "kernels.hpp"
#include "runtime.hpp"
#include "solvers.hpp"

namespace tsylv {

namespace {

int64_t blocks_of(int64_t E) {
  return (E + kern::kBatchXformBlock - 1) / kern::kBatchXformBlock;
}

bool tbs_batch_dims_ok(const tsylv_problem& q) {
  return q.n >= 1 && q.s >= 1 && q.n <= kern::tbs_max_size() && q.s <= kern::tbs_max_size() &&
         q.p >= 1 && q.p <= 4096 && q.A && q.B && q.C && q.X;
}

// A well-formed instance beyond the direct solve's size limit.
bool tbs_fallback_instance(const tsylv_problem& q) {
  return q.n >= 1 && q.s >= 1 && (q.n > kern::tbs_max_size() || q.s > kern::tbs_max_size()) &&
         q.p >= 1 && q.p <= 4096 && q.A && q.B && q.C && q.X;
}

// Splits a batch into the direct solve's instances and the others; false
// when an instance is malformed.
bool split_batch(int count, const tsylv_problem* probs, std::vector<int>& direct,
                 std::vector<int>& krylov) {
  for (int i = 0; i < count; ++i) {
    if (tbs_batch_dims_ok(probs[i]))
      direct.push_back(i);
    else if (tbs_fallback_instance(probs[i]))
      krylov.push_back(i);
    else
      return false;
  }
  return true;
}

std::vector<tsylv_problem> pick(const tsylv_problem* probs, const std::vector<int>& ids) {
  std::vector<tsylv_problem> out;
  for (int i : ids) out.push_back(probs[i]);
  return out;
}

size_t direct_workspace_bytes(int count, const tsylv_problem* probs);
int direct_batch(Ctx& ctx, int count, const tsylv_problem* probs, const tsylv_opts& o,
                 tsylv_info* infos);

}  // namespace

tsylv_opts tbs_fallback_opts(double tol) {
  tsylv_opts o;
  tsylv_default_opts(TSYLV_METHOD_GMRES, &o);
  o.tol = tol;
  return o;
}

size_t tbs_batch_workspace_bytes(int count, const tsylv_problem* probs) {
  if (count <= 0 || !probs) return 0;
  std::vector<int> direct, krylov;
  if (!split_batch(count, probs, direct, krylov)) return 0;
  size_t d = 0, k = 0;
  if (!direct.empty()) {
    const std::vector<tsylv_problem> dp = pick(probs, direct);
    d = direct_workspace_bytes((int)dp.size(), dp.data());
    if (d == 0) return 0;
  }
  if (!krylov.empty()) {
    const std::vector<tsylv_problem> kp = pick(probs, krylov);
    k = batch_workspace_bytes((int)kp.size(), kp.data(), tbs_fallback_opts(1e-8));
    if (k == 0) return 0;
  }
  return std::max(d, k);  // the two parts run one after the other
}

int tbs_batch(Ctx& ctx, int count, const tsylv_problem* probs, const tsylv_opts& o,
              tsylv_info* infos) {
  std::vector<int> direct, krylov;
  if (!split_batch(count, probs, direct, krylov))
    throw Error(TSYLV_EINVAL, "tbs batch: bad instance");
  int worst = TSYLV_OK;
  if (!direct.empty()) {
    const std::vector<tsylv_problem> dp = pick(probs, direct);
    std::vector<tsylv_info> di(dp.size());
    if (direct_batch(ctx, (int)dp.size(), dp.data(), o, di.data()) != TSYLV_OK)
      worst = TSYLV_NOT_CONVERGED;
    for (size_t k = 0; k < direct.size(); ++k) infos[direct[k]] = di[k];
  }
  if (!krylov.empty()) {
    const std::vector<tsylv_problem> kp = pick(probs, krylov);
    std::vector<tsylv_info> ki(kp.size());
    const char* g = std::getenv("TSYLV_BATCH_GRAPH");
    if (gmres_batch(ctx, ctx.stream, (int)kp.size(), kp.data(), nullptr, tbs_fallback_opts(o.tol),
                    ki.data(), !(g && g[0] == '0')) != TSYLV_OK)
      worst = TSYLV_NOT_CONVERGED;
    for (size_t k = 0; k < krylov.size(); ++k) infos[krylov[k]] = ki[k];
  }
  return worst;
}

namespace {

size_t direct_workspace_bytes(int count, const tsylv_problem* probs) {
  if (count <= 0 || !probs) return 0;
  size_t b = 0;
  std::map<int64_t, int> ps;
  int64_t slices = 0;
  for (int i = 0; i < count; ++i) {
    const tsylv_problem& q = probs[i];
    if (!tbs_batch_dims_ok(q)) return 0;
    const int64_t N = q.n * q.s * q.p;
    b += Workspace::bytes_for(q.p * q.n * q.n, 8) + Workspace::bytes_for(q.p * q.s * q.s, 8) +
         2 * Workspace::bytes_for(N, 8) +
         Workspace::bytes_for(2 * kern::tbs_scratch_complex(q.n, q.s, (int)q.p), 8);
    ps[q.p] = 1;
    slices += num_slices((int)q.p);
  }
  for (auto& kv : ps) b += 3 * Workspace::bytes_for(kv.first * kv.first, 8);
  b += Workspace::bytes_for(count, sizeof(kern::TbsArgs)) +
       Workspace::bytes_for(count + 1, sizeof(int)) + Workspace::bytes_for(count, sizeof(int)) +
       Workspace::bytes_for(4 * (int64_t)count, sizeof(kern::XformDesc)) +
       Workspace::bytes_for(4 * (int64_t)count + 1, sizeof(int)) +
       Workspace::bytes_for(2 * slices, 8) + Workspace::bytes_for(2 * (int64_t)count, 8);
  return b;
}

int direct_batch(Ctx& ctx, int count, const tsylv_problem* probs, const tsylv_opts& o,
                 tsylv_info* infos) {
  const auto t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < count; ++i)
    if (!tbs_batch_dims_ok(probs[i])) throw Error(TSYLV_EINVAL, "tbs batch: bad instance");
  hipStream_t st = ctx.stream;
  Workspace ws(ctx.arena, direct_workspace_bytes(count, probs));
  // transform matrices, one set per distinct p
  struct Mats {
    double *op, *fwd, *inv;
  };
  std::map<int64_t, Mats> mats;
  for (int i = 0; i < count; ++i) {
    const int64_t p = probs[i].p;
    if (mats.count(p)) continue;
    Mats M{ws.take<double>(p * p), ws.take<double>(p * p), ws.take<double>(p * p)};
    kern::build_xform(M.op, (int)p, XF_OPERATOR, st);
    kern::build_xform(M.fwd, (int)p, XF_FORWARD, st);
    kern::build_xform(M.inv, (int)p, XF_INVERSE, st);
    mats[p] = M;
  }
  std::vector<kern::TbsArgs> args(count);
  std::vector<int> first(count + 1, 0);
  std::vector<kern::XformDesc> fwd, inv;
  int* d_info = nullptr;
  {
    // per-instance planes and scratch
    std::vector<double*> Ah(count), Bh(count), Zc(count), Zx(count), scr(count);
    for (int i = 0; i < count; ++i) {
      const tsylv_problem& q = probs[i];
      const int64_t N = q.n * q.s * q.p;
      Ah[i] = ws.take<double>(q.p * q.n * q.n);
      Bh[i] = ws.take<double>(q.p * q.s * q.s);
      Zc[i] = ws.take<double>(N);
      Zx[i] = ws.take<double>(N);
      scr[i] = ws.take<double>(2 * kern::tbs_scratch_complex(q.n, q.s, (int)q.p));
    }
    d_info = ws.take<int>(count);
    for (int i = 0; i < count; ++i) {
      const tsylv_problem& q = probs[i];
      const Mats& M = mats[q.p];
      args[i] = kern::TbsArgs{Ah[i], Bh[i], Zc[i], Zx[i], reinterpret_cast<double2*>(scr[i]),
                              d_info + i, (int)q.n, (int)q.s, (int)q.p};
      first[i + 1] = first[i] + num_slices((int)q.p);
      fwd.push_back({q.A, Ah[i], M.op, q.n * q.n, (int)q.p});
      fwd.push_back({q.B, Bh[i], M.op, q.s * q.s, (int)q.p});
      fwd.push_back({q.C, Zc[i], M.fwd, q.n * q.s, (int)q.p});
      inv.push_back({Zx[i], q.X, M.inv, q.n * q.s, (int)q.p});
    }
  }
  const int total_slices = first[count];
  auto bfirst_of = [](const std::vector<kern::XformDesc>& d) {
    std::vector<int> bf(d.size() + 1, 0);
    for (size_t i = 0; i < d.size(); ++i) bf[i + 1] = bf[i] + (int)blocks_of(d[i].E);
    return bf;
  };
  const std::vector<int> bf_fwd = bfirst_of(fwd), bf_inv = bfirst_of(inv);
  kern::TbsArgs* d_args = ws.take<kern::TbsArgs>(count);
  int* d_first = ws.take<int>(count + 1);
  kern::XformDesc* d_desc = ws.take<kern::XformDesc>(4 * (int64_t)count);
  int* d_bf = ws.take<int>(4 * (int64_t)count + 1);
  double* d_part = ws.take<double>(2 * (int64_t)total_slices);
  double* d_norms = ws.take<double>(2 * (int64_t)count);
  // tables: forward descriptors first, then the inverse ones (with their own
  // block offsets) right behind them
  std::vector<kern::XformDesc> descs(fwd);
  descs.insert(descs.end(), inv.begin(), inv.end());
  std::vector<int> bfs(bf_fwd);
  bfs.insert(bfs.end(), bf_inv.begin(), bf_inv.end());
  TSYLV_HIP(hipMemcpyAsync(d_args, args.data(), sizeof(kern::TbsArgs) * count,
                           hipMemcpyHostToDevice, st));
  TSYLV_HIP(hipMemcpyAsync(d_first, first.data(), sizeof(int) * (count + 1),
                           hipMemcpyHostToDevice, st));
  TSYLV_HIP(hipMemcpyAsync(d_desc, descs.data(), sizeof(kern::XformDesc) * descs.size(),
                           hipMemcpyHostToDevice, st));
  TSYLV_HIP(hipMemcpyAsync(d_bf, bfs.data(), sizeof(int) * bfs.size(), hipMemcpyHostToDevice, st));
  TSYLV_HIP(hipMemsetAsync(d_info, 0, sizeof(int) * count, st));
  // Algorithm 1 step 1 for every instance, the slice solves and the
  // residual, Algorithm 1 step 3 for every X
  kern::batch_xform(d_desc, d_bf, (int)fwd.size(), bf_fwd.back(), st);
  kern::tbs_batch(d_args, d_first, count, total_slices, d_part, d_norms, st);
  kern::batch_xform(d_desc + fwd.size(), d_bf + bf_fwd.size(), (int)inv.size(), bf_inv.back(),
                    st);
  std::vector<double> norms(2 * (size_t)count);
  std::vector<int> flags(count);
  TSYLV_HIP(hipMemcpyAsync(norms.data(), d_norms, norms.size() * 8, hipMemcpyDeviceToHost, st));
  TSYLV_HIP(hipMemcpyAsync(flags.data(), d_info, flags.size() * sizeof(int),
                           hipMemcpyDeviceToHost, st));
  ctx.sync();
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  bool all_ok = true;
  for (int i = 0; i < count; ++i) {
    tsylv_info& inf = infos[i];
    inf = tsylv_info{};
    inf.seconds = secs;
    const double rr = norms[2 * i], cc = norms[2 * i + 1];
    inf.relres_true = cc > 0.0 ? std::sqrt(rr / cc) : (rr > 0.0 ? INFINITY : 0.0);
    if (flags[i] == 1)
      inf.status = TSYLV_EBREAKDOWN;
    else if (flags[i] == 2)
      inf.status = TSYLV_ESINGULAR;
    else
      inf.status = inf.relres_true <= o.tol ? TSYLV_OK : TSYLV_NOT_CONVERGED;
    all_ok = all_ok && inf.status == TSYLV_OK;
  }
  return all_ok ? TSYLV_OK : TSYLV_NOT_CONVERGED;
}

}  // namespace

}  // namespace tsylv
