// Driver entry points used by the C ABI.
#pragma once

#include "kernels.hpp"
#include "runtime.hpp"

namespace tsylv {

// Fourier-domain state shared by the solvers: unscaled DFT planes of A and B,
// orthonormal planes of C and X, and the three p x p tube transforms.
struct Setup {
  double *Ah, *Bh, *xf_op, *xf_fwd, *xf_inv, *Zc, *Zx;
};
size_t setup_bytes(int64_t n, int64_t s, int64_t p);
// With `gen` non-null, A, B and C are not read: the instance of seed *gen
// (gen_instance) is drawn inside the transforms (p <= 64).
Setup setup_fourier(Ctx& ctx, hipStream_t st, bool profile, Workspace& ws, int64_t n, int64_t s,
                    int64_t p, const double* A, const double* B, const double* C, const double* X,
                    bool x0_given, const uint64_t* gen = nullptr);

// The synthetic dense instance of `seed` (p-scaled noise): tensor `which`
// (0: A, 1: B, 2: C) of the counter-based stream.  A = 2/sqrt(n p) Z + 4 I
// and B = 2/sqrt(s p) Z - 4 I on frontal slice 1, C = Z.
kern::GenTensor gen_instance(uint64_t seed, int which, int64_t n, int64_t s, int64_t p);

size_t tba_workspace_bytes(int64_t n, int64_t s, int64_t p, int m);
int tba_solve(Ctx& ctx, int64_t n, int64_t s, int64_t p, const double* A, const double* B,
              const double* C, double* X, const tsylv_opts& o, tsylv_info& info);

size_t apply_workspace_bytes(int64_t n, int64_t s, int64_t p);
int apply_spatial(Ctx& ctx, int64_t n, int64_t s, int64_t p, const double* A, const double* B,
                  const double* X, double* Y, int prec);
// The same with every buffer carved from `buf` (bytes >= apply_workspace_bytes),
// enqueued on `st` without synchronising; default tiles.
void apply_spatial_into(char* buf, size_t bytes, hipStream_t st, int64_t n, int64_t s,
                        int64_t p, const double* A, const double* B, const double* X, double* Y,
                        int prec);

size_t krylov_workspace_bytes(int method, int64_t n, int64_t s, int64_t p, const tsylv_opts& o);
int krylov_solve(Ctx& ctx, int method, int64_t n, int64_t s, int64_t p, const double* A,
                 const double* B, const double* C, double* X, const tsylv_opts& o,
                 tsylv_info& info);

// Batched tGMRES (batch.cpp): FP64 instances that fit one workgroup solved
// whole by one launch, other small FP64 instances (n s p <= 2^18) in
// lockstep (restart length o.m <= 63), the rest, and every instance of a
// refined batch, as concurrent solves on eight streams; workspace of all.
size_t batch_workspace_bytes(int count, const tsylv_problem* probs, const tsylv_opts& o);
// Workspace of the lockstep executor alone (every instance in lockstep).
size_t lockstep_workspace_bytes(int count, const tsylv_problem* probs, const tsylv_opts& o);
// Workspace of a batch run without the stream executor (no_streams).
size_t served_batch_bytes(int count, const tsylv_problem* probs, const tsylv_opts& o);
// True when a batch solves this instance whole in one workgroup (the single
// solve's criterion): its result is then bitwise that of tsylv_gmres.
bool batch_solves_whole(const tsylv_problem& q, const tsylv_opts& o);
// Batched t-Bartels-Stewart (tbs_batch.cpp); instances with n or s above 64
// by tGMRES (tbs_fallback_opts with the batch's tolerance) after the direct
// pass.  0 bytes when an instance has n, s or p < 1, p > 4096 or a null
// pointer.
size_t tbs_batch_workspace_bytes(int count, const tsylv_problem* probs);
// The tGMRES options that stand in for the direct solve beyond its size
// limit: the tGMRES defaults with the caller's tolerance.
tsylv_opts tbs_fallback_opts(double tol);
int tbs_batch(Ctx& ctx, int count, const tsylv_problem* probs, const tsylv_opts& o,
              tsylv_info* infos);
// On stream `st`; gens (may be null): gens[i] non-null draws instance i as
// the synthetic instance of seed *gens[i] (its A, B, C are not read).
// no_streams: no stream executor -- the instances it would take run in
// lockstep (FP64 batches of the serving loop, which runs its batches
// concurrently itself; the stream executor's pinned staging is the
// context's, for one caller at a time); instances that fit one workgroup
// keep that executor, so a served instance computes what its batch of one
// does.  arena (may be null: the context's): where the single-workgroup and
// lockstep executors take their workspaces (the serving loop passes a block
// reserved for the batch when it admitted it; the stream executor's solves
// always take the context's).
int gmres_batch(Ctx& ctx, hipStream_t st, int count, const tsylv_problem* probs,
                const uint64_t* const* gens, const tsylv_opts& o, tsylv_info* infos,
                bool use_graph, bool no_streams = false, Arena* arena = nullptr);

// Autotuner (tune.cpp): times every tile variant of the apply at (n, s, p)
// in precision `prec` (`reps` launches each), stores the fastest in
// ctx.tune and returns the number of variants; ms_out[v] (v < ms_cap) gets
// variant v's average launch time.
int autotune(Ctx& ctx, int64_t n, int64_t s, int64_t p, int prec, int reps, int* best,
             float* ms_out, int ms_cap);
void tune_save(const Ctx& ctx, const char* path);
void tune_load(Ctx& ctx, const char* path);

}  // namespace tsylv
