/*
 * tsylv.h -- C ABI of the MI355X tensor Krylov solvers for the Sylvester
 * tensor equation  M(X) = A*X - X*B = C  under the T-product.
 *
 * The operation is defined in section 1, eq. (2) and section 5.2 of
 * Bouyghf, El Guide, El Ichi, "Tensor Krylov subspace methods via the
 * T-product for large Sylvester tensor equations" (arXiv 2405.09233);
 * the T-product is the definition of section 2.1.
 *
 * Tensor layout (every tensor argument): real, frontal-slice major,
 * column-major inside a slice (MATLAB order):
 *     T[i + rows*j + rows*cols*k],  0 <= i < rows, 0 <= j < cols, 0 <= k < p.
 *   A: n x n x p,   B: s x s x p,   C, X, Y: n x s x p.
 * All tensor pointers are DEVICE pointers (HBM of the context's GPU), 8-byte
 * aligned, holding float64.  The caller owns them; the library never frees
 * or retains them after a synchronous call returns.
 *
 * Errors: every call returns a tsylv_status.  Negative values are errors and
 * leave nothing guaranteed in the output tensor; TSYLV_NOT_CONVERGED leaves
 * the best iterate in X.  No exception crosses this boundary.  A context is
 * not thread-safe, except that tsylv_submit and tsylv_poll may be called from
 * any thread.
 *
 * Environment switches (read at each call; each selects another code path
 * for the same mathematics, for comparisons and measurements):
 *   TSYLV_KRYLOV_TINY=0         no single-workgroup solve of small instances
 *                               (tGMRES/tFOM, batches, served requests)
 *   TSYLV_KRYLOV_CGS2=1         three-sweep CGS2 instead of the delayed form
 *   TSYLV_KRYLOV_DEVICE_CYCLE   refined solves' inner cycles on the device:
 *                               1 (default) after a full cycle, 2 always, 0 never
 *   TSYLV_BF16_BASIS=fp32       BF16-refined solves keep an FP32 inner basis
 *   TSYLV_BATCH_GRAPH=0         lockstep batch steps launched, not replayed
 *                               from a recorded HIP graph (bitwise the same)
 *   TSYLV_TBA_HOST_PROJECTED=1  TBAS's projected equation solved on the host
 */
#ifndef TSYLV_H
#define TSYLV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tsylv_ctx tsylv_ctx;

/* Precision of the operator applies of the inner solve. */
typedef enum {
  TSYLV_FP64 = 0, /* everything in FP64                                     */
  TSYLV_FP32 = 1, /* FP32 copies of the Fourier slices, FP32 basis vectors   */
  TSYLV_BF16 = 2  /* BF16 copies of the Fourier slices (FP32 accumulation)   */
} tsylv_prec;

typedef enum {
  TSYLV_METHOD_GMRES = 0, /* tGMRES(m), Algorithm 3                        */
  TSYLV_METHOD_FOM = 1,   /* tFOM(m), Algorithm 3                          */
  TSYLV_METHOD_TBA = 2,   /* TBAS(m), Algorithm 8 (block size s)           */
  TSYLV_METHOD_TBS = 3,   /* t-Bartels-Stewart direct solve, Algorithm 5
                             (n or s above 64: tGMRES(30), see tsylv_tbs)   */
  TSYLV_METHOD_GMRES_BATCHED = 4, /* tGMRES(m) served in lockstep batches
                                     (tsylv_submit only; see below)         */
  TSYLV_METHOD_AUTO = 5  /* tsylv_submit only: the t-Bartels-Stewart direct
                            solve when n, s <= 64 and the request is FP64
                            without refinement, else tGMRES(m)              */
} tsylv_method;

typedef enum {
  TSYLV_OK = 0,
  TSYLV_NOT_CONVERGED = 1, /* max_cycles reached; X holds the last iterate  */
  TSYLV_PENDING = 2,       /* tsylv_poll: request not finished yet          */
  TSYLV_EINVAL = -1,       /* bad size, pointer or option                   */
  TSYLV_ENOMEM = -2,       /* arena too small for the workspace             */
  TSYLV_EBREAKDOWN = -3,   /* non-invertible tube in Normalization (TBA)    */
  TSYLV_ESINGULAR = -4,    /* singular projected problem                    */
  TSYLV_EHIP = -5,         /* HIP runtime error                             */
  TSYLV_ECANCELLED = -6,   /* request dropped (context destroyed)           */
  TSYLV_ESCRATCH = -7      /* sizes beyond the static scratch of
                              tsylv_apply_noalloc                           */
} tsylv_status;

/* Solver options (Algorithm 3 and Algorithm 8 inputs: m, Iter_max, tol, X0). */
typedef struct {
  int m;            /* restart length (Krylov steps per cycle)              */
  int max_cycles;   /* Iter_max: maximum number of restart cycles           */
  double tol;       /* stop when ||C - M(X)||_F / ||C||_F <= tol            */
  int x0_given;     /* 1: X holds the initial guess on entry; 0: X0 = 0     */
  int prec;         /* tsylv_prec of the inner applies                      */
  int refine;       /* 1: FP64 iterative refinement around a prec solve     */
  int inner_m;      /* restart length of the inner solve (refine = 1)       */
  double inner_tol; /* relative tolerance of each inner solve               */
  int max_outer;    /* maximum refinement steps                             */
  double* res_hist; /* optional HOST buffer: relative residual estimates   */
  int res_hist_cap; /* capacity of res_hist (entries)                       */
} tsylv_opts;

/* Result record of a solve. */
typedef struct {
  int status;         /* tsylv_status of the solve                          */
  int steps;          /* applies of M inside Arnoldi (total over cycles)    */
  int cycles;         /* restart cycles run                                 */
  int outer;          /* refinement steps (0 without refinement)           */
  double relres_true; /* ||C - M(X)||_F / ||C||_F, recomputed in FP64       */
  double relres_est;  /* last cheap estimate (|gamma|, h|y|, ||H E Y||)     */
  double seconds;     /* wall time of the call                              */
  int res_hist_len;   /* entries written to opts->res_hist                  */
  int fom_fallback;   /* tFOM cycles that fell back to the tGMRES solution  */
} tsylv_info;

/* Defaults: m = 30 (tGMRES/tFOM) or 10 (TBA), max_cycles = 500,
 * tol = 1e-8, X0 = 0, FP64, no refinement, inner_m = 40, inner_tol = 1e-4,
 * max_outer = 500.
 * Precision rules: without refinement prec must be TSYLV_FP64; with
 * refine = 1, prec is TSYLV_FP32 or TSYLV_BF16 and each refinement step is
 * one tGMRES/tFOM(inner_m) cycle in that precision, stopped early when its
 * residual estimate falls below inner_tol times the current FP64 residual;
 * X, the residual and the stopping test stay FP64. */
void tsylv_default_opts(int method, tsylv_opts* opts);

/* Create a context on HIP device `device`, issuing all work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  `arena` is a DEVICE buffer of
 * `arena_bytes` bytes owned by the caller that holds every workspace the
 * library needs (the HBM budget); it must outlive the context.  If `arena`
 * is NULL the library allocates `arena_bytes` itself at creation (never on
 * the solve path) and frees it in tsylv_destroy. */
int tsylv_create(tsylv_ctx** out, int device, void* hip_stream, void* arena,
                 size_t arena_bytes);

/* Destroy a context: waits for submitted requests (cancelling those not yet
 * admitted), then releases everything the library allocated. */
int tsylv_destroy(tsylv_ctx* ctx);

/* Arena bytes one synchronous call of `method` needs for these sizes
 * (method = -1: tsylv_apply).  0 on invalid arguments. */
size_t tsylv_workspace_bytes(int method, int64_t n, int64_t s, int64_t p,
                             const tsylv_opts* opts);

/* Y = A*X - X*B  (eq. (2)), computed as Algorithm 1 of section 2.1 does:
 * mode-3 DFT, facewise products on the conjugate-symmetric half of the
 * Fourier slices, inverse DFT.  The transforms are FP64; `prec` selects the
 * precision of the slice products (FP64, FP32, or BF16 inputs with FP32
 * accumulation).  Synchronous on the context stream. */
int tsylv_apply(tsylv_ctx* ctx, int64_t n, int64_t s, int64_t p,
                const double* A, const double* B, const double* X, double* Y,
                int prec);

/* tsylv_apply for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same Y = A*X - X*B with every intermediate buffer in a static device
 * array of tsylv_noalloc_scratch_bytes() (256 MiB) that each GPU the library
 * runs on holds until the process ends; the call allocates nothing and takes
 * no context.  Runs on the current HIP device, enqueued on `hip_stream` (a
 * hipStream_t; NULL = the null stream), and returns without synchronising:
 * Y is ready when the stream reaches this point.  Default tile shapes (no
 * tuning table).  Every call on a GPU shares that GPU's scratch, so calls
 * that overlap on one GPU (on different streams, or from threads with no
 * ordering between them) race; calls in order on one stream do not.
 * TSYLV_ESCRATCH (and nothing enqueued) when the sizes need more scratch
 * than that (the workspace of tsylv_apply, tsylv_workspace_bytes(-1, ...));
 * TSYLV_EINVAL for bad sizes, pointers or precision. */
size_t tsylv_noalloc_scratch_bytes(void);
int tsylv_apply_noalloc(void* hip_stream, int64_t n, int64_t s, int64_t p, const double* A,
                        const double* B, const double* X, double* Y, int prec);

/* tFOM(m), Algorithm 3 of section 3 (Galerkin condition, section 3.2). */
int tsylv_fom(tsylv_ctx* ctx, int64_t n, int64_t s, int64_t p, const double* A,
              const double* B, const double* C, double* X,
              const tsylv_opts* opts, tsylv_info* info);

/* tGMRES(m), Algorithm 3 of section 3 (minimal residual, section 3.3).
 * With opts->refine = 1: FP64 iterative refinement whose correction
 * equations are solved by tGMRES(inner_m) in opts->prec. */
int tsylv_gmres(tsylv_ctx* ctx, int64_t n, int64_t s, int64_t p,
                const double* A, const double* B, const double* C, double* X,
                const tsylv_opts* opts, tsylv_info* info);

/* TBAS(m), Algorithm 8 of section 5.2: Tubal Block Arnoldi on A with block
 * size s, projected equation H_m*Y - Y*B = V_m^T*R0 solved per Fourier
 * slice in FP64. */
int tsylv_tba(tsylv_ctx* ctx, int64_t n, int64_t s, int64_t p, const double* A,
              const double* B, const double* C, double* X,
              const tsylv_opts* opts, tsylv_info* info);

/* t-Bartels-Stewart, Algorithm 5 of section 4 (with the t-Schur
 * decomposition of Algorithm 4): the direct method for small sizes,
 * 1 <= n, s <= 64.  Beyond that the call solves the same equation by
 * tGMRES(30) (the tGMRES defaults with opts->tol; info->steps > 0 tells
 * the two apart, and tsylv_workspace_bytes(TSYLV_METHOD_TBS, ...) is then
 * that tGMRES's workspace).  Each Fourier slice is reduced
 * to complex Schur form on the GPU (one wavefront per slice), the triangular
 * equation solved by back substitution and transformed back.  Only opts->tol
 * is read (opts may be NULL): the status is TSYLV_OK when the true relative
 * residual, recomputed in FP64 and returned in info->relres_true, is <= tol,
 * else TSYLV_NOT_CONVERGED with the direct solution in X;
 * TSYLV_ESINGULAR when a slice's spectra of Ahat and Bhat meet (no unique
 * solution), TSYLV_EBREAKDOWN when a Schur iteration does not converge. */
int tsylv_tbs(tsylv_ctx* ctx, int64_t n, int64_t s, int64_t p, const double* A,
              const double* B, const double* C, double* X,
              const tsylv_opts* opts, tsylv_info* info);

/* Batched solves (a project addition for workloads of many independent
 * instances of uneven size; the method per instance is Algorithm 3 --
 * restarted tGMRES(m) -- optionally inside FP64 iterative refinement as in
 * tsylv_gmres).  Each instance runs on the executor that suits it, chosen
 * from the instance alone:
 *   - FP64 instances small enough for a whole solve in one workgroup (those
 *     tsylv_gmres itself solves that way: n s p, the operator planes and
 *     two basis vectors within the workgroup's LDS, m n s p <= 2^18) are
 *     solved by one launch for all of them, a workgroup per instance
 *     running its whole Algorithm 3; each result is bitwise the
 *     tsylv_gmres solve with these opts;
 *   - other small FP64 instances (n s p <= 2^18) advance in lockstep: every kernel
 *     launch of an Arnoldi step serves all of them (work items over the
 *     instances' tiles and vector chunks; classical Gram-Schmidt applied
 *     twice), the Givens rotations and the stop tests run on the device,
 *     and the step is recorded once as a HIP graph and replayed, so the host
 *     synchronises a few times per cycle rather than per instance and step;
 *   - larger instances, and every instance of a refined batch (refine = 1,
 *     prec FP32 or BF16), run as independent solves on up to eight streams
 *     at once, each advanced as its stream finishes a phase, so that the
 *     apply of one overlaps the Gram-Schmidt sweeps of another; each such
 *     result is bitwise the synchronous tsylv_gmres solve with these opts.
 * opts: 1 <= m <= 63; tol, max_cycles, x0_given and the refinement options
 * as for tsylv_gmres (opts may be NULL: m = 30).  Each instance's result
 * does not depend on the rest of the batch (it is bitwise the same alone).
 * infos[i] receives instance i's record (seconds: the whole batch).
 * Returns TSYLV_OK when every instance converged, TSYLV_NOT_CONVERGED when
 * some did not or failed (see infos), or an error for the batch.
 * tsylv_batch_workspace_bytes: the arena bytes the call needs. */
typedef struct {
  int64_t n, s, p;
  const double* A;  /* device pointers, layout as above */
  const double* B;
  const double* C;
  double* X;        /* output (and X0 when opts.x0_given) */
} tsylv_problem;

size_t tsylv_batch_workspace_bytes(int count, const tsylv_problem* probs, const tsylv_opts* opts);
int tsylv_gmres_batch(tsylv_ctx* ctx, int count, const tsylv_problem* probs,
                      const tsylv_opts* opts, tsylv_info* infos);

/* t-Bartels-Stewart (Algorithm 5 of section 4, with the t-Schur
 * decomposition of Algorithm 4) for a batch of small independent instances
 * (1 <= n, s <= 64, 1 <= p <= 4096 each; sizes may differ), in one pass:
 * one launch transforms every A, B and C (mode-3 DFT), one solves every
 * Fourier slice of every instance (one wavefront per (instance, slice):
 * complex Schur forms, triangular Sylvester back substitution), two form the
 * FP64 residual C - M(X) of every instance in the Fourier planes and its
 * norm, one transforms every X back; the host synchronises once.  Only
 * opts->tol is read (opts may be NULL: 1e-8).  infos[i]: TSYLV_OK when
 * instance i's true relative residual (relres_true) is <= tol, else
 * TSYLV_NOT_CONVERGED with the direct solution in X; TSYLV_ESINGULAR when a
 * slice's spectra of Ahat and Bhat meet, TSYLV_EBREAKDOWN when a Schur
 * iteration does not converge; seconds is the whole batch's time.
 * Instances with n or s above 64 (p <= 4096) are solved after that pass by
 * tGMRES(30) to the same tolerance, as tsylv_gmres_batch runs them (their
 * infos report Krylov steps); the workspace is the larger of the two
 * parts'.  Returns TSYLV_OK when every instance is TSYLV_OK,
 * TSYLV_NOT_CONVERGED otherwise, or an error of the whole batch
 * (TSYLV_EINVAL for an instance with n, s or p < 1, p > 4096 or a NULL
 * pointer; TSYLV_ENOMEM, TSYLV_EHIP).  Synchronous on the context stream. */
size_t tsylv_tbs_batch_workspace_bytes(int count, const tsylv_problem* probs);
int tsylv_tbs_batch(tsylv_ctx* ctx, int count, const tsylv_problem* probs,
                    const tsylv_opts* opts, tsylv_info* infos);

/* Synthetic instances drawn on the device (a project addition for serving
 * workloads; not in the paper).  Writes the dense instance of `seed`:
 *   A = 2/sqrt(n p) Z_A + 4 I,  B = 2/sqrt(s p) Z_B - 4 I  (the identity on
 *   frontal slice 1 only),  C = Z_C,
 * with Z i.i.d. N(0,1) from a counter-based stream: Philox4x64-10 (Salmon
 * et al., SC'11) keyed by (seed, tensor id: A 0, B 1, C 2); element (i,j,k)
 * of a rows x cols x p tensor, e = i + rows*j, takes the block at counter
 * (e, k/4, 0, 0); its words w give uniforms ((w >> 12) + 1/2) 2^-52 and
 * Box-Muller pairs (cos, sin) for k%4 = 0,1 from words 0,1 and k%4 = 2,3
 * from words 2,3.  The product with the scale is rounded, then the shift
 * added.  The noise scaling keeps the spectra of the Fourier slices of A and
 * B about 4 apart for every p, so the equation is uniquely solvable.
 * A (n x n x p), B (s x s x p), C (n x s x p): device pointers in the layout
 * above, any of them NULL to skip it.  Runs on the context stream and returns
 * after completion.  Values agree with a host evaluation of the same
 * definition to the rounding of log, sin and cos. */
int tsylv_generate(tsylv_ctx* ctx, uint64_t seed, int64_t n, int64_t s, int64_t p, double* A,
                   double* B, double* C);

/* Asynchronous solves (continuous batching).  A request is admitted when its
 * workspace fits in the arena; admitted requests are stepped together on the
 * GPU.  Requests of method TSYLV_METHOD_GMRES_BATCHED (FP64, m <= 63, X0 =
 * 0) that wait in the queue together with equal options are admitted as one
 * batch run by tsylv_gmres_batch's in-GPU executors (instances that fit one
 * workgroup: one launch for all of them; the others in lockstep: one launch
 * per step stage for all of them, the step replayed from a HIP graph,
 * Givens on the device); each result is bitwise the batch-of-one solve of
 * its instance.  Plain tGMRES requests (FP64, m <= 63) whose instance fits
 * the one-workgroup solve join such batches too (consecutive requests with
 * equal m, tol, max_cycles and x0_given): they run the kernel of their
 * synchronous solve, so each result is bitwise tsylv_gmres's, and `seconds`
 * is the batch's wall time.  The pointers in the request must stay valid until tsylv_poll returns
 * a final status for its ticket.  A request with A, B and C all NULL solves
 * the synthetic instance of `gen_seed` (tsylv_generate), drawn on the device
 * inside its setup transforms, so that the spatial tensors are never stored
 * (p <= 64; the generation counts in the request's latency). */
typedef struct {
  int method;                 /* tsylv_method (GMRES, FOM, TBS, GMRES_BATCHED) */
  int64_t n, s, p;
  const double* A;            /* device pointers, layout as above           */
  const double* B;
  const double* C;
  double* X;                  /* output (and X0 when opts.x0_given)         */
  tsylv_opts opts;
  uint64_t gen_seed;          /* instance seed when A, B and C are NULL     */
} tsylv_request;

/* Queue a request; returns at once with a ticket. */
int tsylv_submit(tsylv_ctx* ctx, const tsylv_request* req, uint64_t* ticket);

/* TSYLV_PENDING while the request runs; otherwise its final status, with
 * `info` filled (info may be NULL).  A ticket may be polled after it is
 * final, until the context is destroyed. */
int tsylv_poll(tsylv_ctx* ctx, uint64_t ticket, tsylv_info* info);

/* Kernel timing for benchmarks.  While enabled, every launch of a timed
 * kernel family is bracketed by HIP events recorded on the context stream
 * (the stream the kernels run on); tsylv_profile_read folds the elapsed
 * times into per-family totals.  Off by default. */
typedef enum {
  TSYLV_K_APPLY = 0,     /* FP64 facewise apply  Ahat_k V_k - V_k Bhat_k      */
  TSYLV_K_ORTHO = 1,     /* Gram-Schmidt dots, updates, norms                  */
  TSYLV_K_XFORM = 2,     /* mode-3 DFT of A and inverse DFT of X               */
  TSYLV_K_APPLY_LOW = 3, /* FP32 / BF16 facewise apply (refinement inner)      */
  TSYLV_K_COUNT = 4
} tsylv_kernel_id;

typedef struct {
  int64_t launches; /* timed launches since tsylv_profile(ctx, 1)           */
  double total_ms;  /* summed event-to-event time of those launches         */
} tsylv_kstat;

/* enable != 0: reset the totals and start timing every family; 0: stop. */
int tsylv_profile(tsylv_ctx* ctx, int enable);

/* The same for the families whose bit (1 << tsylv_kernel_id) is set in
 * `mask` only (0: stop): timing a family puts two event records around each
 * of its launches on the stream, so a benchmark times the family it reports
 * and leaves the others untimed. */
int tsylv_profile_families(tsylv_ctx* ctx, unsigned mask);

/* Synchronises the context stream and returns the totals of one family. */
int tsylv_profile_read(tsylv_ctx* ctx, int kernel_id, tsylv_kstat* out);

/* Tile autotuner of the facewise apply (a project addition; the paper does
 * not tune).  The apply kernel has tsylv_apply_variants(prec) tile shapes,
 * all valid for every (n, s, p) and all computing the same products; by
 * default the shape follows s.  tsylv_autotune times every variant at
 * (n, s, p) in precision `prec` (`reps` >= 1 launches each, on operands of
 * that shape carved from the arena, filled with pseudo-random values: the
 * arena must hold them), keeps the fastest in the context's table -- the
 * default variant of the shape unless another is at least 2 % faster --
 * and every later apply of that exact shape
 * and precision on the context uses it (solves, refinement, serving).
 * `best` (may be NULL) receives the chosen variant; ms[v] for v < ms_cap
 * (ms may be NULL) the average launch time of variant v in milliseconds.
 * Synchronous on the context stream. */
int tsylv_apply_variants(int prec);
int tsylv_autotune(tsylv_ctx* ctx, int64_t n, int64_t s, int64_t p, int prec, int reps,
                   int* best, float* ms, int ms_cap);
/* Set (variant >= 0) or clear (variant = -1) the table entry of a shape. */
int tsylv_tune_set(tsylv_ctx* ctx, int prec, int64_t n, int64_t s, int64_t p, int variant);
/* The entry of a shape in *variant (-1: none, the default is used). */
int tsylv_tune_get(tsylv_ctx* ctx, int prec, int64_t n, int64_t s, int64_t p, int* variant);
/* The variant an apply of precision `prec` with n rows and s columns takes
 * when the table has no entry for its shape (>= 0), or TSYLV_EINVAL for an
 * unknown precision or n, s < 1. */
int tsylv_apply_default_variant(int prec, int64_t n, int64_t s);
/* Write the table to a text file (a header line "tsylv-tune 1", then one
 * line "prec n s p variant" per entry) / merge such a file into the table
 * (TSYLV_EINVAL, and nothing merged, when any line is malformed). */
int tsylv_tune_save(tsylv_ctx* ctx, const char* path);
int tsylv_tune_load(tsylv_ctx* ctx, const char* path);

/* Static string describing a status code. */
const char* tsylv_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* TSYLV_H */
