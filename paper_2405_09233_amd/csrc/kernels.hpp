// Host-side launchers of the HIP kernels (all enqueue on `st`, never sync).
#pragma once

#include "common.hpp"

namespace tsylv {
namespace kern {

// ---- tube transforms (mode-3 DFT as a p x p real matrix on every tube) ----

// M[q*p + j]: the p x p matrix of XformKind `kind` (built on the device from
// (j*k) mod p so the multiples of pi/2 are exact).
void build_xform(double* M, int p, int kind, hipStream_t st);

// out[q*E + e] = scale * sum_j M[q*p + j] * in[j*E + e]  for 0 <= e < E.
void tube_xform_f64(const double* in, double* out, const double* M, int64_t E,
                    int p, hipStream_t st);

// Synthetic instances from the counter-based stream of philox.hpp (tensor
// `g`, frontal slices of E = rows x cols elements).  gen_tensor_f64 writes
// the spatial tensor; tube_xform_gen_f64 writes what tube_xform_f64 would
// make of it, bit for bit, without storing it (p <= kGenXformMaxP).
constexpr int kGenXformMaxP = 64;
struct GenTensor {
  uint64_t seed;
  uint64_t id;    // 0: A, 1: B, 2: C
  int64_t rows;   // column-major rows x cols frontal slices
  double scale;   // value = scale * z, rounded ...
  double shift;   // ... then + shift on the diagonal of frontal slice 1
};
void gen_tensor_f64(const GenTensor& g, double* out, int64_t E, int p, hipStream_t st);
void tube_xform_gen_f64(const GenTensor& g, double* out, const double* M, int64_t E, int p,
                        hipStream_t st);

// `count` pseudo-random values uniform in [-1, 1) (splitmix64 of seed + i),
// stored with `elem` bytes each (8: FP64, 4: FP32, 2: BF16); timing operands.
void fill_random(void* buf, int64_t count, int elem, uint64_t seed, hipStream_t st);

// Down-conversion of `count` doubles (round to nearest even).
void convert_f64_f32(const double* in, float* out, int64_t count, hipStream_t st);
void convert_f64_bf16(const double* in, uint16_t* out, int64_t count, hipStream_t st);
void convert_f32_f64(const float* in, double* out, int64_t count, hipStream_t st);

// ---- facewise operator apply (Fourier planes) ----
//   out_k = alpha * (Ahat_k V_k - V_k Bhat_k) + beta * Y_k   for every slice k
// (the V_k Bhat_k term is skipped when Bh == nullptr; Y may be nullptr when
// beta == 0).  Ah: p planes n x n; Bh: p planes s x s; V, Y, out: p planes n x s.
// `variant` picks the tile shape (0 .. apply_variant_count(prec) - 1; -1:
// the default for s); every variant computes the same products.
void apply_f64(const double* Ah, const double* Bh, const double* V, double* out,
               const double* Y, double alpha, double beta, int64_t n, int64_t s,
               int p, hipStream_t st, int variant = -1);
// Same in FP32 (FP32 MFMA).
void apply_f32(const float* Ah, const float* Bh, const float* V, float* out, const float* Y,
               double alpha, double beta, int64_t n, int64_t s, int p, hipStream_t st,
               int variant = -1);
int apply_variant_count(int prec);             // tsylv_prec
int apply_default_variant(int prec, int64_t n, int64_t s);
int bf16_default_variant(int64_t s);

// BF16 operator planes (BF16 MFMA, the vectors rounded to BF16 on the way
// into the product, FP32 accumulation).  `At` holds the operator in the tiled
// MFMA lane order written by tile_operator_bf16 (bf16_tiled_elems elements);
// `Bb` the plain BF16 planes of Bhat (s x s column-major) or null.  `Vt` is
// scratch of bf16_vtiled_elems elements that receives V in the same order.
int64_t bf16_tiled_elems(int64_t n, int p);
int64_t bf16_vtiled_elems(int64_t n, int64_t s, int p);
void tile_operator_bf16(const double* Ah, uint16_t* At, int64_t n, int p, hipStream_t st);
void apply_bf16(const uint16_t* At, const uint16_t* Bb, const float* V, uint16_t* Vt,
                float* out, const float* Y, double alpha, double beta, int64_t n, int64_t s,
                int p, hipStream_t st, int variant = -1);

// ---- BF16 Krylov vectors (the inner basis of the BF16-refined solves) ----
// A vector of p Fourier planes n x s stored as BF16 bits in the tiled order
// of the BF16 apply's V operand: plane q, 16-column block cb, 32-row block kb
// form one 512-element chunk whose lane i + 16 g holds rows 32 kb + 8 g ..
// + 7 of column 16 cb + i.  bf16_vtiled_elems(n, s, p) elements; the padding
// (rows >= n, columns >= s) is zero, and every kernel below keeps it zero.
struct bf16t {
  uint16_t bits;
};
// Xt = tiled(a X) (X: p planes n x s, FP64), padding written as zero.
void tile_scale_bf16(const double* X, bf16t* Xt, double a, int64_t n, int64_t s, int p,
                     hipStream_t st);
// X -= sum_i y[i] untiled(V_i) (y on the device, nv entries, FP64 sums; the
// sign of mupdate).
void untile_update_bf16(const bf16t* V, int64_t ldv, int nv, const double* y, double* X,
                        int64_t n, int64_t s, int p, hipStream_t st);
// out = alpha (Ahat_k V_k - V_k Bhat_k) for every slice, V and out tiled
// (out's padding written as zero; out must not alias V).
void apply_bf16_tiled(const uint16_t* At, const uint16_t* Bb, const bf16t* V, bf16t* out,
                      double alpha, int64_t n, int64_t s, int p, hipStream_t st,
                      int variant = -1);

// ---- t-Bartels-Stewart direct solve on the Fourier slices ----
// Xhat_k from Ahat_k Xhat_k - Xhat_k Bhat_k = Chat_k for every slice of the
// half spectrum (Ah, Bh: operator planes; Zc, Zx: vector planes), n, s <=
// tbs_max_size().  `scratch` holds 2 tbs_scratch_complex(n, s, p) doubles;
// *info (device int, zero on entry) is raised to 1 if a Schur iteration did
// not converge and to 2 if a slice's triangular equation is singular.
// Arguments of one instance of the direct solve (device pointers).
struct TbsArgs {
  const double* Ah;  // operator planes (p planes n x n)
  const double* Bh;  // p planes s x s
  const double* Zc;  // right-hand side planes (p planes n x s)
  double* Zx;        // solution planes
  double2* scr;      // per slice: S (s x s), V (s x s), G (n x s), F (n x s)
  int* info;         // raised to 1 (Schur did not converge) or 2 (singular)
  int n, s, p;
};
// Many instances at once: d_args[count] (device), d_first[count + 1] the
// prefix sums of the instances' slice counts (total_slices = d_first[count]);
// one wavefront per (instance, slice) solves, then the FP64 residual in the
// Fourier planes: d_norms[2 i] = ||C - M(X)||^2, d_norms[2 i + 1] = ||C||^2
// of instance i (d_part: 2 total_slices doubles).
void tbs_batch(const TbsArgs* d_args, const int* d_first, int count, int total_slices,
               double* d_part, double* d_norms, hipStream_t st);
// Tube transforms of many tensors in one launch (descriptor d: out[q E + e]
// = sum_j M[q p + j] in[j E + e]); d_bfirst[d] the first of its
// ceil(E / kBatchXformBlock) blocks, total_blocks = d_bfirst[ndesc].  The
// fma order is that of tube_xform_f64, so both give the same bits.
constexpr int kBatchXformBlock = 256;
struct XformDesc {
  const double* in;
  double* out;
  const double* M;
  int64_t E;
  int p;
};
void batch_xform(const XformDesc* d_descs, const int* d_bfirst, int ndesc, int total_blocks,
                 hipStream_t st);
int tbs_max_size();
int64_t tbs_scratch_complex(int64_t n, int64_t s, int p);
void tbs_solve(const double* Ah, const double* Bh, const double* Zc, double* Zx, int64_t n,
               int64_t s, int p, double* scratch, int* info, hipStream_t st);

// ---- multi-vector kernels on flat vectors of N reals ----

// Number of per-block partial rows used by mdot for length N.
int mdot_chunks(int64_t N);

// part[c*ldp + i] = sum_{e in chunk c} V_i[e] * w[e]  (i < nv, V_i = V + i*ldv)
// and, if with_ww, part[c*ldp + nv] = sum w[e]^2.  ldp >= nv + with_ww.
// FP32 vectors are summed in FP64.
void mdot_partial(const double* V, int64_t ldv, int nv, const double* w, int64_t N,
                  double* part, int ldp, int with_ww, hipStream_t st);
void mdot_partial(const float* V, int64_t ldv, int nv, const float* w, int64_t N,
                  double* part, int ldp, int with_ww, hipStream_t st);

// out[i] = sum_c part[c*ldp + i] for i < ncols, in a fixed order.
void reduce_partials(const double* part, int nchunks, int ldp, int ncols,
                     double* out, hipStream_t st);

// w[e] -= sum_i h[i] * V_i[e]   (h on the device, nv entries; FP64 arithmetic)
void mupdate(const double* V, int64_t ldv, int nv, const double* h, double* w,
             int64_t N, hipStream_t st);
void mupdate(const float* V, int64_t ldv, int nv, const double* h, float* w,
             int64_t N, hipStream_t st);
void mupdate(const float* V, int64_t ldv, int nv, const double* h, double* w,
             int64_t N, hipStream_t st);

// Fused CGS2 passes over a basis whose vectors V_i are stored unnormalised
// with sigma[i] = 1 / ||V_i|| (device array).  ortho_chunks(N) partial rows.
// BF16 vectors are widened on load and the results rounded to nearest even
// on store; every sum runs in FP64.
//   ortho_dots:   part[c][i] = sigma_i V_i . w (i < nv), part[c][nv] = ||w||^2
//   ortho_update: w -= sum_i h[i] sigma[i] V_i; then mode 0: part[c][i] =
//                 sigma_i V_i . w (the next pass), mode 1: part[c][0] = ||w||^2
// nv <= ortho_max_vectors(fp32).
int ortho_chunks(int64_t N);
int ortho_max_vectors(bool fp32);
void ortho_dots(const double* V, int64_t ldv, int nv, const double* sigma, const double* w,
                int64_t N, double* part, int ldp, hipStream_t st);
void ortho_dots(const float* V, int64_t ldv, int nv, const double* sigma, const float* w,
                int64_t N, double* part, int ldp, hipStream_t st);
void ortho_update(const double* V, int64_t ldv, int nv, const double* h, const double* sigma,
                  double* w, int64_t N, double* part, int ldp, int mode, hipStream_t st);
void ortho_update(const float* V, int64_t ldv, int nv, const double* h, const double* sigma,
                  float* w, int64_t N, double* part, int ldp, int mode, hipStream_t st);
void ortho_dots(const bf16t* V, int64_t ldv, int nv, const double* sigma, const bf16t* w,
                int64_t N, double* part, int ldp, hipStream_t st);
void ortho_update(const bf16t* V, int64_t ldv, int nv, const double* h, const double* sigma,
                  bf16t* w, int64_t N, double* part, int ldp, int mode, hipStream_t st);

// Delayed reorthogonalisation sweeps (V: nv basis vectors, sigma as above):
//   ortho_dots2:   part[c] = [sigma_i V_i . u, sigma_i V_i . w, u . w, u . u,
//                  w . w] (2 nv + 3 values, ldp >= 2 nv + 3);
//   ortho_update2: coef = [ac (nv), bc (nv), alpha, gamma]; u <- u - sum ac_i
//                  V_i (if u is not null), then w <- alpha w + sum bc_i V_i +
//                  gamma u.
void ortho_dots2(const double* V, int64_t ldv, int nv, const double* sigma, const double* u,
                 const double* w, int64_t N, double* part, int ldp, hipStream_t st);
void ortho_dots2(const float* V, int64_t ldv, int nv, const double* sigma, const float* u,
                 const float* w, int64_t N, double* part, int ldp, hipStream_t st);
void ortho_update2(const double* V, int64_t ldv, int nv, const double* coef, double* u, double* w,
                   int64_t N, hipStream_t st);
void ortho_update2(const float* V, int64_t ldv, int nv, const double* coef, float* u, float* w,
                   int64_t N, hipStream_t st);
void ortho_dots2(const bf16t* V, int64_t ldv, int nv, const double* sigma, const bf16t* u,
                 const bf16t* w, int64_t N, double* part, int ldp, hipStream_t st);
void ortho_update2(const bf16t* V, int64_t ldv, int nv, const double* coef, bf16t* u, bf16t* w,
                   int64_t N, hipStream_t st);

// One round of the delayed CGS2 process on the device (the arithmetic of the
// Krylov driver's host step, for a cycle enqueued at once): consumes the
// round's reduced sums `res`, finalises Hessenberg column j - 1 in H
// (leading dimension ldh), and unless final_round writes sigma[j], the next
// update coefficients `coef` and first projection `h1p`; scal = [||M
// q_{j-1}||^2, round of a breakdown or -1].  0 <= j <= 63.
void dcgs2_round(const double* res, int j, bool final_round, int ldh, double* H, double* h1p,
                 double* sigma, double* coef, double* scal, hipStream_t st);

// out[e] = a * x[e]  (the FP64 -> FP32 form rounds the scaled value)
void scale(const double* x, double* out, double a, int64_t N, hipStream_t st);
void scale(const float* x, float* out, double a, int64_t N, hipStream_t st);
void scale(const double* x, float* out, double a, int64_t N, hipStream_t st);

// ---- batched planar-complex FP64 GEMM over the Fourier slices ----

// Element (r, c) of slice k of a planar matrix sits at
//   base + q * plane + r + (c % cb) * ld + (c / cb) * bs
// where q is the Re (or Im) plane of slice k in the half-spectrum layout.
struct PMat {
  const double* base;
  int64_t plane, ld, cb, bs;
};

inline PMat dense_pmat(const double* base, int64_t plane, int64_t ld) {
  return PMat{base, plane, ld, (int64_t)1 << 40, 0};
}

// Projected equations of TBAS(m) on the device (kernels_projected.hip):
// solves (Hm_k - lam_{k,j} I) z = d for the nsys = p_h s systems k s + j.
// Hm: p_h interleaved-complex ms x ms column-major slices, lower bandwidth s
// (block upper Hessenberg); lam: nsys shifts; D: p_h interleaved s x s
// slices, column j = the first s rows of system (k, j)'s right-hand side
// (the rest is zero); z: nsys x ms, receives the solutions; Wrk (2 nsys s ms)
// and U (nsys proj_u_stride(s, m)) complex scratch, G (proj_g_doubles(s,
// nsys) doubles) scratch for each panel's L^{-1} and row permutation; info:
// nsys flags, 1 where a pivot vanished.  Requires 1 <= s <= proj_max_block(),
// ms = m s.
int proj_max_block();
int64_t proj_u_stride(int s, int m);
int64_t proj_g_doubles(int s, int nsys);
void proj_solve(const double* Hm, const double* lam, const double* D, double* z, double* Wrk,
                double* U, double* G, int* info, int ms, int s, int m, int nsys,
                hipStream_t st);

// Device small linear algebra of a TBAS cycle (kernels_tba.hip).  Planar
// matrices use the half-spectrum plane layout (p planes, s x s or J x s,
// column-major); Hm, Hlast, D, W, Winv and z are interleaved complex.
//  cholqr_pass: one shifted-Cholesky-QR pass per slice: Rinv = R^{-1},
//    Racc = R Racc (first pass: Racc = R, and the diagonal of G shifted by
//    shift_factor trace(G)); *flag |= 1 on a pivot <= rel_tol max diag.
//  tube_test: *flag |= 1 when a diagonal tube of Racc is not invertible.
//  hm_column: block column j of Hm from G1 + G2 and the QR factor Rq (to
//    Hlast for the last column).
//  proj_rhs: D_k = H0_k W_k.  proj_y: Y_k = Z_k Winv_k (planar) and
//    est[k] = ||Hlast_k Y_k(last block row)||^2.  proj_check: *flag |= 1 on
//    a zero pivot or a non-finite solution.
int cholqr_max_block();
void cholqr_pass(const double* G, double* Rinv, double* Racc, int s, int p, double shift_factor,
                 bool first, double rel_tol, int* flag, hipStream_t st);
void tube_test(const double* Racc, int s, int p, bool scaled, int* flag, hipStream_t st);
void hm_column(const double* G1, const double* G2, const double* Rq, double* Hm, double* Hlast,
               int j, int s, int m, int p, hipStream_t st);
void proj_rhs(const double* H0, const double* W, double* D, int s, int p, hipStream_t st);
void proj_y(const double* z, const double* Winv, const double* Hlast, double* Y, double* est,
            int s, int m, int p, hipStream_t st);
void proj_check(const int* info, const double* z, int64_t nsys, int64_t nz, int* flag,
                hipStream_t st);

// Number of K splits zgemm uses when given a partial buffer, and the size of
// that buffer in doubles.
int zgemm_splits(int64_t M, int64_t N, int64_t K, int p);
int64_t zgemm_partial_elems(int64_t M, int64_t N, int64_t K, int p);

// C_k = alpha op(A_k) B_k + beta C_k for every slice k, op(A) = A (M x K) or
// A^H (A stored K x M) when conjA.  C is dense: plane stride planeC, leading
// dimension ldC, and must not overlap A or B.  With `partial` non-null the
// contraction is split over K (partial: zgemm_partial_elems doubles).
void zgemm(const PMat& A, bool conjA, const PMat& B, double* C, int64_t planeC, int64_t ldC,
           int64_t M, int64_t N, int64_t K, double alpha, double beta, int p, double* partial,
           hipStream_t st);


// ---- small instances: a whole restarted solve in one workgroup ----------
// (kernels_tiny.hip)  tiny_krylov_fits: n s p, the operator planes, the
// iterate and two basis vectors fit the workgroup's LDS (n s p <= 8192,
// m <= 1024, m n s p <= 2^18).  tiny_krylov: restarted tGMRES(m) (fom = false) or tFOM(m) on
// the Fourier planes Ah, Bh (p planes), Zc (C, orthonormal planes), with X
// in Zx (X0 on entry when x0_given); basis: (m + 1) n s p doubles, Rg: m m
// doubles, hist: hist_cap estimates (may be null); out receives the record
// [status, steps, cycles, relres_true, relres_est, fom_fallback, hist_len].
bool tiny_krylov_fits(int64_t n, int64_t s, int64_t p, int m);
constexpr int kTinyRecord = 8;
void tiny_krylov(const double* Ah, const double* Bh, const double* Zc, double* Zx, double* basis,
                 double* Rg, double* hist, int hist_cap, double* out, int n, int s, int p, int m,
                 int max_cycles, bool fom, bool x0_given, double tol, hipStream_t st);
// Many such solves in one launch, one workgroup per job (each job's fields
// as the arguments of tiny_krylov; lslots from tiny_krylov_slots for the
// launch's LDS size).  tiny_krylov_lds: the LDS bytes that hold every basis
// slot of a shape (at most the workgroup's LDS); a batch launches with the
// largest of its jobs'.
struct TinyJob {
  const double* Ah;
  const double* Bh;
  const double* Zc;
  double* Zx;
  double* Vg;
  double* Rg;
  double* hist;
  double* out;
  double tol;
  int n, s, p, m, max_cycles, fom, x0_given, hist_cap, lslots;
};
size_t tiny_krylov_lds(int64_t n, int64_t s, int64_t p, int m);
int tiny_krylov_slots(int64_t n, int64_t s, int64_t p, int m, size_t lds);
void tiny_krylov_batch(const TinyJob* jobs, int count, size_t lds, hipStream_t st);

// ---- batched lockstep tGMRES (many independent instances per launch) ----
//
// Every launch serves all instances of a batch: blockIdx.x runs over the
// concatenated work of the instances (apply tiles, or vector chunks of
// kBatchChunk elements), each block finds its instance by binary search over
// the instances' first work index, and the step index j is read from device
// memory, so one captured step replays for every j.  An instance's
// arithmetic (its chunks, tiles and fixed-order reductions) does not depend
// on the other instances.

constexpr int64_t kBatchChunk = 8192;  // elements per vector work item
constexpr int kBatchMaxM = 63;         // restart length limit (H columns)

struct BatchItem {
  const double* Ah;
  const double* Bh;
  double* V;          // basis: m + 1 vectors at stride ldv
  double* W;          // work vector of the step
  const double* Zc;   // orthonormal planes of C
  double* Zx;         // orthonormal planes of X (the iterate)
  double* H;          // (m + 1) x m, column-major, Givens-rotated in place
  double* cs;         // rotations (m)
  double* sn;
  double* g;          // rotated right-hand side (m + 1)
  double* y;          // least-squares solution of the cycle (m)
  double* coef;       // CGS coefficients of the current pass (m + 1)
  int64_t n, s, N, ldv;
  int p;
  int chunk0, nchunks;  // vector work items
};

struct BatchState {
  int active;   // stepping in the current cycle
  int done;     // converged or out of cycles: no more work
  int jdone;    // steps taken in the current cycle
  int status;   // tsylv_status once done
  int steps, cycles;
  int reorth;    // the current step takes the second Gram-Schmidt pass
  int pad0;
  double beta;   // ||R|| at the start of the cycle
  double cnorm;  // ||C||
  double hn;     // ||W|| after the Gram-Schmidt passes of the step
  double est;    // residual estimate |g_{j+1}|
  double mv2;    // ||M(V_j)||^2 of the current step
  double pad1;
};

// Apply tiles of one tile variant over a subset of the batch, in order of
// their first tile.
struct BatchApplyRef {
  int item, tile0, nrt, nct;
};

enum BatchMode {
  BM_STEP = 0,      // apply: W = M(V_j); dots: V_0..V_j . W and W . W; update: W -= V c
  BM_WNORM = 1,     // dots: W . W (reorth steps); reduce: ||W||, Givens, stop test
  BM_RESID = 2,     // apply: V_0 = Zc - M(Zx); dots: V_0 . V_0; reduce: restart
  BM_CNORM = 3,     // dots: Zc . Zc; reduce: ||C||
  BM_PASS2 = 4,     // dots / reduce / update of the second pass (reorth steps only)
  BM_XUPDATE = 5,   // update: Zx += V y
  BM_RESID0 = 6,    // reduce: restart test on the initial residual (no cycle counted)
};

int batch_apply_variant(int64_t s);
// Tiles of one instance under a batch tile variant (row and column tiles out).
int batch_apply_tiles(int variant, int64_t n, int64_t s, int p, int* nrt, int* nct);
void batch_apply(const BatchItem* items, const BatchApplyRef* refs, int nref, int total_tiles,
                 int variant, BatchState* st, const int* jp, int mode, hipStream_t st_);
void batch_dots(const BatchItem* items, int count, int total_chunks, const BatchState* st,
                const int* jp, double* part, int ldp, int mode, hipStream_t s);
void batch_reduce(const BatchItem* items, int count, BatchState* st, const int* jp,
                  const double* part, int ldp, int mode, int m, double tol, int max_cycles,
                  hipStream_t s);
void batch_update(const BatchItem* items, int count, int total_chunks, const BatchState* st,
                  const int* jp, int mode, hipStream_t s);
void batch_scale(const BatchItem* items, int count, int total_chunks, const BatchState* st,
                 const int* jp, int mode, hipStream_t s);
void batch_backsub(const BatchItem* items, int count, const BatchState* st, int m,
                   hipStream_t s);
void batch_set_j(int* jp, int value, hipStream_t s);
void batch_advance(int* jp, hipStream_t s);

}  // namespace kern
}  // namespace tsylv
