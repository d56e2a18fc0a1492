// Driver entry points used by the C ABI.
#pragma once

#include "runtime.hpp"

namespace tsylv {

// Fourier-domain state shared by the solvers: unscaled DFT planes of A and B,
// orthonormal planes of C and X, and the three p x p tube transforms.
struct Setup {
  double *Ah, *Bh, *xf_op, *xf_fwd, *xf_inv, *Zc, *Zx;
};
size_t setup_bytes(int64_t n, int64_t s, int64_t p);
Setup setup_fourier(Ctx& ctx, hipStream_t st, bool profile, Workspace& ws, int64_t n, int64_t s,
                    int64_t p, const double* A, const double* B, const double* C, const double* X,
                    bool x0_given);

size_t tba_workspace_bytes(int64_t n, int64_t s, int64_t p, int m);
int tba_solve(Ctx& ctx, int64_t n, int64_t s, int64_t p, const double* A, const double* B,
              const double* C, double* X, const tsylv_opts& o, tsylv_info& info);

size_t apply_workspace_bytes(int64_t n, int64_t s, int64_t p);
int apply_spatial(Ctx& ctx, int64_t n, int64_t s, int64_t p, const double* A, const double* B,
                  const double* X, double* Y, int prec);

size_t krylov_workspace_bytes(int method, int64_t n, int64_t s, int64_t p, const tsylv_opts& o);
int krylov_solve(Ctx& ctx, int method, int64_t n, int64_t s, int64_t p, const double* A,
                 const double* B, const double* C, double* X, const tsylv_opts& o,
                 tsylv_info& info);

}  // namespace tsylv
