// Driver entry points used by the C ABI.
#pragma once

#include "runtime.hpp"

namespace tsylv {

size_t apply_workspace_bytes(int64_t n, int64_t s, int64_t p);
int apply_spatial(Ctx& ctx, int64_t n, int64_t s, int64_t p, const double* A, const double* B,
                  const double* X, double* Y, int prec);

size_t krylov_workspace_bytes(int64_t n, int64_t s, int64_t p, const tsylv_opts& o);
int krylov_solve(Ctx& ctx, int method, int64_t n, int64_t s, int64_t p, const double* A,
                 const double* B, const double* C, double* X, const tsylv_opts& o,
                 tsylv_info& info);

}  // namespace tsylv
