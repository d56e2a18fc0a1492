// Test driver: reads a command and complex matrices (re im pairs, column-major)
// from stdin, runs one host_linalg routine, writes the result to stdout.
#include <cstdio>
#include <iostream>
#include <vector>

#include "host_linalg.hpp"

using tsylv::host::cplx;

static std::vector<cplx> read_mat(size_t count) {
  std::vector<cplx> m(count);
  for (auto& v : m) {
    double re, im;
    std::cin >> re >> im;
    v = cplx(re, im);
  }
  return m;
}

static void write_mat(const std::vector<cplx>& m) {
  for (auto& v : m) std::printf("%.17g %.17g\n", v.real(), v.imag());
}

int main() {
  std::string cmd;
  std::cin >> cmd;
  if (cmd == "chol") {
    int s;
    std::cin >> s;
    auto G = read_mat((size_t)s * s);
    bool ok = tsylv::host::cholesky_upper(G.data(), s, 1e-14);
    std::printf("%d\n", ok ? 1 : 0);
    write_mat(G);
  } else if (cmd == "triinv") {
    int s;
    std::cin >> s;
    auto R = read_mat((size_t)s * s);
    std::vector<cplx> Ri((size_t)s * s);
    tsylv::host::tri_inv_upper(R.data(), Ri.data(), s);
    write_mat(Ri);
  } else if (cmd == "schur") {
    int n;
    std::cin >> n;
    auto A = read_mat((size_t)n * n);
    std::vector<cplx> U((size_t)n * n);
    bool ok = tsylv::host::schur(A.data(), U.data(), n);
    std::printf("%d\n", ok ? 1 : 0);
    write_mat(A);
    write_mat(U);
  } else if (cmd == "sylv") {
    int ms, band, s;
    std::cin >> ms >> band >> s;
    auto H = read_mat((size_t)ms * ms);
    auto B = read_mat((size_t)s * s);
    auto C = read_mat((size_t)ms * s);
    std::vector<cplx> Y((size_t)ms * s);
    bool ok = tsylv::host::sylvester_banded(H.data(), ms, band, B.data(), s, C.data(), Y.data());
    std::printf("%d\n", ok ? 1 : 0);
    write_mat(Y);
  } else if (cmd == "eig") {
    int n;
    std::cin >> n;
    auto A = read_mat((size_t)n * n);
    std::vector<cplx> U((size_t)n * n), lam(n), W((size_t)n * n), Wi((size_t)n * n);
    bool ok = tsylv::host::schur(A.data(), U.data(), n);
    double kappa = ok ? tsylv::host::eig_from_schur(A.data(), U.data(), n, lam.data(), W.data(),
                                                   Wi.data())
                      : -1.0;
    std::printf("%d %.17g\n", ok ? 1 : 0, kappa);
    write_mat(lam);
    write_mat(W);
    write_mat(Wi);
  }
  return 0;
}
