// Counter-based normal generator for synthetic instances made on the device.
//
// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
// as easy as 1, 2, 3", SC'11): ten rounds of two 64 x 64 -> 128-bit
// multiplications on a 256-bit counter under a 128-bit key bumped by Weyl
// constants between rounds.  The stream of a tensor (key = (seed, tensor
// id)): element (i, j, k) of a rows x cols x p tensor, e = i + rows j, takes
// the block at counter (e, floor(k/4), 0, 0); its words give uniforms
// u_r = ((w_r >> 12) + 1/2) 2^-52, exact and inside (0, 1), and Box-Muller
// on (u0, u1) gives k % 4 = 0, 1 (cos, sin), on (u2, u3) k % 4 = 2, 3.
// One thread therefore makes a whole tube (the p values of one e) with
// ceil(p/4) blocks, which is what the tube transform wants.
#pragma once

#include "kernels.hpp"

namespace tsylv {
namespace kern {

__device__ __forceinline__ void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

__device__ __forceinline__ double philox_uniform(uint64_t w) {
  return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

// Values k = 4 kb .. 4 kb + 3 of tube e of tensor g (the caller drops those
// at k >= p).  The rounding order is fixed: (r cos t) or (r sin t), times
// scale, then the shift -- contraction is off here, or the compiler could
// fuse the last product and the shift into one fma in one kernel and not in
// another, and the kernels that draw the same tensor would disagree.
__device__ __forceinline__ void gen_block4(const GenTensor& g, int64_t e, int64_t kb,
                                           double (&x)[4]) {
#pragma clang fp contract(off)
  uint64_t c[4] = {(uint64_t)e, (uint64_t)kb, 0ull, 0ull};
  philox4x64_10(c, g.seed, g.id);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double r = sqrt(-2.0 * log(philox_uniform(c[2 * h])));
    const double t = (2.0 * M_PI) * philox_uniform(c[2 * h + 1]);
    double sn, cs;
    sincos(t, &sn, &cs);
    x[2 * h] = g.scale * (r * cs);
    x[2 * h + 1] = g.scale * (r * sn);
  }
  if (kb == 0 && (e % g.rows) == (e / g.rows)) x[0] = x[0] + g.shift;
}

}  // namespace kern
}  // namespace tsylv
