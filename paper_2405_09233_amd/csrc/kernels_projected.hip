// Device solve of the TBAS(m) projected equations (eq. (TBslowrank)),
//   Hm_k Y_k - Y_k Bhat_k = [H0_k; 0]        for every Fourier slice k,
// after diagonalising Bhat_k = W_k diag(lam_k) W_k^{-1} on the host: with
// Z = Y W the columns decouple into the shifted systems
//   (Hm_k - lam_{k,j} I) z_{k,j} = d_{k,j},   d = [H0_k W_k; 0] e_j,
// one per (slice, eigenvalue) -- p_h s independent solves instead of s
// dependent ones per slice (Bartels-Stewart's triangular recursion).
//
// Hm_k (ms x ms, ms = m s) is block upper Hessenberg with s x s blocks
// (lower bandwidth s).  Each system is solved by block LU with s x s blocks:
// panel b is the 2s x s block column [row block b as updated so far; row
// block b + 1 as built], factorised with partial pivoting inside the panel
// (band-limited pivoting, as in banded LU) and applied on the fly to the
// right-hand side.  With the panel's row permutation T of the two block
// rows and G = L^{-1} [I_s; 0] = [L11^{-1}; -L21 L11^{-1}], the trailing
// columns become [U12; next row block] = G T_top + [0; T_bot]: one dense
// 2s x s by s x (trailing columns) product per panel, on the FP64 matrix
// cores.  The finished row blocks of U are kept for the back substitution.
// Per panel two launches: the factorisation (one workgroup per system, the
// panel in registers) and the trailing product (many workgroups per
// system).
#include <type_traits>

#include "kernels.hpp"

namespace tsylv {
namespace kern {

namespace {

constexpr int kPB = 256;     // threads per workgroup
constexpr int kPMax = 64;    // largest block size s handled here

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a - l p in four fused multiply-adds
__device__ __forceinline__ double2 cmsub(double2 a, double2 l, double2 p) {
  return make_double2(fma(-l.x, p.x, fma(l.y, p.y, a.x)), fma(-l.x, p.y, fma(-l.y, p.x, a.y)));
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
// 1 / a by the hardware reciprocal and two Newton steps (within about an
// ulp; a is a pivot, never zero, infinite or subnormal when it is used)
__device__ __forceinline__ double rcp_nr(double a) {
  double y = __builtin_amdgcn_rcp(a);
  double e = fma(-a, y, 1.0);
  y = fma(y, e, y);
  e = fma(-a, y, 1.0);
  return fma(y, e, y);
}
// 1 / b with Smith's scaling, by rcp_nr
__device__ __forceinline__ double2 crecip_fast(double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y * rcp_nr(b.x), inv = rcp_nr(b.x + b.y * r);
    return make_double2(inv, -r * inv);
  }
  const double r = b.x * rcp_nr(b.y), inv = rcp_nr(b.y + b.x * r);
  return make_double2(r * inv, -inv);
}

// Largest key over each 16-lane row of the wave (every lane of a row ends
// with it): max with the lanes at xor 1 and xor 2 inside each quad, then
// with the mirrored lane inside each half row and inside the row.
__device__ __forceinline__ unsigned max_dpp(unsigned k) {
  unsigned o;
  o = (unsigned)__builtin_amdgcn_update_dpp((int)k, (int)k, 0xB1, 0xF, 0xF, false);  // quad [1,0,3,2]
  k = o > k ? o : k;
  o = (unsigned)__builtin_amdgcn_update_dpp((int)k, (int)k, 0x4E, 0xF, 0xF, false);  // quad [2,3,0,1]
  k = o > k ? o : k;
  o = (unsigned)__builtin_amdgcn_update_dpp((int)k, (int)k, 0x141, 0xF, 0xF, false);  // half mirror
  k = o > k ? o : k;
  o = (unsigned)__builtin_amdgcn_update_dpp((int)k, (int)k, 0x140, 0xF, 0xF, false);  // row mirror
  return o > k ? o : k;
}
// x of lane `lane` (a wave-uniform index)
__device__ __forceinline__ double2 read_lane(double2 x, int lane) {
  const int l = __builtin_amdgcn_readfirstlane(lane);
  return make_double2(
      __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x.x), l),
                       __builtin_amdgcn_readlane(__double2loint(x.x), l)),
      __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x.y), l),
                       __builtin_amdgcn_readlane(__double2loint(x.y), l)));
}


struct ProjArgs {
  const double2* Hm;  // p_h slices of ms x ms, column-major
  const double2* lam; // nsys shifts, system k s + j
  const double2* D;   // p_h slices of s x s: first s rows of the right-hand sides
  double2* z;         // nsys x ms: right-hand side, then solution
  double2* Wrk;       // 2 x nsys x (s x ms): the current row block, ping-pong by panel
  double2* U;         // nsys x ustride: finished row blocks of U
  int* info;          // nsys flags (1: zero pivot)
  double* G;          // nsys x g_sys_doubles(s): G and the permutation of a panel
  int ms, s, m, nsys;
  int64_t ustride;
};

// Row block b of system sys as updated by the panels before it (panel b
// reads buffer b % 2, its trailing update writes buffer (b + 1) % 2).
__device__ __forceinline__ double2* wrk(const ProjArgs& a, int b, int sys) {
  return a.Wrk + ((int64_t)(b & 1) * a.nsys + sys) * a.s * a.ms;
}

__device__ __forceinline__ int64_t uoff(const ProjArgs& a, int b) {
  return (int64_t)a.s * a.s * ((int64_t)b * a.m - (int64_t)b * (b - 1) / 2);
}

__global__ void proj_init_kernel(ProjArgs a) {
  const int64_t nw = (int64_t)a.nsys * a.s * a.ms;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nw;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sys = e / ((int64_t)a.s * a.ms);
    const int64_t rem = e % ((int64_t)a.s * a.ms);
    const int r = (int)(rem % a.s), c = (int)(rem / a.s);
    const int k = (int)(sys / a.s);
    double2 v = a.Hm[(int64_t)k * a.ms * a.ms + r + (int64_t)a.ms * c];
    if (r == c) v = csub(v, a.lam[sys]);
    a.Wrk[e] = v;
  }
  const int64_t nz = (int64_t)a.nsys * a.ms;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sys = e / a.ms;
    const int i = (int)(e % a.ms);
    const int k = (int)(sys / a.s), j = (int)(sys % a.s);
    a.z[e] = i < a.s ? a.D[(int64_t)k * a.s * a.s + i + (int64_t)a.s * j] : make_double2(0.0, 0.0);
    if (i == 0) a.info[sys] = 0;
  }
}

// Row permutation and G = L^{-1} [I_s; 0] of panel b, per system: G's
// top s rows are L11^{-1}, its bottom s rows -L21 L11^{-1}, stored in the
// operand order of v_mfma_f64_16x16x4 (element (i, k) of row block i / 16
// and k-step k / 4 in lane i % 16 + 16 (k % 4)); rows and columns padded to
// sp = s rounded up to 16 (top rows 0 .. sp-1, bottom rows sp .. 2 sp - 1),
// Re plane then Im plane, then 2 kPMax ints of the permutation.
__host__ __device__ inline int pad16(int s) { return (s + 15) & ~15; }
__host__ __device__ inline int64_t g_sys_doubles(int s) {
  return 4 * (int64_t)pad16(s) * pad16(s) + kPMax;
}

__device__ __forceinline__ int xcd_tile(int b, int total) {
  const int q = total / 8, r = total % 8;
  const int x = b % 8;
  return x * q + (x < r ? x : r) + b / 8;
}

// The panel kernel's thread grid: thread (tr, tc) holds rows tr + kTR i
// (i < kRI) and columns tc + kTC j (j < kCJ) of the 2s x s panel in
// registers; consecutive threads hold consecutive rows (coalesced loads).
constexpr int kLB = 512;
constexpr int kTR = 32, kTC = kLB / kTR;
constexpr int kRI = 2 * kPMax / kTR, kCJ = kPMax / kTC;

// Runs body(std::integral_constant<int, J>) for J = 0 .. kCJ - 1 in order:
// loops over the columns of slot J (columns kTC J .. kTC J + kTC - 1 of the
// thread grid) see J at compile time, so register arrays are only ever
// indexed at compile time and no branch merges them.
template <typename F>
__device__ __forceinline__ void for_each_slot(F&& body) {
  static_assert(kCJ == 4, "one call per column slot");
  body(std::integral_constant<int, 0>{});
  body(std::integral_constant<int, 1>{});
  body(std::integral_constant<int, 2>{});
  body(std::integral_constant<int, 3>{});
}

// Runs body(std::integral_constant<int, c / kTC>) for the column slot of
// c, so that register arrays are only ever indexed at compile time.
template <typename F>
__device__ __forceinline__ void with_slot(int c, F&& body) {
  static_assert(kCJ == 4, "one case per column slot");
  switch (c / kTC) {
    case 0: body(std::integral_constant<int, 0>{}); break;
    case 1: body(std::integral_constant<int, 1>{}); break;
    case 2: body(std::integral_constant<int, 2>{}); break;
    default: body(std::integral_constant<int, 3>{}); break;
  }
}

// Panel b of every system, one workgroup each, the panel in registers:
// LU with partial pivoting inside the panel (band-limited pivoting, as in
// banded LU), applied on the fly to the right-hand side; the finished U
// block; then, for the trailing update, the row order and
// G = L^{-1} [I_s; 0] by forward substitution, formed in place: column l of
// L is broadcast at step l and never read again, so its registers take
// column l of G.
//
// Rows are never moved: each row records the step at which it became the
// pivot (its position in the factorisation's row order), the last s
// unpivoted rows taking positions s .. 2s-1 in row order.  The multipliers
// of pivoted rows are zero and the pivot row is broadcast with its columns
// up to c zeroed, so every thread updates all its entries with no
// conditions.  Two barriers per LU column, one per substitution step; only
// the pivot row and the multipliers pass through LDS.
constexpr int kUnpivoted = 1 << 20;  // position of a row not yet pivoted
constexpr int kOutside = 1 << 21;    // position of a thread slot past the panel's rows

// (registers capped for two workgroups per CU: 128 with 11 spilled outside
// the column loop, 0.43 against 0.60 ms per launch at one workgroup per CU)
__global__ __launch_bounds__(kLB, 4) void proj_lu_kernel(ProjArgs a, int b) {
  __shared__ double2 prow[kPMax + 1];     // pivot row: its columns, then its right-hand side
  __shared__ double2 lcol[2][2 * kPMax];  // multipliers / L columns by row (zero where none)
  __shared__ double2 grow[2][kPMax];      // row l of G (columns past l zero)
  __shared__ double2 ccol[2 * kPMax];     // the next pivot column, by row
  __shared__ unsigned left[4];            // rows never pivoted (bit r of word r / 32)
  __shared__ int spiv;
  __shared__ double sbest;
  __shared__ double2 sdinv;               // 1 / pivot

  const int sys = blockIdx.x, tid = threadIdx.x;
  const int tr = tid % kTR, tc = tid / kTR;
  const int s = a.s, ms = a.ms, m = a.m;
  const int k = sys / s;
  const bool has_bot = b + 1 < m;
  const int nr = has_bot ? 2 * s : s;
  const int col0 = b * s;
  const double2* Hk = a.Hm + (int64_t)k * ms * ms;
  const double2* W = wrk(a, b, sys);
  double2* zs = a.z + (int64_t)sys * ms;
  const double2 zero = make_double2(0.0, 0.0);

  // row r of the panel: r < s the current row block b, else row
  // (b + 1) s + r - s of Hm (block column b, off the diagonal: no shift)
  double2 v[kRI][kCJ];
#pragma unroll
  for (int i = 0; i < kRI; ++i)
#pragma unroll
    for (int j = 0; j < kCJ; ++j) {
      const int r = tr + kTR * i, c = tc + kTC * j;
      double2 x = zero;
      if (r < nr && c < s)
        x = r < s ? W[r + (int64_t)s * (col0 + c)]
                  : Hk[(int64_t)(col0 + r) + (int64_t)ms * (col0 + c)];
      v[i][j] = x;
    }
  // the right-hand side of each row, held by the row's owner in column
  // group 0 (zero elsewhere), and each row's position
  double2 rhs[kRI];
  int pos[kRI];
#pragma unroll
  for (int i = 0; i < kRI; ++i) {
    const int r = tr + kTR * i;
    rhs[i] = zero;
    if (tc == 0 && r < nr) rhs[i] = zs[col0 + r];
    pos[i] = r < nr ? kUnpivoted : kOutside;
  }
  for (int e = tid; e < 2 * 2 * kPMax; e += kLB) lcol[e / (2 * kPMax)][e % (2 * kPMax)] = zero;
  if (tid < 4) left[tid] = 0u;

  // Pivot of column `col`: largest |Re| + |Im| of v(r, col) over the
  // unpivoted rows (the complex magnitude of LAPACK's izamax), smallest row
  // on ties, found by the kTR = 32 owners of the column -- one half of a
  // wave -- and left in spiv / sbest for the next barrier.  Each lane packs
  // its best as a 32-bit key: the top bits of the magnitude (sign, exponent
  // and 13 mantissa bits of the double: ordered like the magnitude, so the
  // pivot is within a factor 1 + 2^-13 of the largest) over 127 - row; the
  // keys meet in four DPP steps inside each 16-lane row and two lane reads.
  auto pivot_search = [&](auto slot, int col) {
    constexpr int JC = decltype(slot)::value;
    if (tc + kTC * JC != col) return;
    {
#pragma unroll
      for (int i = 0; i < kRI; ++i) ccol[tr + kTR * i] = v[i][JC];  // the column, for (A)
      unsigned key = 0u;
#pragma unroll
      for (int i = 0; i < kRI; ++i) {
        const int r = tr + kTR * i;
        if (pos[i] == kUnpivoted) {
          const double mag = fabs(v[i][JC].x) + fabs(v[i][JC].y);
          const unsigned kk = ((unsigned)__double2hiint(mag) & ~0x7Fu) | (unsigned)(127 - r);
          key = kk > key ? kk : key;
        }
      }
      key = max_dpp(key);
      const int base = __builtin_amdgcn_readfirstlane(32 * (tc & 1));
      const unsigned k0 = (unsigned)__builtin_amdgcn_readlane((int)key, base);
      const unsigned k1 = (unsigned)__builtin_amdgcn_readlane((int)key, base + 16);
      const unsigned kw = k0 > k1 ? k0 : k1;
      // the pivot, read from its owner's lane, and its reciprocal
      const int pr = 127 - (int)(kw & 0x7Fu);
      double2 xp = zero;
#pragma unroll
      for (int i = 0; i < kRI; ++i)
        if (tr + kTR * i == pr) xp = v[i][JC];
      const double2 d = read_lane(xp, base + (pr & (kTR - 1)));
      if (tr == 0) {
        spiv = pr;
        sbest = __hiloint2double((int)(kw & ~0x7Fu), 0);
        sdinv = crecip_fast(d);
      }
    }
  };
  pivot_search(std::integral_constant<int, 0>{}, 0);
  __syncthreads();
  bool singular = false;  // a zero or non-finite pivot met so far (same in every thread)

  for_each_slot([&](auto slot) {
  constexpr int JC = decltype(slot)::value;
  for (int cl = 0; cl < kTC; ++cl) {
    const int c = kTC * JC + cl;
    if (c >= s) break;
    // the pivot row: an unpivoted row (a column of NaN picks no candidate,
    // which the flag reports; any unpivoted row then serves)
    int pr = spiv;
    singular = singular || !(sbest > 0.0) || !isfinite(sbest);
    // (A) the multipliers of column c, each thread for its own rows (from
    // the broadcast column and reciprocal); the pivot row to LDS
    const double2 dinv = singular ? make_double2(1.0, 0.0) : sdinv;
    double2 lv[kRI];
#pragma unroll
    for (int i = 0; i < kRI; ++i) {
      const int r = tr + kTR * i;
      lv[i] = zero;
      if (pos[i] == kUnpivoted && r != pr) lv[i] = cmul(ccol[r], dinv);
      if (tc + kTC * JC == c && pos[i] == kUnpivoted && r != pr) v[i][JC] = lv[i];
      if (r == pr) {
#pragma unroll
        for (int j = JC; j < kCJ; ++j) prow[tc + kTC * j] = v[i][j];
        if (tc == 0) prow[kPMax] = rhs[i];
      }
    }
    __syncthreads();
    // (B) rank-1 update of every entry: pivoted rows have multiplier zero,
    // the pivot row's columns up to c are zeroed.  The slots before JC hold
    // only columns before c (zero in the broadcast row), so they are left
    // as they are.
    double2 pv[kCJ];
#pragma unroll
    for (int j = JC; j < kCJ; ++j) {
      pv[j] = prow[tc + kTC * j];
      if (tc + kTC * j <= c) pv[j] = zero;
    }
    const double2 px = prow[kPMax];
#pragma unroll
    for (int i = 0; i < kRI; ++i) {
#pragma unroll
      for (int j = JC; j < kCJ; ++j) v[i][j] = cmsub(v[i][j], lv[i], pv[j]);
      rhs[i] = cmsub(rhs[i], lv[i], px);
      if (tr + kTR * i == pr) pos[i] = c;
    }
    if (c + 1 < s) {
      if (cl + 1 < kTC) {
        pivot_search(slot, c + 1);
      } else if constexpr (JC + 1 < kCJ) {
        pivot_search(std::integral_constant<int, JC + 1>{}, c + 1);
      }
    }
    __syncthreads();
  }
  });
  if (tid == 0 && singular) a.info[sys] = 1;

  // positions s .. 2s-1 of the rows never pivoted, in row order
#pragma unroll
  for (int i = 0; i < kRI; ++i) {
    const int r = tr + kTR * i;
    if (tc == 0 && pos[i] == kUnpivoted) atomicOr(&left[r / 32], 1u << (r % 32));
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kRI; ++i) {
    const int r = tr + kTR * i;
    if (pos[i] == kUnpivoted) {
      int below = 0;
#pragma unroll
      for (int w = 0; w < 4; ++w)
        below += __popc(w < r / 32 ? left[w] : (w == r / 32 ? left[w] & ((1u << (r % 32)) - 1u) : 0u));
      pos[i] = s + below;
    }
  }

  // the finished U block (s x s, zero below the diagonal), the eliminated rhs
  double2* Ub = a.U + (int64_t)sys * a.ustride + uoff(a, b);
#pragma unroll
  for (int i = 0; i < kRI; ++i) {
    const int p = pos[i];
    if (p < s) {
#pragma unroll
      for (int j = 0; j < kCJ; ++j) {
        const int c = tc + kTC * j;
        if (c < s) {
          // (a value select: a select between the array element and another
          // lvalue would take the array's address and keep it out of registers)
          double2 x = v[i][j];
          if (p > c) x = zero;
          Ub[p + (int64_t)s * c] = x;
        }
      }
    }
    if (tc == 0 && p < nr) zs[col0 + p] = rhs[i];
  }
  if (!has_bot) return;

  const int sp = pad16(s), nks = sp / 4, nrbt = sp / 8;
  double* Gs = a.G + (int64_t)sys * g_sys_doubles(s);
  const int64_t gim = (int64_t)nrbt * nks * 64;  // Im plane offset
  int* Gp = reinterpret_cast<int*>(Gs + 4 * (int64_t)sp * sp);
#pragma unroll
  for (int i = 0; i < kRI; ++i) {
    const int r = tr + kTR * i;
    if (tc == 0 && pos[i] < nr) Gp[pos[i]] = r;
  }

  // G = L^{-1} [I_s; 0] in the factorisation's row order: for l = 0 ..
  // s-1, the rows at positions past l lose L(., l) G(l, :); the broadcast
  // column is zero at positions up to l, the broadcast row past column l
  for_each_slot([&](auto slot) {
  constexpr int JL = decltype(slot)::value;
  for (int ll = 0; ll < kTC; ++ll) {
    const int l = kTC * JL + ll;
    if (l >= s) break;
    const int q = l & 1;
    if (tc + kTC * JL == l) {
#pragma unroll
      for (int i = 0; i < kRI; ++i) {
        const int r = tr + kTR * i;
        double2 x = zero;
        if (pos[i] > l && pos[i] < nr) x = v[i][JL];
        lcol[q][r] = x;
        v[i][JL] = make_double2(pos[i] == l ? 1.0 : 0.0, 0.0);
      }
    }
    // (the slots past JL hold only columns past l, zero in the broadcast
    // row: they are neither sent nor updated)
#pragma unroll
    for (int i = 0; i < kRI; ++i)
      if (pos[i] == l)
#pragma unroll
        for (int j = 0; j <= JL; ++j) {
          double2 x = v[i][j];
          if (tc + kTC * j > l) x = zero;
          grow[q][tc + kTC * j] = x;
        }
    __syncthreads();
    double2 gv[kCJ], lv[kRI];
#pragma unroll
    for (int j = 0; j <= JL; ++j) gv[j] = grow[q][tc + kTC * j];
#pragma unroll
    for (int i = 0; i < kRI; ++i) lv[i] = lcol[q][tr + kTR * i];
#pragma unroll
    for (int i = 0; i < kRI; ++i)
#pragma unroll
      for (int j = 0; j <= JL; ++j) v[i][j] = cmsub(v[i][j], lv[i], gv[j]);
  }
  });

  // G to its fragment order; padding rows and columns are zero
  if (sp != s) {
    for (int64_t e = tid; e < 4 * (int64_t)sp * sp; e += kLB) Gs[e] = 0.0;
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < kRI; ++i)
#pragma unroll
    for (int j = 0; j < kCJ; ++j) {
      const int p = pos[i], c = tc + kTC * j;
      if (p < nr && c < s) {
        const int gr = p < s ? p : sp + (p - s);
        const int64_t off = ((int64_t)(gr / 16) * nks + c / 4) * 64 + (gr % 16) + 16 * (c % 4);
        Gs[off] = v[i][j].x;
        Gs[gim + off] = v[i][j].y;
      }
    }
}

typedef double d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kTB = 512;  // threads of the trailing kernel: one wave per 16-row block
constexpr int kTW = 64;   // columns per workgroup (four MFMA column blocks)

// Trailing update of panel b: for the columns of one tile of one system,
//   [U12; A22'] = G T_top + [0; T_bot],
// T the panel's row permutation of the two block rows (the current row
// block and row block b + 1 of Hm, shifted on the diagonal).  Wave w owns
// row block w of the 2 sp rows (its G fragments in registers) and all four
// column blocks; T_top passes through LDS once per workgroup (Re and Im
// planes), T_bot goes straight into the bottom waves' accumulators;
// v_mfma_f64_16x16x4 in planar complex form, and the blocks of the top
// half above the diagonal of L11^{-1} (zero) are skipped.  Workgroups of
// one system are consecutive in the XCD-aware order, so the system's G is
// read from one L2.
__global__ __launch_bounds__(kTB, 4) void proj_trail_kernel(ProjArgs a, int b, int ntile) {
  __shared__ double Tt[2][kPMax][kTW + 2];
  __shared__ int sperm[2 * kPMax];
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int sys = t / ntile, tile = t % ntile;
  const int tid = threadIdx.x, lane = tid & 63;
  const int rb = tid >> 6;  // this wave's row block
  const int lr = lane & 15, lk = lane >> 4;
  const int s = a.s, ms = a.ms;
  const int sp = pad16(s), nks = sp / 4, nrbt = sp / 8, nrb_top = sp / 16;
  const int col0 = b * s;
  const int k = sys / s;
  const double2 lamv = a.lam[sys];
  const double2* Hk = a.Hm + (int64_t)k * ms * ms;
  const double2* W = wrk(a, b, sys);
  double2* Wn = wrk(a, b + 1, sys);  // the next row block, in the other buffer
  double2* Ub = a.U + (int64_t)sys * a.ustride + uoff(a, b);
  const double* Gs = a.G + (int64_t)sys * g_sys_doubles(s);
  const int64_t gim = (int64_t)nrbt * nks * 64;
  const int* Gp = reinterpret_cast<const int*>(Gs + 4 * (int64_t)sp * sp);
  const int c0 = col0 + s + tile * kTW;  // first column of the tile
  const bool live = rb < nrbt;           // waves past the padded rows idle
  const bool top = rb < nrb_top;

  for (int i = tid; i < 2 * s; i += kTB) sperm[i] = Gp[i];
  // row q (0 .. 2s-1) of the unpermuted two-block-row stack at column gc
  auto stack = [&](int q, int gc) -> double2 {
    if (q < s) return W[q + (int64_t)s * gc];
    const int grow = col0 + q;  // (b + 1) s + q - s
    double2 x = Hk[grow + (int64_t)ms * gc];
    if (grow == gc) x = csub(x, lamv);
    return x;
  };
  double gr[16], gi[16];
#pragma unroll
  for (int ks = 0; ks < 16; ++ks) {
    const bool ok = live && ks < nks;
    const int64_t off = ((int64_t)rb * nks + ks) * 64 + lane;
    gr[ks] = ok ? Gs[off] : 0.0;
    gi[ks] = ok ? Gs[gim + off] : 0.0;
  }
  __syncthreads();  // sperm

  // T_top to LDS (rows s .. sp-1 zero)
  for (int e = tid; e < sp * kTW; e += kTB) {
    const int r = e % sp, c = e / sp, gc = c0 + c;
    double2 x = make_double2(0.0, 0.0);
    if (r < s && gc < ms) x = stack(sperm[r], gc);
    Tt[0][r][c] = x.x;
    Tt[1][r][c] = x.y;
  }
  __syncthreads();
  if (!live) return;
  // two column blocks at a time (half the accumulators: two workgroups fit
  // a CU, one's staging under the other's products); T_bot goes straight
  // into the bottom waves' accumulators (D element (i, j) of a block: lane
  // j + 16 (i % 4), register i / 4)
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    d4 accr[2], acci[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int gc = c0 + 16 * (2 * half + h) + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = 16 * rb + 4 * q + lk - sp;  // bottom-half row
        double2 x = make_double2(0.0, 0.0);
        if (!top && rr < s && gc < ms) x = stack(sperm[s + rr], gc);
        accr[h][q] = x.x;
        acci[h][q] = x.y;
      }
    }
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      if (ks < nks && (!top || ks <= 4 * rb + 3)) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int cc = 16 * (2 * half + h) + lr;
          const double fr = Tt[0][4 * ks + lk][cc];
          const double fi = Tt[1][4 * ks + lk][cc];
          accr[h] = mfma64(gr[ks], fr, accr[h]);
          accr[h] = mfma64(gi[ks], -fi, accr[h]);
          acci[h] = mfma64(gr[ks], fi, acci[h]);
          acci[h] = mfma64(gi[ks], fr, acci[h]);
        }
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int gc = c0 + 16 * (2 * half + h) + lr;
      if (gc >= ms) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 16 * rb + 4 * q + lk;
        const double2 x = make_double2(accr[h][q], acci[h][q]);
        if (top) {
          if (row < s) Ub[row + (int64_t)s * (gc - col0)] = x;
        } else if (row - sp < s) {
          Wn[(row - sp) + (int64_t)s * gc] = x;
        }
      }
    }
  }
}

// Back substitution U z = y per system, row block by row block from the
// bottom; z is kept in LDS (ms complex values).  Per row block: its product
// with the solved part of z (every thread, eight column loads in flight),
// the diagonal block's upper triangle staged in LDS by the same pass, then
// the triangular solve by one wave, column by column: lane r holds row r's
// remainder, at column q lane q's remainder times 1 / U(q, q) is z(q),
// broadcast by a lane read, and the rows above subtract U(r, q) z(q).
constexpr int kBU = 8;  // column loads in flight per thread

__global__ __launch_bounds__(kPB) void proj_back_kernel(ProjArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  double2* zl = reinterpret_cast<double2*>(smem);  // ms
  double2* part = zl + a.ms;                       // kPB
  double2* ud = part + kPB;                        // s (s + 1) / 2, column q at q (q + 1) / 2
  const int sys = blockIdx.x, tid = threadIdx.x;
  const int s = a.s, ms = a.ms, m = a.m;
  const double2 zero = make_double2(0.0, 0.0);
  double2* zs = a.z + (int64_t)sys * ms;
  for (int i = tid; i < ms; i += kPB) zl[i] = zs[i];
  __syncthreads();
  const int groups = kPB / s;  // threads per row of the product
  for (int b = m - 1; b >= 0; --b) {
    const double2* Ub = a.U + (int64_t)sys * a.ustride + uoff(a, b);
    for (int e = tid; e < s * s; e += kPB) {
      const int r = e % s, q = e / s;
      if (r <= q) ud[q * (q + 1) / 2 + r] = Ub[e];
    }
    if (tid < s * groups) {
      const int r = tid % s, g = tid / s;
      const double2* Ur = Ub + r - (int64_t)s * b * s;  // element (r, c) at Ur[s c]
      double2 acc[kBU];
#pragma unroll
      for (int u = 0; u < kBU; ++u) acc[u] = zero;
      int c = (b + 1) * s + g;
      for (; c + (kBU - 1) * groups < ms; c += kBU * groups) {
        double2 uv[kBU];
#pragma unroll
        for (int u = 0; u < kBU; ++u) uv[u] = Ur[(int64_t)s * (c + u * groups)];
#pragma unroll
        for (int u = 0; u < kBU; ++u) acc[u] = cmsub(acc[u], uv[u], zl[c + u * groups]);
      }
      for (; c < ms; c += groups) acc[0] = cmsub(acc[0], Ur[(int64_t)s * c], zl[c]);
#pragma unroll
      for (int u = 1; u < kBU; ++u) acc[0] = cadd(acc[0], acc[u]);
      part[tid] = acc[0];  // minus the row's sum
    }
    __syncthreads();
    if (tid < 64) {
      double2 rem = zero, dinv = zero, zr = zero;
      if (tid < s) {
        rem = zl[b * s + tid];
        for (int g = 0; g < groups; ++g) rem = cadd(rem, part[tid + s * g]);
        dinv = crecip_fast(ud[tid * (tid + 1) / 2 + tid]);
      }
      for (int q = s - 1; q >= 0; --q) {
        const double2 w = cmul(rem, dinv);
        const double2 zq = read_lane(w, q);
        if (tid == q) zr = w;
        if (tid < q) rem = cmsub(rem, ud[q * (q + 1) / 2 + tid], zq);
      }
      if (tid < s) zl[b * s + tid] = zr;
    }
    __syncthreads();  // z(b) written, the diagonal block and partials read
  }
  for (int i = tid; i < ms; i += kPB) zs[i] = zl[i];
}

}  // namespace

int proj_max_block() { return kPMax; }

int64_t proj_u_stride(int s, int m) { return (int64_t)s * s * ((int64_t)m * (m + 1) / 2); }

int64_t proj_g_doubles(int s, int nsys) { return (int64_t)nsys * g_sys_doubles(s); }

void proj_solve(const double* Hm, const double* lam, const double* D, double* z, double* Wrk,
                double* U, double* G, int* info, int ms, int s, int m, int nsys,
                hipStream_t st) {
  if (s < 1 || s > kPMax || ms != m * s || nsys < 1)
    throw Error(TSYLV_EINVAL, "projected solve: unsupported sizes");
  ProjArgs a;
  a.Hm = reinterpret_cast<const double2*>(Hm);
  a.lam = reinterpret_cast<const double2*>(lam);
  a.D = reinterpret_cast<const double2*>(D);
  a.z = reinterpret_cast<double2*>(z);
  a.Wrk = reinterpret_cast<double2*>(Wrk);
  a.U = reinterpret_cast<double2*>(U);
  a.info = info;
  a.G = G;
  a.ms = ms;
  a.s = s;
  a.m = m;
  a.nsys = nsys;
  a.ustride = proj_u_stride(s, m);
  const int64_t work = (int64_t)nsys * s * ms;
  const int gi = (int)std::min<int64_t>((work + 255) / 256, 16384);
  hipLaunchKernelGGL(proj_init_kernel, dim3(gi), dim3(256), 0, st, a);
  TSYLV_LAUNCH_CHECK();
  for (int b = 0; b < m; ++b) {
    hipLaunchKernelGGL(proj_lu_kernel, dim3(nsys), dim3(kLB), 0, st, a, b);
    TSYLV_LAUNCH_CHECK();
    const int cols = ms - (b + 1) * s;  // trailing columns of the panel
    if (cols <= 0) continue;
    const int ntile = (cols + kTW - 1) / kTW;
    const int64_t total = (int64_t)nsys * ntile;
    if (total > 0x7fffffff) throw Error(TSYLV_EINVAL, "projected solve: too many systems");
    hipLaunchKernelGGL(proj_trail_kernel, dim3((unsigned)total), dim3(kTB), 0, st, a, b, ntile);
    TSYLV_LAUNCH_CHECK();
  }
  const size_t lds_back = sizeof(double2) * ((size_t)ms + kPB + (size_t)s * (s + 1) / 2);
  if (lds_back > 160 * 1024) throw Error(TSYLV_EINVAL, "projected solve: ms too large");
  TSYLV_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&proj_back_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_back));
  hipLaunchKernelGGL(proj_back_kernel, dim3(nsys), dim3(kPB), lds_back, st, a);
  TSYLV_LAUNCH_CHECK();
}

}  // namespace kern
}  // namespace tsylv
