// Pieces shared by the small-basis LDL^T solves (Alg. 2's per-node solve on
// the normal equations): the blocked storage of a factor, the pivot
// threshold and reciprocal, the condition-estimate probes and bounds, and the
// flag for coefficients that are not finite.
#pragma once

#include "k_level.h"

namespace fmt {

typedef double solve_d4 __attribute__((ext_vector_type(4)));

// Pivots of the equilibrated Gram (unit diagonal) at or below this are
// treated as linear dependence: the column is dropped from the factor.
constexpr double PIVOT_EPS = 1e-13;

// ---------------------------------------------------------------------------
// Blocked lower-triangular storage of an n x n symmetric matrix in LDS,
// n padded to T blocks of 16: block (I, J), I >= J, holds 16 x 16 doubles;
// element (r, c) of a block sits at 16 r + (c ^ (r >> 1)) so that the MFMA
// operand pattern (16 rows, one column each) spreads over the LDS banks.
// ---------------------------------------------------------------------------
template <int L>
struct BlockShape {
  static constexpr int T = (L + 15) / 16;
  static constexpr int LP = 16 * T;
  static constexpr int NBLK = T * (T + 1) / 2;
  static constexpr int WORDS = NBLK * 256;
};

__device__ __forceinline__ int bidx(int I, int J) { return (I * (I + 1) / 2 + J) * 256; }
__device__ __forceinline__ int bel(int r, int c) { return r * 16 + (c ^ (r >> 1)); }
// element (i, j), i and j in the lower block triangle (i >> 4 >= j >> 4)
__device__ __forceinline__ int belem(int i, int j) { return bidx(i >> 4, j >> 4) + bel(i & 15, j & 15); }

// Value of a double held by lane `l` (a wave-uniform index), in scalar
// registers: two v_readlane_b32, no LDS round trip.
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long bits = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(bits & 0xffffffffll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 1 / d for a pivot of the equilibrated matrix (0 < d <= ~1): the hardware
// reciprocal estimate refined by two Newton steps (error well under 1 ulp
// of the estimate's square), instead of the full IEEE division sequence.
__device__ __forceinline__ double pivot_recip(double d) {
  double x = __builtin_amdgcn_rcp(d);
  double e = fma(-d, x, 1.0);
  x = fma(x, e, x);
  e = fma(-d, x, 1.0);
  return fma(x, e, x);
}

// With a status word, a node's coefficients that are not all finite mark the
// node (FLAG_NONFINITE) and the fit (status bit 2); `bad` is this thread's
// finding for the coefficients it wrote.  Callers test with isfinite: the
// test c - c == 0 on a product just computed may be contracted into a fused
// multiply-add that returns the product's rounding error.
__device__ __forceinline__ void mark_nonfinite(bool bad, uint32_t* flag, uint32_t* status) {
  if (status && bad) {
    atomicOr(flag, FLAG_NONFINITE);
    atomicOr(status, 2u);
  }
}

// Refinement is needed where the equilibrated normal equations are
// ill-conditioned: with the estimate below at or under this bound the float64
// solve's fitted values are accurate to ~1e-13 relative, and one sweep is
// applied above it.
constexpr double REFINE_KAPPA = 1e6;
// Mixed path: a float32 Gram carries entry errors of a few 1e-10 relative
// (float32 sums over short runs of points, flushed to float64), so above
// this estimated condition number its solve, even refined, misses the
// float64 answer; such nodes are solved again from float64 moments.
constexpr double REGRAM_KAPPA = 1e6;

// Entry i of the fixed probe vector `which` (0 or 1): +-1/sqrt(L) with signs
// from an integer hash, so the estimate is deterministic.
__device__ __forceinline__ double probe_entry(int i, int which, int L) {
  uint32_t h = (uint32_t)i * 0x9E3779B1u + (uint32_t)which * 0x85EBCA77u + 0x165667B1u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  return ((h >> 7) & 1u ? 1.0 : -1.0) * rsqrt((double)L);
}

// Doubles of one kept factor: [blocked L and D | D | D^-1 | scales].
template <int L>
__host__ __device__ constexpr size_t factor_words() {
  return (size_t)BlockShape<L>::WORDS + 3 * (size_t)L;
}

}  // namespace fmt
