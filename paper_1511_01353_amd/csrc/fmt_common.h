// Internal definitions shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fmt.h"

namespace fmt {

// ---------------------------------------------------------------------------
// Basis: monomials of total degree <= P in graded order (Section 2, geometric
// moments and rank stride).  Exponent tables are compile-time constants.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int basis_size(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
__host__ __device__ constexpr int pad16(int n) { return (n + 15) / 16 * 16; }

template <int P>
struct Basis {
  static constexpr int L = basis_size(P);
  int lx[L > 0 ? L : 1], ly[L > 0 ? L : 1], lz[L > 0 ? L : 1];
  double inv_fact[L > 0 ? L : 1];
  constexpr Basis() : lx(), ly(), lz(), inv_fact() {
    int i = 0;
    for (int k = 0; k <= P; ++k)
      for (int l = k; l >= 0; --l)
        for (int m = k - l; m >= 0; --m) {
          int n = k - l - m;
          lx[i] = l; ly[i] = m; lz[i] = n;
          double f = 1.0;
          for (int a = 2; a <= l; ++a) f *= a;
          for (int a = 2; a <= m; ++a) f *= a;
          for (int a = 2; a <= n; ++a) f *= a;
          inv_fact[i] = 1.0 / f;
          ++i;
        }
  }
};

// Position of the monomial u^a v^b w^c in the graded order.
__host__ __device__ __forceinline__ int graded(int a, int b, int c) {
  const int k = a + b + c;
  return k * (k + 1) * (k + 2) / 6 + (k - a) * (k - a + 1) / 2 + (k - a - b);
}

// Scaled powers t^k / k! for k = 0..P, built by repeated multiplication.
template <int P, typename T>
__device__ __forceinline__ void scaled_powers(T t, T (&pw)[P + 1]) {
  pw[0] = T(1);
#pragma unroll
  for (int k = 1; k <= P; ++k) pw[k] = pw[k - 1] * t * (T(1) / T(k));
}

// sum_i F[i] Lambda_i(u) with compile-time indices; F read through a pointer
// (LDS or global).  Nested Horner form, w innermost:
//   sum_l u^l/l! sum_m v^m/m! sum_n F_lmn w^n/n!,
// each level evaluated as c_0 + (t/1)(c_1 + (t/2)(c_2 + ...)), so every
// coefficient costs one fused multiply-add and few values stay live.
template <int P, typename T, typename FPtr>
__device__ __forceinline__ T poly_eval(const FPtr F, T u, T v, T w) {
  T ud[P + 1], vd[P + 1], wd[P + 1];
#pragma unroll
  for (int k = 0; k <= P; ++k) {
    ud[k] = u * (T(1) / T(k + 1));
    vd[k] = v * (T(1) / T(k + 1));
    wd[k] = w * (T(1) / T(k + 1));
  }
  T f = T(0);
#pragma unroll
  for (int l = P; l >= 0; --l) {
    T g = T(0);
#pragma unroll
    for (int m = P - l; m >= 0; --m) {
      T h = T(0);
#pragma unroll
      for (int n = P - l - m; n >= 0; --n) {
        const int k = l + m + n;
        const int idx = k * (k + 1) * (k + 2) / 6 + (k - l) * (k - l + 1) / 2 + (k - l - m);
        h = T(F[idx]) + h * wd[n];
      }
      g = h + g * vd[m];
    }
    f = g + f * ud[l];
  }
  return f;
}

// poly_eval for NPT points at once: every coefficient is read once and feeds
// NPT independent Horner chains.
template <int P, int NPT, typename FPtr>
__device__ __forceinline__ void poly_eval_multi(const FPtr F, const double (&u)[NPT], const double (&v)[NPT],
                                                const double (&w)[NPT], double (&out)[NPT]) {
  double f[NPT];
#pragma unroll
  for (int q = 0; q < NPT; ++q) f[q] = 0.0;
#pragma unroll
  for (int l = P; l >= 0; --l) {
    double g[NPT];
#pragma unroll
    for (int q = 0; q < NPT; ++q) g[q] = 0.0;
#pragma unroll
    for (int m = P - l; m >= 0; --m) {
      double h[NPT];
#pragma unroll
      for (int q = 0; q < NPT; ++q) h[q] = 0.0;
#pragma unroll
      for (int n = P - l - m; n >= 0; --n) {
        const int k = l + m + n;
        const int idx = k * (k + 1) * (k + 2) / 6 + (k - l) * (k - l + 1) / 2 + (k - l - m);
        const double c = F[idx];
#pragma unroll
        for (int q = 0; q < NPT; ++q) h[q] = c + h[q] * (w[q] * (1.0 / (double)(n + 1)));
      }
#pragma unroll
      for (int q = 0; q < NPT; ++q) g[q] = h[q] + g[q] * (v[q] * (1.0 / (double)(m + 1)));
    }
#pragma unroll
    for (int q = 0; q < NPT; ++q) f[q] = g[q] + f[q] * (u[q] * (1.0 / (double)(l + 1)));
  }
#pragma unroll
  for (int q = 0; q < NPT; ++q) out[q] = f[q];
}


// ---------------------------------------------------------------------------
// Tunables
// ---------------------------------------------------------------------------
constexpr int CHUNK = 2048;          // points per (node, chunk) work item
constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 16;       // keys per thread per tile
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;
constexpr int MAX_RADIX_BITS = 10;  // radix sort digits are 8 to 10 bits wide

// ---------------------------------------------------------------------------
// Device node table (structure of arrays, capacity `cap` nodes).
// Nodes are stored level by level; a node's children are contiguous and in
// octant order, so (level, prefix) order is the storage order within each
// problem.
// ---------------------------------------------------------------------------
struct NodeTable {
  uint32_t* begin;       // first sorted point
  uint32_t* count;       // points
  uint32_t* prefix;      // Morton prefix of the cell (3*level bits)
  uint32_t* level;       // depth
  uint32_t* problem;     // problem index inside the forest
  uint32_t* parent;      // parent node (self for a root)
  uint32_t* first_child; // first child node (valid if child_mask != 0)
  uint32_t* child_mask;  // bit o set if octant o is a node
  uint32_t* flags;       // FLAG_DEFLATED, FLAG_NONFINITE, FLAG_REFINE (below)
  double* geo;           // 6 per node: centre x,y,z then dilation 2/h x,y,z
  double* coef;          // L per node
};

constexpr uint32_t FLAG_DEFLATED = 1u;
constexpr uint32_t FLAG_NONFINITE = 2u;
constexpr uint32_t FLAG_REFINE = 4u;   // the refinement sweeps apply to this node
// mixed path: the node's float32 Gram was too ill-conditioned to solve from,
// so its normal equations were formed again from float64 moments
constexpr uint32_t FLAG_REGRAM = 8u;

// Per-problem parameters of one batched fit.
struct ProblemParams {
  double lo[3];
  double qscale[3];   // 2^D / (hi - lo)
  double hi[3];
  uint32_t n;         // points
  uint32_t offset;    // first global point index
};

// ---------------------------------------------------------------------------
// Cells and Morton keys
// ---------------------------------------------------------------------------
// Spread the low 10 bits of v so that bit b lands on bit 3b.
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Cell index at the finest depth along one axis.  The subtraction and the
// product are separate roundings (no fused multiply-add).
__device__ __forceinline__ uint32_t cell_of(double x, double lo, double qscale, uint32_t cmax,
                                            bool* bad) {
  double t = floor(__dmul_rn(__dsub_rn(x, lo), qscale));
  if (!(t == t)) { *bad = true; return 0u; }
  if (t < 0.0) return 0u;
  if (t > (double)cmax) return cmax;
  return (uint32_t)t;
}

}  // namespace fmt
