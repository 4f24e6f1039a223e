// Moment pyramid: the power moments M_gamma (|gamma| <= 2p) of every cell of
// the top levels of the octree, accumulated once over the points at the
// pyramid's finest level and carried upward by an exact change of frame.
//
// The normal equations of Alg. 2 at a node use M (which does not depend on
// the residual) and B_alpha = sum r u^alpha (which changes from level to
// level, Alg. 1).  A cell's M is the sum over its eight children of their
// moments re-expressed in the parent's frame: with u_parent = (u_child +
// sigma) / 2 on each axis (sigma = +1 for the upper half, -1 for the lower),
//   sum u_p^a = 2^-a sum_{a' <= a} C(a, a') sigma^(a - a') sum u_c^a',
// applied axis by axis.  So each level's point pass needs only B, and M is
// read from the pyramid.
//
// Each problem q of a batch has its own pyramid of levels 0 .. kp_q (kp_q =
// 0: none), stored problem after problem: cell `prefix` of level d of
// problem q is entry base_q + (8^d - 1) / 7 + prefix, so the children of a
// cell are 8 consecutive entries of the next level.  The finest cells of
// all pyramids are also numbered flat, problem after problem.
#include "k_level.h"

namespace fmt {

// Flat finest cell of a sorted key (0xffffffff: its problem has no pyramid).
__device__ __forceinline__ uint32_t flat_cell(uint32_t key, int D, int nprob, const uint32_t* __restrict__ tab) {
  const uint32_t q = nprob > 1 ? key >> (3 * D) : 0u;
  const uint32_t* t = tab + PYR_TAB_WORDS * q;
  const int kp = (int)t[1];
  if (kp == 0) return 0xffffffffu;
  return t[2] + ((key & ((1u << (3 * D)) - 1u)) >> (3 * (D - kp)));
}

// Boundary pass over the sorted keys: the first point of each non-empty
// finest cell records itself as the cell's begin, the last one the cell's
// end (stored in count; empty cells keep the zeros they start with).
__global__ void __launch_bounds__(256) k_pyr_mark(const uint32_t* __restrict__ skey, uint32_t n, int D, int nprob,
                                                  const uint32_t* __restrict__ tab, uint32_t* __restrict__ begin,
                                                  uint32_t* __restrict__ end) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t f = flat_cell(skey[i], D, nprob, tab);
  if (f == 0xffffffffu) return;
  if (i == 0 || flat_cell(skey[i - 1], D, nprob, tab) != f) begin[f] = i;
  if (i + 1 == n || flat_cell(skey[i + 1], D, nprob, tab) != f) end[f] = i + 1;
}

// Per finest cell (flat numbering, problem bq[j] owns cells cstart[j] ..
// cstart[j+1]-1): point count from the boundary pass, frame, chunk count and
// pyramid entry (one thread per cell).
__global__ void __launch_bounds__(256) k_pyr_cells(const ProblemParams* __restrict__ prm, PyrTab pt, uint32_t ncell,
                                                   const uint32_t* __restrict__ begin, uint32_t* __restrict__ count,
                                                   double* __restrict__ geo, uint32_t* __restrict__ nchk,
                                                   uint32_t* __restrict__ dst) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  uint32_t lo = 0, hi = pt.nbase - 1;   // last j with cstart[j] <= c
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (pt.cstart[mid] <= c) lo = mid;
    else hi = mid - 1;
  }
  const uint32_t q = pt.bq[lo], pre = c - pt.cstart[lo];
  const uint32_t* t = pt.tab + PYR_TAB_WORDS * q;
  const int kp = (int)t[1];
  double g[6];
  node_geo(prm[q], kp, pre, g);
  const uint32_t cnt = count[c] - begin[c];   // count holds the end until here
  count[c] = cnt;
#pragma unroll
  for (int i = 0; i < 6; ++i) geo[6 * (size_t)c + i] = g[i];
  nchk[c] = (cnt + CHUNK - 1) / CHUNK;
  dst[c] = t[0] + level_first(kp) + pre;
}

// Exclusive scan of the cells' chunk counts into off[0..ncell] (one
// workgroup; each thread scans a contiguous run of cells).
__global__ void __launch_bounds__(1024) k_pyr_scan(const uint32_t* __restrict__ nchk, uint32_t ncell,
                                                   uint32_t* __restrict__ off) {
  __shared__ uint32_t wsum[16];
  const uint32_t t = threadIdx.x, per = (ncell + 1023) / 1024;
  const uint32_t b = t * per, e = min(b + per, ncell);
  uint32_t s = 0;
  for (uint32_t i = b; i < e; ++i) s += nchk[i];
  const int lane = (int)(t & 63), w = (int)(t >> 6);
  uint32_t x = s;   // inclusive scan inside the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t base = 0;
  for (int q = 0; q < w; ++q) base += wsum[q];
  uint32_t run = base + x - s;
  for (uint32_t i = b; i < e; ++i) {
    off[i] = run;
    run += nchk[i];
  }
  if (t == 1023) off[ncell] = base + x;
}

// Finest pyramid levels: each cell's chunk partials summed in a fixed order
// (zeros for an empty cell) into its pyramid entry dst[k].  Workgroups stride
// over the cells; a cell with several chunks is summed by 16 rows of 64
// columns, 8 accumulators each.
__global__ void __launch_bounds__(1024) k_pyr_base(const uint32_t* __restrict__ off, uint32_t ncell,
                                                   const double* __restrict__ part, uint32_t width,
                                                   const uint32_t* __restrict__ dsts, double* __restrict__ pyr) {
  __shared__ double red[16][64];
  const uint32_t lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  for (uint32_t k = blockIdx.x; k < ncell; k += gridDim.x) {
    const uint32_t c0 = off[k], c1 = off[k + 1];
    double* dst = pyr + (size_t)dsts[k] * width;
    if (c1 == c0) {
      for (uint32_t e = threadIdx.x; e < width; e += 1024) dst[e] = 0.0;
      continue;
    }
    if (c1 - c0 == 1) {
      const double* src = part + (size_t)c0 * width;
      for (uint32_t e = threadIdx.x; e < width; e += 1024) dst[e] = src[e];
      continue;
    }
    for (uint32_t e0 = 0; e0 < width; e0 += 64) {
      const uint32_t e = e0 + lane;
      double acc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = 0.0;
      if (e < width) {
        uint32_t g = c0 + q;
        for (; g + 16 * 7 < c1; g += 16 * 8) {
#pragma unroll
          for (int u = 0; u < 8; ++u) acc[u] += part[(size_t)(g + 16 * u) * width + e];
        }
        for (; g < c1; g += 16) acc[0] += part[(size_t)g * width + e];
      }
      red[q][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
      __syncthreads();
      if (q == 0 && e < width) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = red[2 * u][lane] + red[2 * u + 1][lane];
        dst[e] = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
      }
      __syncthreads();
    }
  }
}

// Binomial coefficients C(n, m), n, m <= 16, as compile-time constants.
struct Binomials {
  double c[17][17];
  constexpr Binomials() : c() {
    for (int n = 0; n <= 16; ++n) {
      c[n][0] = 1.0;
      for (int m = 1; m <= n; ++m) c[n][m] = c[n - 1][m - 1] + (m <= n - 1 ? c[n - 1][m] : 0.0);
    }
  }
};

// The lines of the moment tensor (|gamma| <= P2) along one axis: line j
// fixes the exponents (f0, f1) of the other two axes, f0 + f1 <= P2.
template <int P2>
struct Lines {
  static constexpr int N = (P2 + 1) * (P2 + 2) / 2;
  int f0[N], f1[N];
  constexpr Lines() : f0(), f1() {
    int j = 0;
    for (int a = 0; a <= P2; ++a)
      for (int b = 0; a + b <= P2; ++b) {
        f0[j] = a;
        f1[j] = b;
        ++j;
      }
  }
};

// One line along AXIS (other exponents f0, f1 in axis order) of the pair of
// children (hi, lo) that differ only along AXIS, in their parent's frame:
// out_n = 2^-n sum_{m <= n} C(n, m) (hi_m + (-1)^(n - m) lo_m).  The line's
// entries are read once into registers.
template <int P2, int AXIS>
__device__ __forceinline__ void shift_line(const double* hi, const double* lo, double* out, int f0, int f1) {
  constexpr Binomials BN{};
  const int len = P2 - f0 - f1 + 1;
  int idx[P2 + 1];
  double sp[P2 + 1], sm[P2 + 1];   // hi + lo, hi - lo
#pragma unroll
  for (int m = 0; m <= P2; ++m) {
    const int e = m < len ? m : 0;
    const int x = AXIS == 0 ? e : f0;
    const int y = AXIS == 1 ? e : (AXIS == 0 ? f0 : f1);
    const int z = AXIS == 2 ? e : f1;
    idx[m] = graded(x, y, z);
    const double h = hi[idx[m]], l = lo[idx[m]];
    sp[m] = h + l;
    sm[m] = h - l;
  }
#pragma unroll
  for (int n = 0; n <= P2; ++n) {
    if (n < len) {
      double sum = 0.0;
#pragma unroll
      for (int m = 0; m <= n; ++m) sum = fma(BN.c[n][m], ((n - m) & 1) ? sm[m] : sp[m], sum);
      out[idx[n]] = ldexp(sum, -n);
    }
  }
}

// One level up, for the problems whose pyramid extends below level d: the
// parent is cell `prefix` of level d of problem list[j], built from its
// children (8 consecutive entries of level d+1) by shifting along z (pairs
// 2q, 2q+1), then y, then x, one tensor line per thread.  One workgroup of
// UP_THREADS per parent.
constexpr int UP_THREADS = 512;

template <int P>
__global__ void __launch_bounds__(UP_THREADS) k_pyr_up(double* __restrict__ pyr, const uint32_t* __restrict__ tab,
                                                       const uint32_t* __restrict__ list, int d) {
  constexpr int P2 = 2 * P;
  constexpr int NM = basis_size(P2);
  constexpr Lines<P2> LN{};
  constexpr int NL = Lines<P2>::N;
  __shared__ double A[8 * NM], Bv[4 * NM];
  const int tid = threadIdx.x;
  const uint32_t j = blockIdx.x >> (3 * d), pre = blockIdx.x & ((1u << (3 * d)) - 1u);
  const uint32_t base = tab[PYR_TAB_WORDS * list[j]];
  const size_t parent = (size_t)base + level_first(d) + pre;
  const size_t child = (size_t)base + level_first(d + 1) + 8ull * pre;
  copy_to_lds<UP_THREADS, 8 * NM>(A, pyr + child * NM, tid);
  __syncthreads();
  // z: lines (x, y fixed) of the pairs (2q, 2q+1)
  for (int t = tid; t < 4 * NL; t += UP_THREADS) {
    const int q = t / NL, l = t - q * NL;
    shift_line<P2, 2>(A + (2 * q + 1) * NM, A + 2 * q * NM, Bv + q * NM, LN.f0[l], LN.f1[l]);
  }
  __syncthreads();
  // y: lines (x, z fixed) of the pairs (2q, 2q+1) of the z results
  for (int t = tid; t < 2 * NL; t += UP_THREADS) {
    const int q = t / NL, l = t - q * NL;
    shift_line<P2, 1>(Bv + (2 * q + 1) * NM, Bv + 2 * q * NM, A + q * NM, LN.f0[l], LN.f1[l]);
  }
  __syncthreads();
  // x: lines (y, z fixed), straight to the parent's entry
  for (int t = tid; t < NL; t += UP_THREADS)
    shift_line<P2, 0>(A + NM, A, pyr + parent * NM, LN.f0[t], LN.f1[t]);
}

hipError_t launch_pyr_cells(const uint32_t* skey, uint32_t n, int D, int nprob, const ProblemParams* prm,
                            const PyrTab& pt, uint32_t ncell, uint32_t* begin, uint32_t* count, double* geo,
                            uint32_t* nchk, uint32_t* dst, hipStream_t s) {
  if (ncell == 0) return hipSuccess;
  if (n) hipLaunchKernelGGL(k_pyr_mark, dim3((n + 255) / 256), dim3(256), 0, s, skey, n, D, nprob, pt.tab, begin, count);
  hipLaunchKernelGGL(k_pyr_cells, dim3((ncell + 255) / 256), dim3(256), 0, s, prm, pt, ncell, begin, count, geo,
                     nchk, dst);
  return hipGetLastError();
}

hipError_t launch_pyr_scan(const uint32_t* nchk, uint32_t ncell, uint32_t* off, hipStream_t s) {
  hipLaunchKernelGGL(k_pyr_scan, dim3(1), dim3(1024), 0, s, nchk, ncell, off);
  return hipGetLastError();
}

hipError_t launch_pyr_base(const uint32_t* off, uint32_t ncell, const double* part, uint32_t width,
                           const uint32_t* dst, double* pyr, hipStream_t s) {
  if (ncell == 0) return hipSuccess;
  const uint32_t grid = ncell < 2048 ? ncell : 2048;
  hipLaunchKernelGGL(k_pyr_base, dim3(grid), dim3(1024), 0, s, off, ncell, part, width, dst, pyr);
  return hipGetLastError();
}

template <int P>
static hipError_t pyr_up_impl(double* pyr, const uint32_t* tab, const uint32_t* list, uint32_t nlist, int d,
                              hipStream_t s) {
  if (nlist == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pyr_up<P>, dim3(nlist << (3 * d)), dim3(UP_THREADS), 0, s, pyr, tab, list, d);
  return hipGetLastError();
}

hipError_t launch_pyr_up(int p, double* pyr, const uint32_t* tab, const uint32_t* list, uint32_t nlist, int d,
                         hipStream_t s) {
  FMT_DISPATCH_P(p, pyr_up_impl, pyr, tab, list, nlist, d, s);
}

}  // namespace fmt
