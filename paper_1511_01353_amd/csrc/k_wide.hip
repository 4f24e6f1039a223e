// Per-node solve for large bases (p = 10, 12, 14: calL = 286, 455, 680).
//
// The equilibrated normal equations of such a node (calL^2 doubles, up to
// 3.7 MB) do not fit a workgroup's LDS, so they live in device memory as
// 32 x 32 tiles of the lower triangle and are factored by a blocked
// right-looking Cholesky: per block column J, (1) the diagonal tile is
// factored in LDS and its triangular inverse formed, (2) the tiles below it
// become L_IJ = A_IJ L_JJ^-T, (3) the trailing tiles take A_IK -= L_IJ L_KJ^T.
// Each phase is one launch over every node of the level (grid x: node, grid
// y: tile), so a level of many nodes fills the chip and a single large node
// spreads its trailing updates over many workgroups.
//
// The matrix is the one the small-basis solve factors (Alg. 2's least-squares
// problem in normal-equation form, reading 15): G_ik = M[a_i + a_k] /
// (a_i! a_k!) from the node's power moments, equilibrated to unit diagonal:
// A_ik = M[a_i + a_k] w_i w_k with w_i = 1 / sqrt(M[2 a_i]), right-hand side
// b_i = B[a_i] w_i, coefficients F_i = a_i! w_i z_i.  A pivot at or below
// 1e-13 is deflated as in the small-basis LDL^T: its row of the diagonal
// tile's inverse is zeroed, so its column of L is zero and the solves give
// that unknown 0.
#include "k_level.h"

namespace fmt {

constexpr int WT = 32;                    // tile edge
constexpr int WT2 = WT * WT;
constexpr double WIDE_PIVOT_EPS = 1e-13;  // as the small-basis factor
constexpr double WIDE_REFINE_KAPPA = 1e6; // as the small-basis solve

struct WideShape {
  int L, T, LP;
  size_t tiles;   // lower-triangle tiles
  size_t words;   // doubles of one node's factor
};

__host__ __device__ inline WideShape wide_shape(int L) {
  WideShape w;
  w.L = L;
  w.T = (L + WT - 1) / WT;
  w.LP = w.T * WT;
  w.tiles = (size_t)w.T * (w.T + 1) / 2;
  // [tiles | inverse diagonal tiles | F scale a_i! w_i | w_i | kept (1/0)]
  w.words = (w.tiles + (size_t)w.T) * WT2 + 2 * (size_t)L + (size_t)w.LP;
  return w;
}

// offsets inside one node's factor
__device__ __forceinline__ size_t wtile(int I, int J) { return ((size_t)I * (I + 1) / 2 + J) * WT2; }
__device__ __forceinline__ size_t winv(const WideShape& s, int J) { return (s.tiles + (size_t)J) * WT2; }
__device__ __forceinline__ size_t wscale(const WideShape& s) { return (s.tiles + (size_t)s.T) * WT2; }
__device__ __forceinline__ size_t wweight(const WideShape& s) { return wscale(s) + s.L; }
__device__ __forceinline__ size_t wkept(const WideShape& s) { return wscale(s) + 2 * (size_t)s.L; }

bool wide_order(int p) { return p == 10 || p == 12 || p == 14; }

size_t wide_factor_doubles(int p) { return wide_shape(basis_size(p)).words; }

// A node whose coefficients are not all finite is marked (FLAG_NONFINITE)
// and so is the fit (status bit 2); `bad` is this thread's finding.
__device__ __forceinline__ void flag_nonfinite(bool bad, uint32_t* flag, uint32_t* status) {
  if (status && bad) {
    atomicOr(flag, FLAG_NONFINITE);
    atomicOr(status, 2u);
  }
}

// Exponents (l, m, n) of basis index i in graded order (degree k, then l
// descending, then m descending), and l! m! n!.
__device__ __forceinline__ void graded_exponents(int i, int& l, int& m, int& n) {
  int k = 0;
  while ((k + 1) * (k + 2) * (k + 3) / 6 <= i) ++k;
  int j = i - k * (k + 1) * (k + 2) / 6;
  l = k;
  while (j >= k - l + 1) {
    j -= k - l + 1;
    --l;
  }
  m = (k - l) - j;
  n = k - l - m;
}

__device__ __forceinline__ double factorial3(int l, int m, int n) {
  double f = 1.0;
  for (int a = 2; a <= l; ++a) f *= (double)a;
  for (int a = 2; a <= m; ++a) f *= (double)a;
  for (int a = 2; a <= n; ++a) f *= (double)a;
  return f;
}

// ---------------------------------------------------------------------------
// Assembly: workgroup (node k, tile row I) writes tiles (I, 0..I) of the
// equilibrated matrix (padding rows and columns: the identity) and the
// scales of its 32 rows.  mom: the node's summed mode-0 partial (M in graded
// order up to degree 2p, then B).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_wide_assemble(LevelArgs a, const double* __restrict__ part_m,
                                                       double* __restrict__ fac, int L, int NOUT) {
  const WideShape ws = wide_shape(L);
  __shared__ uint32_t ex[WT * 24];   // packed exponents of the rows and columns of this tile row (LP <= 768)
  __shared__ double wv[WT * 24];
  const int tid = threadIdx.x;
  const uint32_t k = blockIdx.x;
  const int I = blockIdx.y;
  const double* mom = part_m + (size_t)a.chunk_off[k] * NOUT;
  double* fo = fac + (size_t)k * ws.words;
  const int ncol = WT * (I + 1);
  for (int i = tid; i < ncol; i += 256) {
    uint32_t e = 0;
    double w = 0.0;
    if (i < L) {
      int l, m, n;
      graded_exponents(i, l, m, n);
      e = (uint32_t)l | ((uint32_t)m << 8) | ((uint32_t)n << 16);
      const double d = mom[graded(2 * l, 2 * m, 2 * n)];
      w = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
      if (i >= WT * I) {   // this tile row's own rows: their scales
        fo[wscale(ws) + i] = w * factorial3(l, m, n);
        fo[wweight(ws) + i] = w;
      }
    }
    ex[i] = e;
    wv[i] = w;
  }
  __syncthreads();
  for (int e = tid; e < (I + 1) * WT2; e += 256) {
    const int J = e / WT2, r = (e % WT2) / WT, c = e % WT;
    const int i = WT * I + r, q = WT * J + c;
    double v;
    if (i < L && q < L) {
      const uint32_t s = ex[i] + ex[q];
      v = mom[graded((int)(s & 255u), (int)((s >> 8) & 255u), (int)(s >> 16))] * wv[i] * wv[q];
    } else {
      v = i == q ? 1.0 : 0.0;
    }
    fo[wtile(I, J) + (size_t)r * WT + c] = v;
  }
}

// ---------------------------------------------------------------------------
// Phase 1: factor the diagonal tile J of every node in LDS (Cholesky with
// deflation), then invert it (forward substitution on the unit columns) and
// zero the inverse's rows of deflated pivots; store the inverse and the kept
// flags of the tile's columns.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_wide_potrf(LevelArgs a, double* __restrict__ fac, int L, int J) {
  const WideShape ws = wide_shape(L);
  __shared__ double t[WT][WT + 1];
  __shared__ double x[WT][WT + 1];
  __shared__ double keep[WT];
  const int tid = threadIdx.x;
  double* fo = fac + (size_t)blockIdx.x * ws.words;
  const double* src = fo + wtile(J, J);
  for (int e = tid; e < WT2; e += 256) t[e / WT][e % WT] = src[e];
  __syncthreads();
  for (int kk = 0; kk < WT; ++kk) {
    const double d = t[kk][kk];
    const bool kept = d > WIDE_PIVOT_EPS;
    const double lkk = kept ? sqrt(d) : 1.0;
    __syncthreads();   // every thread has read the pivot
    if (tid > kk && tid < WT) t[tid][kk] = kept ? t[tid][kk] / lkk : 0.0;
    if (tid == 0) {
      t[kk][kk] = lkk;
      keep[kk] = kept ? 1.0 : 0.0;
    }
    __syncthreads();
    // trailing update of the tile's lower part: (r, c), kk < c <= r
    for (int e = tid; e < WT2; e += 256) {
      const int r = e / WT, c = e % WT;
      if (c > kk && c <= r) t[r][c] -= t[r][kk] * t[c][kk];
    }
    __syncthreads();
  }
  // inverse of the lower-triangular tile, one column per thread
  if (tid < WT) {
    const int j = tid;
    for (int i = 0; i < WT; ++i) {
      if (i < j) {
        x[i][j] = 0.0;
        continue;
      }
      double s = i == j ? 1.0 : 0.0;
      for (int m = j; m < i; ++m) s -= t[i][m] * x[m][j];
      x[i][j] = s / t[i][i];
    }
  }
  __syncthreads();
  double* inv = fo + winv(ws, J);
  for (int e = tid; e < WT2; e += 256) {
    const int r = e / WT, c = e % WT;
    inv[e] = keep[r] != 0.0 ? x[r][c] : 0.0;
  }
  if (tid < WT) fo[wkept(ws) + WT * J + tid] = keep[tid];
}

// 32 x 32 product out[r][c] (+)= s * sum_m A[r][m] B[c][m] with the tiles in
// LDS: 256 threads, four outputs each (row tid / 8, columns 4 (tid % 8) + q).
__device__ __forceinline__ void tile_abt(const double (*A)[WT + 1], const double (*B)[WT + 1], double (&acc)[4]) {
  const int tid = threadIdx.x, r = tid >> 3, c0 = (tid & 7) * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = 0.0;
#pragma unroll 8
  for (int m = 0; m < WT; ++m) {
    const double av = A[r][m];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = fma(av, B[c0 + q][m], acc[q]);
  }
}

// ---------------------------------------------------------------------------
// Phase 2: L_IJ = A_IJ Linv_JJ^T for the tiles below the diagonal tile J
// (grid y: I - J - 1).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_wide_trsm(LevelArgs a, double* __restrict__ fac, int L, int J) {
  const WideShape ws = wide_shape(L);
  __shared__ double ta[WT][WT + 1];
  __shared__ double tb[WT][WT + 1];
  const int tid = threadIdx.x;
  const int I = J + 1 + (int)blockIdx.y;
  double* fo = fac + (size_t)blockIdx.x * ws.words;
  double* dst = fo + wtile(I, J);
  const double* inv = fo + winv(ws, J);
  for (int e = tid; e < WT2; e += 256) {
    ta[e / WT][e % WT] = dst[e];
    tb[e / WT][e % WT] = inv[e];
  }
  __syncthreads();
  double acc[4];
  tile_abt(ta, tb, acc);
  const int r = tid >> 3, c0 = (tid & 7) * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) dst[r * WT + c0 + q] = acc[q];
}

// ---------------------------------------------------------------------------
// Phase 3: trailing update A_IK -= L_IJ L_KJ^T for J < K <= I (grid y: the
// pair's index, column by column).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_wide_syrk(LevelArgs a, double* __restrict__ fac, int L, int J) {
  const WideShape ws = wide_shape(L);
  __shared__ double ta[WT][WT + 1];
  __shared__ double tb[WT][WT + 1];
  const int tid = threadIdx.x;
  int p = (int)blockIdx.y, K = J + 1;
  while (p >= ws.T - K) {
    p -= ws.T - K;
    ++K;
  }
  const int I = K + p;
  double* fo = fac + (size_t)blockIdx.x * ws.words;
  const double* li = fo + wtile(I, J);
  const double* lk = fo + wtile(K, J);
  for (int e = tid; e < WT2; e += 256) {
    ta[e / WT][e % WT] = li[e];
    tb[e / WT][e % WT] = lk[e];
  }
  __syncthreads();
  double acc[4];
  tile_abt(ta, tb, acc);
  double* dst = fo + wtile(I, K);
  const int r = tid >> 3, c0 = (tid & 7) * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) dst[r * WT + c0 + q] -= acc[q];
}

// ---------------------------------------------------------------------------
// Solves L L^T x = y for NR right-hand sides held in LDS (y[q][0 .. LP)),
// in place, by one workgroup: forward block rows J = 0 .. T-1 (r_J = y_J -
// sum_{I<J} L_JI y_I, y_J = Linv_J r_J), then backward (r_J = y_J -
// sum_{I>J} L_IJ^T x_I, x_J = Linv_J^T r_J).  The off-diagonal tiles of a
// block row are split over the four waves, each staging its tile in LDS.
// ---------------------------------------------------------------------------
template <int NR>
__device__ void wide_tri_solve(const double* __restrict__ fo, const WideShape& ws, double (*y)[WT * 24],
                               double (*tile)[WT][WT + 1], double (*red)[NR][WT], double (*rv)[WT]) {
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int pass = 0; pass < 2; ++pass) {
    const bool fwd = pass == 0;
    for (int step = 0; step < ws.T; ++step) {
      const int J = fwd ? step : ws.T - 1 - step;
      double acc[NR];
#pragma unroll
      for (int q = 0; q < NR; ++q) acc[q] = 0.0;
      // off-diagonal tiles: forward (J, I) for I < J, backward (I, J) for I > J
      const int i0 = fwd ? 0 : J + 1, i1 = fwd ? J : ws.T;
      for (int I = i0 + w; I < i1; I += 4) {
        const double* src = fo + (fwd ? wtile(J, I) : wtile(I, J));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int e = lane; e < WT2; e += 64) tile[w][e / WT][e % WT] = src[e];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < WT) {
          // forward: row `lane` of L_JI times y_I; backward: column `lane` of
          // L_IJ times x_I
#pragma unroll 4
          for (int m = 0; m < WT; ++m) {
            const double lv = fwd ? tile[w][lane][m] : tile[w][m][lane];
#pragma unroll
            for (int q = 0; q < NR; ++q) acc[q] = fma(lv, y[q][WT * I + m], acc[q]);
          }
        }
      }
      if (lane < WT) {
#pragma unroll
        for (int q = 0; q < NR; ++q) red[w][q][lane] = acc[q];
      }
      __syncthreads();
      if (tid < WT * NR) {
        const int q = tid / WT, r = tid % WT;
        rv[q][r] = y[q][WT * J + r] - (((red[0][q][r] + red[1][q][r]) + red[2][q][r]) + red[3][q][r]);
      }
      __syncthreads();
      // diagonal block: y_J = Linv_J r (forward), x_J = Linv_J^T r (backward)
      if (tid < WT * NR) {
        const int q = tid / WT, r = tid % WT;
        const double* inv = fo + winv(ws, J);
        double s = 0.0;
        for (int m = 0; m < WT; ++m) s = fma(fwd ? inv[r * WT + m] : inv[m * WT + r], rv[q][m], s);
        y[q][WT * J + r] = s;
      }
      __syncthreads();
    }
  }
}

// Entry i of the fixed probe vector `which` (0 or 1): +-1/sqrt(L), signs
// from an integer hash (deterministic), as the small-basis estimate.
__device__ __forceinline__ double wide_probe(int i, int which, int L) {
  uint32_t h = (uint32_t)i * 0x9E3779B1u + (uint32_t)which * 0x85EBCA77u + 0x165667B1u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  return ((h >> 7) & 1u ? 1.0 : -1.0) * rsqrt((double)L);
}

// ---------------------------------------------------------------------------
// Solve of every node of the level with its factor: b from the node's B,
// the coefficients, and (refine == 1) the condition estimate L max |A^-1 x|
// over the two probes; flags as the small-basis solve sets them.
// ---------------------------------------------------------------------------
template <int NR>
__global__ void __launch_bounds__(256) k_wide_solve(LevelArgs a, const double* __restrict__ part_m,
                                                    const double* __restrict__ fac, int L, int NM, int NOUT) {
  const WideShape ws = wide_shape(L);
  __shared__ double y[NR][WT * 24];
  __shared__ double tile[4][WT][WT + 1];
  __shared__ double red[4][NR][WT];
  __shared__ double rv[NR][WT];
  __shared__ int flags_sh;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const uint32_t k = blockIdx.x;
  const uint32_t node = a.node0 + k;
  const double* fo = fac + (size_t)k * ws.words;
  const double* bm = part_m + (size_t)a.chunk_off[k] * NOUT + NM;
  if (tid == 0) flags_sh = 0;
  for (int i = tid; i < ws.LP; i += 256) {
    y[0][i] = i < L ? bm[i] * fo[wweight(ws) + i] : 0.0;
    if (NR == 3) {
      y[1 % NR][i] = i < L ? wide_probe(i, 0, L) : 0.0;
      y[2 % NR][i] = i < L ? wide_probe(i, 1, L) : 0.0;
    }
  }
  __syncthreads();
  wide_tri_solve<NR>(fo, ws, y, tile, red, rv);
  bool bad = false, defl = false;
  double* coef = a.nt.coef + (size_t)node * L;
  for (int i = tid; i < L; i += 256) {
    const double c = fo[wscale(ws) + i] * y[0][i];
    coef[i] = c;
    bad |= !__builtin_isfinite(c);
    defl |= fo[wkept(ws) + i] == 0.0;
  }
  flag_nonfinite(bad, a.nt.flags + node, a.status);
  if (defl) atomicOr(&flags_sh, (int)FLAG_DEFLATED);
  if (NR == 3 && (w == 1 || w == 2)) {
    double ss = 0.0;
    for (int i = lane; i < L; i += 64) ss += y[w % NR][i] * y[w % NR][i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) ss += __shfl_xor(ss, off);
    if (lane == 0 && (double)L * sqrt(ss) > WIDE_REFINE_KAPPA) atomicOr(&flags_sh, (int)FLAG_REFINE);
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t f = (uint32_t)flags_sh;
    if (a.refine == 2) f |= FLAG_REFINE;
    else if (a.refine == 1 && (f & FLAG_DEFLATED)) f |= FLAG_REFINE;
    else if (a.refine == 0) f &= ~FLAG_REFINE;
    if (f) atomicOr(a.nt.flags + node, f);
  }
}

// ---------------------------------------------------------------------------
// Refinement: delta = A^-1 (W Lambda^T r') with the node's factor (B' of the
// node summed beforehand into its first chunk's slot), F += scale * delta.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_wide_refine_solve(LevelArgs a, const double* __restrict__ part_b,
                                                           const double* __restrict__ fac, int L) {
  const WideShape ws = wide_shape(L);
  __shared__ double y[1][WT * 24];
  __shared__ double tile[4][WT][WT + 1];
  __shared__ double red[4][1][WT];
  __shared__ double rv[1][WT];
  const int tid = threadIdx.x;
  const uint32_t k = blockIdx.x;
  const uint32_t node = a.node0 + k;
  if (!(a.nt.flags[node] & FLAG_REFINE)) return;   // whole workgroup: its node needs no refinement
  const double* fo = fac + (size_t)k * ws.words;
  const double* bm = part_b + (size_t)a.chunk_off[k] * L;
  for (int i = tid; i < ws.LP; i += 256) y[0][i] = i < L ? bm[i] * fo[wweight(ws) + i] : 0.0;
  __syncthreads();
  wide_tri_solve<1>(fo, ws, y, tile, red, rv);
  double* F = a.nt.coef + (size_t)node * L;
  bool bad = false;
  for (int i = tid; i < L; i += 256) {
    const double dl = fo[wscale(ws) + i] * y[0][i];
    const double c = F[i] + dl;
    F[i] = c;
    if (a.delta) a.delta[(size_t)k * L + i] = dl;
    bad |= !__builtin_isfinite(c);
  }
  flag_nonfinite(bad, a.nt.flags + node, a.status);
}

hipError_t launch_wide_factor(int p, const LevelArgs& a, const double* part_m, double* fac, hipStream_t s) {
  if (!wide_order(p)) return hipErrorInvalidValue;
  if (a.nnodes == 0) return hipSuccess;
  const int L = basis_size(p);
  const WideShape ws = wide_shape(L);
  const int NOUT = (int)moment_partial_doubles(p);
  hipLaunchKernelGGL(k_wide_assemble, dim3(a.nnodes, ws.T), dim3(256), 0, s, a, part_m, fac, L, NOUT);
  for (int J = 0; J < ws.T; ++J) {
    hipLaunchKernelGGL(k_wide_potrf, dim3(a.nnodes), dim3(256), 0, s, a, fac, L, J);
    const int below = ws.T - 1 - J;
    if (below == 0) break;
    hipLaunchKernelGGL(k_wide_trsm, dim3(a.nnodes, below), dim3(256), 0, s, a, fac, L, J);
    hipLaunchKernelGGL(k_wide_syrk, dim3(a.nnodes, below * (below + 1) / 2), dim3(256), 0, s, a, fac, L, J);
  }
  return hipGetLastError();
}

hipError_t launch_wide_solve(int p, const LevelArgs& a, const double* part_m, const double* fac, hipStream_t s) {
  if (!wide_order(p)) return hipErrorInvalidValue;
  if (a.nnodes == 0) return hipSuccess;
  const int L = basis_size(p), NM = basis_size(2 * p), NOUT = (int)moment_partial_doubles(p);
  if (a.refine == 1)
    hipLaunchKernelGGL(k_wide_solve<3>, dim3(a.nnodes), dim3(256), 0, s, a, part_m, fac, L, NM, NOUT);
  else
    hipLaunchKernelGGL(k_wide_solve<1>, dim3(a.nnodes), dim3(256), 0, s, a, part_m, fac, L, NM, NOUT);
  return hipGetLastError();
}

hipError_t launch_wide_refine_solve(int p, const LevelArgs& a, const double* part_b, const double* fac,
                                    hipStream_t s) {
  if (!wide_order(p)) return hipErrorInvalidValue;
  if (a.nnodes == 0) return hipSuccess;
  hipLaunchKernelGGL(k_wide_refine_solve, dim3(a.nnodes), dim3(256), 0, s, a, part_b, fac, basis_size(p));
  return hipGetLastError();
}

}  // namespace fmt
