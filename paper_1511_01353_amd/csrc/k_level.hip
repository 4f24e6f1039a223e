// Per-node solve, refinement, residual update and child activation of one
// octree level (Alg. 1 and Alg. 2), plus the topology step that lays out the
// next level's nodes.
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

size_t factor_doubles(int p) {
  const int L = basis_size(p);
  const int T = (L + 15) / 16;
  return (size_t)T * (T + 1) / 2 * 256 + 3 * (size_t)L;
}

// ---------------------------------------------------------------------------
// Right-looking blocked Cholesky of the unit-diagonal matrix A (blocked
// storage, padding rows/columns set to the identity), in place, by all 256
// threads.  Per block column J:
//   (a) wave 0 factors the diagonal block in registers (lane = column
//       c = lane % 16, rows lane / 16 + 4m), broadcasting pivots and column
//       values with lane shuffles;
//   (b) one thread per row below solves the panel row against L_JJ^T;
//   (c) the trailing blocks take A_IK -= L_IJ L_KJ^T on float64 MFMA.
// Deflated pivots (<= PIVOT_EPS) give a zero column; dg holds the diagonal
// of the factor and rdg its reciprocal (0 where deflated); both hold
// BlockShape<L>::LP entries (the padding pivots included).
// ---------------------------------------------------------------------------
template <int L>
__device__ void cholesky_blocked(double* A, double* dg, double* rdg) {
  using S = BlockShape<L>;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int J = 0; J < S::T; ++J) {
    // (a) diagonal block
    if (w == 0) {
      const int c = lane & 15, rg = lane >> 4;
      double* blk = A + bidx(J, J);
      double v[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int r = rg + 4 * m;
        v[m] = r >= c ? blk[bel(r, c)] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const double d = __shfl(v[k >> 2], 16 * (k & 3) + k);
        const bool ok = d > PIVOT_EPS;
        const double ld = ok ? sqrt(d) : 0.0;
        const double rl = ok ? 1.0 / ld : 0.0;
        if (c == k) {
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int r = rg + 4 * m;
            if (r > k) v[m] *= rl;
            else if (r == k) v[m] = ld;
          }
        }
        // L[r][k] for this lane's rows, and L[c][k] for its column
        double lrk[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) lrk[m] = __shfl(v[m], 16 * rg + k);
        const double t0 = __shfl(v[0], 16 * (c & 3) + k);
        const double t1 = __shfl(v[1], 16 * (c & 3) + k);
        const double t2 = __shfl(v[2], 16 * (c & 3) + k);
        const double t3 = __shfl(v[3], 16 * (c & 3) + k);
        const int cm = c >> 2;
        const double lck = cm == 0 ? t0 : (cm == 1 ? t1 : (cm == 2 ? t2 : t3));
        if (c > k) {
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int r = rg + 4 * m;
            if (r >= c) v[m] -= lrk[m] * lck;
          }
        }
        if (lane == k) {
          dg[16 * J + k] = ld;
          rdg[16 * J + k] = rl;
        }
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int r = rg + 4 * m;
        if (r >= c) blk[bel(r, c)] = v[m];
      }
    }
    __syncthreads();
    if (J + 1 == S::T) break;
    // (b) panel: rows i of blocks I > J, x = a L_JJ^{-T}
    {
      const int i = 16 * (J + 1) + tid;
      if (i < S::LP) {
        const double* ljj = A + bidx(J, J);
        double* row = A + bidx(i >> 4, J) + (i & 15) * 16;
        const int sw = (i & 15) >> 1;
        double x[16];
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) x[cc] = row[cc ^ sw];
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
          double t = x[cc];
#pragma unroll
          for (int m = 0; m < cc; ++m) t -= x[m] * ljj[bel(cc, m)];
          x[cc] = t * rdg[16 * J + cc];
        }
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) row[cc ^ sw] = x[cc];
      }
    }
    __syncthreads();
    // (c) trailing update A_IK -= L_IJ L_KJ^T for J < K <= I, on MFMA
    {
      const int nb = S::T - J - 1;
      const int npair = nb * (nb + 1) / 2;
      for (int pidx = w; pidx < npair; pidx += 4) {
        int rem = pidx, I = J + 1;
        while (rem > I - J - 1) { rem -= I - J; ++I; }
        const int K = J + 1 + rem;
        double* out = A + bidx(I, K);
        const double* li = A + bidx(I, J);
        const double* lk = A + bidx(K, J);
        solve_d4 acc;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = out[bel((lane >> 4) + 4 * q, lane & 15)];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int kk = 4 * s4 + (lane >> 4);
          const double av = -li[bel(lane & 15, kk)];
          const double bv = lk[bel(lane & 15, kk)];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) out[bel((lane >> 4) + 4 * q, lane & 15)] = acc[q];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// (L L^T) z = b with the blocked factor, run by wave 0 alone: lane l owns rows
// l, l+64, l+128 in registers; each step's value is broadcast from its owner
// lane; reciprocal pivots replace divisions.  Deflated pivots give 0.  The
// caller synchronises the workgroup before reading z.
// ---------------------------------------------------------------------------
template <int L>
__device__ void tri_solve_wave(const double* A, const double* rdg, const double* b, double* z) {
  constexpr int NS = (L + 63) / 64;
  const int lane = threadIdx.x & 63;
  double bb[NS], yy[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = lane + 64 * s;
    bb[s] = i < L ? b[i] : 0.0;
    yy[s] = 0.0;
  }
  // forward: L y = b
#pragma unroll
  for (int s0 = 0; s0 < NS; ++s0) {
    const int jn = (L - 64 * s0) < 64 ? (L - 64 * s0) : 64;
    for (int jj = 0; jj < jn; ++jj) {
      const int j = 64 * s0 + jj;
      const double yj = __shfl(bb[s0], jj) * rdg[j];
      if (lane == jj) yy[s0] = yj;
#pragma unroll
      for (int s = s0; s < NS; ++s) {
        const int i = lane + 64 * s;
        if (i > j && i < L) bb[s] -= A[belem(i, j)] * yj;
      }
    }
  }
  // backward: L^T z = y
  double zz[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) zz[s] = 0.0;
#pragma unroll
  for (int s0 = NS - 1; s0 >= 0; --s0) {
    const int jn = (L - 64 * s0) < 64 ? (L - 64 * s0) : 64;
    for (int jj = jn - 1; jj >= 0; --jj) {
      const int j = 64 * s0 + jj;
      const double zj = __shfl(yy[s0], jj) * rdg[j];
      if (lane == jj) zz[s0] = zj;
#pragma unroll
      for (int s = 0; s <= s0; ++s) {
        const int i = lane + 64 * s;
        if (i < j) yy[s] -= A[belem(j, i)] * zj;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = lane + 64 * s;
    if (i < L) z[i] = zz[s];
  }
}

// Factor, solve, write F and (optionally) the factor; shared tail of both
// K6 variants.  A holds the equilibrated matrix (blocked, padding = identity),
// b the scaled right-hand side, sc the equilibration scales.
template <int L>
__device__ __forceinline__ void factor_solve_store(double* A, double* b, double* z, double* dg, double* rdg,
                                                   const double* sc, const LevelArgs& a, uint32_t k, uint32_t node,
                                                   double* fac) {
  using S = BlockShape<L>;
  const int tid = threadIdx.x;
  cholesky_blocked<L>(A, dg, rdg);
  if (tid < 64) tri_solve_wave<L>(A, rdg, b, z);
  __syncthreads();
  double* F = a.nt.coef + (size_t)node * L;
  bool deflated = false;
  for (int i = tid; i < L; i += 256) {
    F[i] = sc[i] * z[i];
    if (dg[i] == 0.0) deflated = true;
  }
  if (fac) {
    double* fo = fac + (size_t)k * (S::WORDS + 3 * L);
    for (int e = tid; e < S::WORDS; e += 256) fo[e] = A[e];
    for (int i = tid; i < L; i += 256) {
      fo[S::WORDS + i] = dg[i];
      fo[S::WORDS + L + i] = rdg[i];
      fo[S::WORDS + 2 * L + i] = sc[i];
    }
  }
  if (deflated) atomicOr(a.nt.flags + node, FLAG_DEFLATED);
}

// Identity on the padding rows and columns [L, LP) of the blocked matrix.
template <int L>
__device__ __forceinline__ void pad_identity(double* A) {
  using S = BlockShape<L>;
  for (int i = L + threadIdx.x; i < S::LP; i += 256)
    for (int q = 0; q <= i; ++q) A[belem(i, q)] = q == i ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------
// K6 from Gram partials (the MFMA Gram layout: 16x16 blocks of the upper
// triangle of [Lambda | r]^T [Lambda | r]).  One workgroup per node.
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_solve(LevelArgs a, const double* __restrict__ partial,
                                               double* __restrict__ fac) {
  constexpr int L = basis_size(P);
  constexpr int TG = pad16(L + 1) / 16;
  constexpr int NPAIR = TG * (TG + 1) / 2;
  using S = BlockShape<L>;
  __shared__ double A[S::WORDS];
  __shared__ double b[L], z[L], dg[S::LP], rdg[S::LP], sc[L];   // pivots cover the padding too
  const int tid = threadIdx.x;
  const uint32_t k = blockIdx.x;
  const uint32_t node = a.node0 + k;
  const uint32_t c0 = a.chunk_off[k];   // chunks of the node were summed into this one
  const double* G = partial + (size_t)c0 * NPAIR * 256;
  // Gram element (i, j) of the augmented matrix, i <= j
  auto gram = [&](int i, int j) {
    const int t1 = i >> 4, t2 = j >> 4;
    const int pj = t1 * TG - t1 * (t1 - 1) / 2 + (t2 - t1);
    return G[(size_t)pj * 256 + (i & 15) * 16 + (j & 15)];
  };
  for (int i = tid; i < L; i += 256) {
    const double d = gram(i, i);
    sc[i] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  }
  __syncthreads();
  for (int i = tid; i < L; i += 256) {
    const double si = sc[i];
    for (int q = 0; q <= i; ++q) A[belem(i, q)] = gram(q, i) * si * sc[q];
    b[i] = gram(i, L) * si;
  }
  pad_identity<L>(A);
  __syncthreads();
  factor_solve_store<L>(A, b, z, dg, rdg, sc, a, k, node, fac);
}

// ---------------------------------------------------------------------------
// K6 from power moments: G_ik = M[alpha_i + alpha_k] / (alpha_i! alpha_k!),
// b_i = B[alpha_i] / alpha_i!.  Equilibration is folded into the assembly:
// with s_i = 1 / sqrt(G_ii) and w_i = s_i / alpha_i!, the scaled matrix is
// A_ik = M[alpha_i + alpha_k] w_i w_k and the scaled right-hand side
// B[alpha_i] w_i.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int graded(int a, int b, int c) {
  const int k = a + b + c;
  return k * (k + 1) * (k + 2) / 6 + (k - a) * (k - a + 1) / 2 + (k - a - b);
}

template <int P>
__global__ void __launch_bounds__(256) k_solve_m(LevelArgs a, const double* __restrict__ part,
                                                 double* __restrict__ fac) {
  constexpr int L = basis_size(P);
  constexpr int NM = basis_size(2 * P);
  constexpr int NOUT = NM + L + 1;
  constexpr Basis<P> B{};
  using S = BlockShape<L>;
  __shared__ double A[S::WORDS];
  __shared__ double mom[NOUT];
  __shared__ double b[L], z[L], dg[S::LP], rdg[S::LP], sc[L], wv[L];   // pivots cover the padding too
  __shared__ int ex[L][3];
  const int tid = threadIdx.x;
  const uint32_t k = blockIdx.x;
  const uint32_t node = a.node0 + k;
  const uint32_t c0 = a.chunk_off[k];   // chunks of the node were summed into this one
  for (int e = tid; e < NOUT; e += 256) mom[e] = part[(size_t)c0 * NOUT + e];
  for (int i = tid; i < L; i += 256) {
    ex[i][0] = B.lx[i];
    ex[i][1] = B.ly[i];
    ex[i][2] = B.lz[i];
  }
  __syncthreads();
  for (int i = tid; i < L; i += 256) {
    const double f = B.inv_fact[i];
    const double gii = mom[graded(2 * ex[i][0], 2 * ex[i][1], 2 * ex[i][2])] * f * f;
    const double s = gii > 0.0 ? 1.0 / sqrt(gii) : 0.0;
    sc[i] = s;
    wv[i] = s * f;
    b[i] = mom[NM + i] * s * f;
  }
  __syncthreads();
  for (int i = tid; i < L; i += 256) {
    const int xi = ex[i][0], yi = ex[i][1], zi = ex[i][2];
    const double wi = wv[i];
    for (int q = 0; q <= i; ++q)
      A[belem(i, q)] = mom[graded(xi + ex[q][0], yi + ex[q][1], zi + ex[q][2])] * wi * wv[q];
  }
  pad_identity<L>(A);
  __syncthreads();
  factor_solve_store<L>(A, b, z, dg, rdg, sc, a, k, node, fac);
}

// ---------------------------------------------------------------------------
// K7: refinement.  The sweep (power moments of r' = r - Lambda F, float64,
// in k_moments.hip) gives B'[alpha] = sum r' u^alpha per chunk; the solve
// takes delta = G^{-1} Lambda^T r' with the kept factor and sets F += delta.
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_refine_solve(LevelArgs a, const double* __restrict__ part_b,
                                                      const double* __restrict__ fac) {
  constexpr int L = basis_size(P);
  constexpr Basis<P> B{};
  using S = BlockShape<L>;
  __shared__ double A[S::WORDS];
  __shared__ double b[L], z[L], rdg[L], sc[L];
  const int tid = threadIdx.x;
  const uint32_t k = blockIdx.x;
  const uint32_t node = a.node0 + k;
  const uint32_t c0 = a.chunk_off[k];   // chunks of the node were summed into this one
  const double* fo = fac + (size_t)k * (S::WORDS + 3 * L);
  for (int e = tid; e < S::WORDS; e += 256) A[e] = fo[e];
  for (int i = tid; i < L; i += 256) {
    rdg[i] = fo[S::WORDS + L + i];
    sc[i] = fo[S::WORDS + 2 * L + i];
    b[i] = part_b[(size_t)c0 * L + i] * B.inv_fact[i] * fo[S::WORDS + 2 * L + i];
  }
  __syncthreads();
  if (tid < 64) tri_solve_wave<L>(A, rdg, b, z);
  __syncthreads();
  double* F = a.nt.coef + (size_t)node * L;
  for (int i = tid; i < L; i += 256) F[i] += sc[i] * z[i];
}

// ---------------------------------------------------------------------------
// K8: residual update r <- r - Lambda F (Alg. 2) and, per chunk, the sum of
// r^2 over each child octant (Alg. 1's E_RMS numerator), reduced in a fixed
// order so that results do not depend on scheduling.
// ---------------------------------------------------------------------------
template <int P, typename TIN>
__global__ void __launch_bounds__(256) k_residual(LevelArgs a, double* __restrict__ part_ss) {
  constexpr int L = basis_size(P);
  __shared__ double Fs[L];
  __shared__ double red[4][8];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const uint32_t g = blockIdx.x;
  const uint32_t k = chunk_node(a.chunk_off, a.nnodes, g);
  const uint32_t node = a.node0 + k;
  const uint32_t nb = a.nt.begin[node], nc = a.nt.count[node];
  const uint32_t start = nb + (g - a.chunk_off[k]) * CHUNK;
  const uint32_t end = min(nb + nc, start + (uint32_t)CHUNK);
  const double* geo = a.nt.geo + 6 * (size_t)node;
  const double cx = geo[0], cy = geo[1], cz = geo[2], sx = geo[3], sy = geo[4], sz = geo[5];
  for (int i = tid; i < L; i += 256) Fs[i] = a.nt.coef[(size_t)node * L + i];
  __syncthreads();
  const bool stats = a.level < a.D;
  const int shift = stats ? 3 * (a.D - a.level - 1) : 0;
  double ss[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) ss[q] = 0.0;
  for (uint32_t i = start + tid; i < end; i += 256) {
    double x, y, z;
    load_point<TIN>(a.px, a.py, a.pz, i, x, y, z);
    const double val = poly_eval<P, double>(Fs, (x - cx) * sx, (y - cy) * sy, (z - cz) * sz);
    const double rn = a.r[i] - val;
    a.r[i] = rn;
    const uint32_t o = (a.skey[i] >> shift) & 7u;
    const double r2 = rn * rn;
#pragma unroll
    for (int q = 0; q < 8; ++q) ss[q] += (o == (uint32_t)q) ? r2 : 0.0;
  }
  if (!stats) return;
  // fixed-order reduction: butterfly inside the wave, then waves in order
#pragma unroll
  for (int q = 0; q < 8; ++q) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) ss[q] += __shfl_xor(ss[q], off);
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) red[w][q] = ss[q];
  }
  __syncthreads();
  if (tid < 8) part_ss[(size_t)g * 8 + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

// ---------------------------------------------------------------------------
// Child activation (Alg. 1): octant o of a node at depth d becomes a node iff
// d + 1 <= D, n_o >= calL (tested first) and sqrt(sum r^2 / n_o) > tol.
// One thread per node.  Octant ranges come from binary searches of the sorted
// keys, so counts are exact integers.
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_children(LevelArgs a, const double* __restrict__ part_ss,
                                                  uint32_t* __restrict__ cbeg, uint32_t* __restrict__ ccnt,
                                                  uint32_t* __restrict__ nact) {
  constexpr uint32_t L = (uint32_t)basis_size(P);
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.nnodes) return;
  const uint32_t node = a.node0 + k;
  if (a.level >= a.D) {
    a.nt.child_mask[node] = 0;
    nact[k] = 0;
    return;
  }
  const uint32_t nb = a.nt.begin[node], ne = nb + a.nt.count[node];
  const uint64_t full = ((uint64_t)a.nt.problem[node] << (3 * a.level)) | a.nt.prefix[node];
  const int shift = 3 * (a.D - a.level - 1);
  uint32_t bnd[9];
  bnd[0] = nb;
  bnd[8] = ne;
  for (int o = 1; o < 8; ++o) {
    const uint64_t target = ((full << 3) | (uint64_t)o) << shift;
    uint32_t lo = bnd[o - 1], hi = ne;   // first position with key >= target
    while (lo < hi) {
      uint32_t mid = lo + ((hi - lo) >> 1);
      if ((uint64_t)a.skey[mid] < target) lo = mid + 1; else hi = mid;
    }
    bnd[o] = lo;
  }
  const uint32_t c0 = a.chunk_off[k];   // chunks of the node were summed into this one
  uint32_t mask = 0;
  for (int o = 0; o < 8; ++o) {
    const uint32_t n_o = bnd[o + 1] - bnd[o];
    cbeg[(size_t)k * 8 + o] = bnd[o];
    ccnt[(size_t)k * 8 + o] = n_o;
    if (n_o < L) continue;
    const double s = part_ss[(size_t)c0 * 8 + o];
    if (sqrt(s / (double)n_o) > a.tol) mask |= 1u << o;
  }
  a.nt.child_mask[node] = mask;
  nact[k] = (uint32_t)__popc(mask);
}

// Sum the per-chunk partials of every multi-chunk node into the node's first
// chunk slot (deterministic).  `width` doubles per chunk.  A workgroup covers
// 64 elements of one node with 4 lane groups; group q sums chunks q, q+4, ...
// and the four group sums are added in a fixed order.  Single-chunk nodes
// exit at once.
__global__ void __launch_bounds__(256) k_chunk_reduce(const uint32_t* __restrict__ chunk_off, uint32_t nnodes,
                                                      double* __restrict__ buf, uint32_t width, uint32_t eblocks) {
  __shared__ double part[4][64];
  const uint32_t k = blockIdx.x / eblocks;
  if (k >= nnodes) return;
  const uint32_t c0 = chunk_off[k], c1 = chunk_off[k + 1];
  if (c1 - c0 < 2) return;
  const uint32_t e = (blockIdx.x % eblocks) * 64 + (threadIdx.x & 63);
  const uint32_t q = threadIdx.x >> 6;
  double s = 0.0;
  if (e < width)
    for (uint32_t g = c0 + q; g < c1; g += 4) s += buf[(size_t)g * width + e];
  part[q][threadIdx.x & 63] = s;
  __syncthreads();
  if (q == 0 && e < width)
    buf[(size_t)c0 * width + e] = ((part[0][threadIdx.x] + part[1][threadIdx.x]) + part[2][threadIdx.x]) +
                                  part[3][threadIdx.x];
}

// Cell coordinates (i, j, k) of a Morton prefix with `level` triples.
__device__ __forceinline__ void decode_cell(uint32_t prefix, int level, uint32_t& ci, uint32_t& cj, uint32_t& ck) {
  ci = cj = ck = 0;
  for (int b = level - 1; b >= 0; --b) {
    const uint32_t t = (prefix >> (3 * b)) & 7u;
    ci = (ci << 1) | ((t >> 2) & 1u);
    cj = (cj << 1) | ((t >> 1) & 1u);
    ck = (ck << 1) | (t & 1u);
  }
}

// Centre and dilation of a node: h = (hi - lo) / 2^level, c = lo + (i + 1/2) h,
// u = (x - c) * (2 / h).  Separate roundings, no fused multiply-add.
__device__ __forceinline__ void node_geo(const ProblemParams& P, int level, uint32_t prefix, double* geo) {
  uint32_t c[3];
  decode_cell(prefix, level, c[0], c[1], c[2]);
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const double h = ldexp(__dsub_rn(P.hi[ax], P.lo[ax]), -level);
    geo[ax] = __dadd_rn(P.lo[ax], __dmul_rn((double)c[ax] + 0.5, h));
    geo[3 + ax] = __ddiv_rn(2.0, h);
  }
}

__global__ void k_roots(NodeTable nt, const ProblemParams* __restrict__ prm, int nprob) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nprob) return;
  nt.begin[k] = prm[k].offset;
  nt.count[k] = prm[k].n;
  nt.prefix[k] = 0;
  nt.level[k] = 0;
  nt.problem[k] = (uint32_t)k;
  nt.parent[k] = (uint32_t)k;
  nt.first_child[k] = 0;
  nt.child_mask[k] = 0;
  nt.flags[k] = 0;
  node_geo(prm[k], 0, 0u, nt.geo + 6 * (size_t)k);
}

// Geometry of nodes given (level, prefix, problem), e.g. after an import.
__global__ void k_node_geo(NodeTable nt, const ProblemParams* __restrict__ prm, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  node_geo(prm[nt.problem[i]], (int)nt.level[i], nt.prefix[i], nt.geo + 6 * (size_t)i);
}

// Lay out the next level: child ids in (parent, octant) order, their fields,
// and the next level's chunk offsets.  One workgroup of 1024 threads; each
// thread owns a contiguous run of parents.
__global__ void __launch_bounds__(1024) k_emit(LevelArgs a, const ProblemParams* __restrict__ prm,
                                               const uint32_t* __restrict__ cbeg, const uint32_t* __restrict__ ccnt,
                                               uint32_t* __restrict__ nact, uint32_t next0,
                                               uint32_t* __restrict__ next_chunk_off,
                                               uint32_t* __restrict__ counters) {
  __shared__ uint32_t s[1024];
  const uint32_t tid = threadIdx.x;
  const uint32_t m = a.nnodes;
  const uint32_t seg = (m + 1023u) / 1024u;
  const uint32_t b = min(m, tid * seg), e = min(m, b + seg);
  uint32_t sum = 0;
  for (uint32_t i = b; i < e; ++i) sum += nact[i];
  s[tid] = sum;
  __syncthreads();
  for (uint32_t off = 1; off < 1024; off <<= 1) {
    uint32_t v = tid >= off ? s[tid - off] : 0u;
    __syncthreads();
    s[tid] += v;
    __syncthreads();
  }
  const uint32_t total = s[1023];
  uint32_t run = s[tid] - sum;
  uint32_t pts = 0;
  for (uint32_t i = b; i < e; ++i) {
    const uint32_t node = a.node0 + i;
    const uint32_t mask = a.nt.child_mask[node];
    if (mask) a.nt.first_child[node] = next0 + run;
    const uint32_t prob = a.nt.problem[node];
    const uint32_t pre = a.nt.prefix[node];
    for (int o = 0; o < 8; ++o) {
      if (!((mask >> o) & 1u)) continue;
      const uint32_t cid = next0 + run;
      const uint32_t cpre = (pre << 3) | (uint32_t)o;
      a.nt.begin[cid] = cbeg[(size_t)i * 8 + o];
      const uint32_t cn = ccnt[(size_t)i * 8 + o];
      a.nt.count[cid] = cn;
      a.nt.prefix[cid] = cpre;
      a.nt.level[cid] = (uint32_t)(a.level + 1);
      a.nt.problem[cid] = prob;
      a.nt.parent[cid] = node;
      a.nt.first_child[cid] = 0;
      a.nt.child_mask[cid] = 0;
      a.nt.flags[cid] = 0;
      node_geo(prm[prob], a.level + 1, cpre, a.nt.geo + 6 * (size_t)cid);
      next_chunk_off[run] = (cn + CHUNK - 1) / CHUNK;
      pts += cn;
      ++run;
    }
  }
  __syncthreads();
  // total points of the next level (fixed-order integer sum)
  s[tid] = pts;
  __syncthreads();
  for (uint32_t off = 512; off >= 1; off >>= 1) {
    if (tid < off) s[tid] += s[tid + off];
    __syncthreads();
  }
  const uint32_t next_points = s[0];
  __syncthreads();
  // exclusive scan of the children's chunk counts
  const uint32_t seg2 = (total + 1023u) / 1024u;
  const uint32_t b2 = min(total, tid * seg2), e2 = min(total, b2 + seg2);
  uint32_t sum2 = 0;
  for (uint32_t i = b2; i < e2; ++i) sum2 += next_chunk_off[i];
  __syncthreads();
  s[tid] = sum2;
  __syncthreads();
  for (uint32_t off = 1; off < 1024; off <<= 1) {
    uint32_t v = tid >= off ? s[tid - off] : 0u;
    __syncthreads();
    s[tid] += v;
    __syncthreads();
  }
  uint32_t run2 = s[tid] - sum2;
  for (uint32_t i = b2; i < e2; ++i) {
    const uint32_t v = next_chunk_off[i];
    next_chunk_off[i] = run2;
    run2 += v;
  }
  if (tid == 1023) {
    next_chunk_off[total] = s[1023];
    counters[0] = total;
    counters[1] = s[1023];
    counters[2] = next_points;
  }
}

template <int P>
__global__ void k_check_coef(NodeTable nt, uint32_t nnodes, uint32_t* status) {
  constexpr int L = basis_size(P);
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnodes) return;
  bool bad = false;
  for (int i = 0; i < L; ++i) {
    const double c = nt.coef[(size_t)k * L + i];
    if (!(c - c == 0.0)) bad = true;
  }
  if (bad) {
    atomicOr(nt.flags + k, FLAG_NONFINITE);
    atomicOr(status, 2u);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int P>
static hipError_t solve_impl(const LevelArgs& a, const double* partial, double* fac, hipStream_t s) {
  if (a.nnodes == 0) return hipSuccess;
  hipLaunchKernelGGL(k_solve<P>, dim3(a.nnodes), dim3(256), 0, s, a, partial, fac);
  return hipGetLastError();
}
hipError_t launch_solve(int p, const LevelArgs& a, const double* partial, double* fac, hipStream_t s) {
  FMT_DISPATCH_P(p, solve_impl, a, partial, fac, s);
}

template <int P>
static hipError_t solve_m_impl(const LevelArgs& a, const double* part, double* fac, hipStream_t s) {
  if (a.nnodes == 0) return hipSuccess;
  hipLaunchKernelGGL(k_solve_m<P>, dim3(a.nnodes), dim3(256), 0, s, a, part, fac);
  return hipGetLastError();
}
hipError_t launch_solve_moments(int p, const LevelArgs& a, const double* part, double* fac, hipStream_t s) {
  FMT_DISPATCH_P(p, solve_m_impl, a, part, fac, s);
}

template <int P>
static hipError_t rsolve_impl(const LevelArgs& a, const double* part_b, const double* fac, hipStream_t s) {
  if (a.nnodes == 0) return hipSuccess;
  hipLaunchKernelGGL(k_refine_solve<P>, dim3(a.nnodes), dim3(256), 0, s, a, part_b, fac);
  return hipGetLastError();
}
hipError_t launch_refine_solve(int p, const LevelArgs& a, const double* part_b, const double* fac, hipStream_t s) {
  FMT_DISPATCH_P(p, rsolve_impl, a, part_b, fac, s);
}

template <int P>
static hipError_t resid_impl(int dtype, const LevelArgs& a, double* part_ss, hipStream_t s) {
  if (a.nchunks == 0) return hipSuccess;
  if (dtype == FMT_F32) hipLaunchKernelGGL((k_residual<P, float>), dim3(a.nchunks), dim3(256), 0, s, a, part_ss);
  else hipLaunchKernelGGL((k_residual<P, double>), dim3(a.nchunks), dim3(256), 0, s, a, part_ss);
  return hipGetLastError();
}
hipError_t launch_residual(int p, int dtype, const LevelArgs& a, double* part_ss, hipStream_t s) {
  FMT_DISPATCH_P(p, resid_impl, dtype, a, part_ss, s);
}

template <int P>
static hipError_t children_impl(const LevelArgs& a, const double* part_ss, uint32_t* cbeg, uint32_t* ccnt,
                                uint32_t* nact, hipStream_t s) {
  if (a.nnodes == 0) return hipSuccess;
  hipLaunchKernelGGL(k_children<P>, dim3((a.nnodes + 255) / 256), dim3(256), 0, s, a, part_ss, cbeg, ccnt, nact);
  return hipGetLastError();
}
hipError_t launch_children(int p, const LevelArgs& a, const double* part_ss, uint32_t* cbeg, uint32_t* ccnt,
                           uint32_t* nact, hipStream_t s) {
  FMT_DISPATCH_P(p, children_impl, a, part_ss, cbeg, ccnt, nact, s);
}

hipError_t launch_emit(const LevelArgs& a, const ProblemParams* prm, const uint32_t* cbeg, const uint32_t* ccnt,
                       uint32_t* nact, uint32_t next0, uint32_t* next_chunk_off, uint32_t* counters, hipStream_t s) {
  hipLaunchKernelGGL(k_emit, dim3(1), dim3(1024), 0, s, a, prm, cbeg, ccnt, nact, next0, next_chunk_off, counters);
  return hipGetLastError();
}

hipError_t launch_chunk_reduce(const LevelArgs& a, double* buf, uint32_t width, hipStream_t s) {
  if (a.nnodes == 0 || a.nchunks <= a.nnodes) return hipSuccess;
  const uint32_t eblocks = (width + 63) / 64;
  hipLaunchKernelGGL(k_chunk_reduce, dim3(a.nnodes * eblocks), dim3(256), 0, s, a.chunk_off, a.nnodes, buf, width,
                     eblocks);
  return hipGetLastError();
}

hipError_t launch_node_geo(const NodeTable& nt, const ProblemParams* prm, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_node_geo, dim3((n + 255) / 256), dim3(256), 0, s, nt, prm, n);
  return hipGetLastError();
}

hipError_t launch_roots(const NodeTable& nt, const ProblemParams* prm, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(k_roots, dim3((nprob + 255) / 256), dim3(256), 0, s, nt, prm, nprob);
  return hipGetLastError();
}

template <int P>
static hipError_t check_impl(const NodeTable& nt, uint32_t nnodes, uint32_t* status, hipStream_t s) {
  if (nnodes == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_coef<P>, dim3((nnodes + 255) / 256), dim3(256), 0, s, nt, nnodes, status);
  return hipGetLastError();
}
hipError_t launch_check_coef(int p, const NodeTable& nt, uint32_t nnodes, uint32_t* status, hipStream_t s) {
  FMT_DISPATCH_P(p, check_impl, nt, nnodes, status, s);
}

}  // namespace fmt
