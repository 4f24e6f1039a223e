// K9: evaluation of a fitted tree at query points.
//
// Section 2 evaluates a fit as f'_q = Lambda'_q . F_p (no need to form the
// transform matrix).  The octree fit is a residual decomposition (Alg. 1), so
// the value at a query is the sum of the polynomials of every node on its
// root-to-leaf chain.  That sum is itself a polynomial of degree <= p in the
// frame of the deepest node reached, so it is formed once per node
// (k_compose) and a query then evaluates a single polynomial.
#include "k_level.h"

namespace fmt {

// ---------------------------------------------------------------------------
// Composite coefficients.  A child's frame relates to its parent's by
// u_parent = (u_child + sigma) / 2 on each axis (sigma = +1 for the upper
// half of the parent cell, -1 for the lower), so one scaled monomial
// re-expands as
//   u_p^l / l! = sum_{k <= l} (u_c^k / k!) sigma^(l-k) / (2^l (l-k)!),
// applied axis by axis: a node's composite is its parent's composite shifted
// into its frame plus its own polynomial (a root's is its own).  One wave per
// node, four nodes per workgroup, all levels in one launch: each wave walks
// its node's chain from the root down, shifting and adding level by level,
// so no node waits for another's result (the same operations, in the same
// order, as composing level by level).
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_compose(NodeTable nt, uint32_t first, uint32_t count,
                                                 double* __restrict__ cc) {
  constexpr int L = basis_size(P);
  constexpr int CS = ccoef_stride(L);
  constexpr Basis<P> B{};
  __shared__ double buf[4][2][L];
  __shared__ int ex[L][3];
  __shared__ uint32_t chain[4][FMT_MAX_LEVELS];
  __shared__ double invf[P + 1];   // 1 / m!
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int i = tid; i < L; i += 256) {
    ex[i][0] = B.lx[i];
    ex[i][1] = B.ly[i];
    ex[i][2] = B.lz[i];
  }
  if (tid <= P) {
    double f = 1.0;
    for (int m = 2; m <= tid; ++m) f *= (double)m;   // exact: m! < 2^53 for m <= 18
    invf[tid] = 1.0 / f;
  }
  __syncthreads();
  const uint32_t k = blockIdx.x * 4 + (uint32_t)w;
  if (k >= count) return;   // the whole wave leaves; no workgroup barrier follows
  const uint32_t v = first + k;
  const int depth = (int)nt.level[v];
  if (lane == 0) {
    // chain[w][d] = the ancestor of v at level d (v itself at its level)
    uint32_t u = v;
    for (int d = depth; d >= 0; --d) {
      chain[w][d] = u;
      if (d > 0) u = nt.parent[u];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double* cur = buf[w][0];
  double* nxt = buf[w][1];
  constexpr int QL = (L + 63) / 64;
  double own[QL];
  {
    const double* F = nt.coef + (size_t)chain[w][0] * L;
#pragma unroll
    for (int q = 0; q < QL; ++q) own[q] = lane + 64 * q < L ? F[lane + 64 * q] : 0.0;
  }
  for (int d = 1; d <= depth; ++d) {
    // own holds the composite of the level d-1 ancestor; shift it into the
    // frame of the level d ancestor a and add a's own polynomial
    const uint32_t a = chain[w][d];
    const uint32_t o = nt.prefix[a] & 7u;
    const double* F = nt.coef + (size_t)a * L;
#pragma unroll
    for (int q = 0; q < QL; ++q)
      if (lane + 64 * q < L) cur[lane + 64 * q] = own[q];
#pragma unroll
    for (int q = 0; q < QL; ++q) own[q] = lane + 64 * q < L ? F[lane + 64 * q] : 0.0;
#pragma unroll
    for (int axis = 0; axis < 3; ++axis) {
      const double sg = ((o >> (2 - axis)) & 1u) ? 1.0 : -1.0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int e = lane; e < L; e += 64) {
        int xyz[3] = {ex[e][0], ex[e][1], ex[e][2]};
        const int kk = xyz[axis];
        const int top = P - (xyz[0] + xyz[1] + xyz[2] - kk);
        double sum = 0.0;
        for (int l = kk; l <= top; ++l) {
          // sigma^(l-kk) / (2^l (l-kk)!): a table entry, an exact power of
          // two and a sign (no division in the loop)
          const int m = l - kk;
          const double t = ldexp((sg < 0.0 && (m & 1)) ? -invf[m] : invf[m], -l);
          xyz[axis] = l;
          sum = fma(cur[graded(xyz[0], xyz[1], xyz[2])], t, sum);
        }
        nxt[e] = sum;
      }
      double* tmp = cur;
      cur = nxt;
      nxt = tmp;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int q = 0; q < QL; ++q)
      if (lane + 64 * q < L) own[q] += cur[lane + 64 * q];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
#pragma unroll
  for (int q = 0; q < (CS + 63) / 64; ++q) {
    const int e = lane + 64 * q;
    if (e < CS) cc[(size_t)v * CS + e] = e < L ? own[q] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Cell table: for every cell of depth T, the deepest node (level <= T) whose
// cell contains it, found by walking down from the root.  One thread per
// cell.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_cell_table(NodeTable nt, uint32_t root, int T, ProblemParams prm,
                                                   double* __restrict__ lvl, uint32_t* __restrict__ cells) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c <= (uint32_t)FMT_MAX_DEPTH) {
    // frame of level c: h = (hi - lo) / 2^c, 2 / h (as the fit's node frames)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double h = ldexp(__dsub_rn(prm.hi[a], prm.lo[a]), -(int)c);
      lvl[6 * c + a] = h;
      lvl[6 * c + 3 + a] = __ddiv_rn(2.0, h);
    }
  }
  if (c >= (1u << (3 * T))) return;
  uint32_t node = root;
  int d = 0;
  for (; d < T; ++d) {
    const uint32_t m = nt.child_mask[node];
    const uint32_t o = (c >> (3 * (T - d - 1))) & 7u;
    if (!((m >> o) & 1u)) break;
    node = nt.first_child[node] + (uint32_t)__popc(m & ((1u << o) - 1u));
  }
  cells[c] = node | ((uint32_t)d << 28);
}

// Bits 3b + shift of v gathered into bit b (inverse of spread3).
__device__ __forceinline__ uint32_t compact3(uint32_t v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030C30C3u;
  v = (v | (v >> 4)) & 0x0300F00Fu;
  v = (v | (v >> 8)) & 0x030000FFu;
  v = (v | (v >> 16)) & 0x000003FFu;
  return v;
}

// ---------------------------------------------------------------------------
// One query per thread: the cell table gives the deepest node down to depth
// T, the walk continues below T while the child holding the query's cell
// exists (integer loads only), and the composite polynomial of the node
// reached is evaluated.  The node's frame follows from its level and the
// query's cell, exactly as the fit computes it, so no geometry is loaded.
// In sorted mode the coordinates arrive in key order (moved by the sort),
// skeys holds their keys and perm their positions in the caller's order,
// where the result is written.
// Coefficient rows: a wave whose queries all reach one node reads the row
// with wave-uniform (scalar) loads.  Otherwise the rows come through LDS in
// two rounds of 32 queries, each round loaded as two batches of 16: the 4
// lanes of a quad load one query's row together (each instruction reads 64
// contiguous bytes, half of one 128-byte line, per query, instead of one
// line per lane), and the query's own lane evaluates it.  One wave per
// workgroup; a round's 32 rows take 22 KB of LDS at p = 6.
// ---------------------------------------------------------------------------
constexpr int EVAL_THREADS = 64;

// Row staging of order P: lanes per row (each lane loads every G-th double
// pair of the row) and rows per batch; small bases stage two batches of 16
// rows per round (4 lanes a row), the large ones (p = 10..14, rows of up to
// 5.4 KB) one batch of 8 rows (8 lanes a row), so a round stays within 48 KB
// of LDS.
template <int P>
struct EvalStage {
  static constexpr bool WIDE = P > 8;
  static constexpr int G = WIDE ? 8 : 4;          // lanes per row
  static constexpr int BATCH = 64 / G;            // rows per batch
  static constexpr int NB = WIDE ? 1 : 2;         // batches per round
  static constexpr int ROWS = BATCH * NB;         // rows per round
};

template <int P, typename TIN>
__global__ void __launch_bounds__(EVAL_THREADS) k_eval(EvalTree t, const double* __restrict__ cc,
                                                       const TIN* __restrict__ qx, const TIN* __restrict__ qy,
                                                       const TIN* __restrict__ qz, const uint32_t* __restrict__ perm,
                                                       const uint32_t* __restrict__ skeys, uint32_t nq,
                                                       double* __restrict__ out) {
  constexpr int L = basis_size(P);
  constexpr int CS = ccoef_stride(L);
  constexpr int UP = (L + 1) / 2;   // double pairs of a row that hold coefficients
  // LDS row stride (doubles): rows 16-byte aligned, and LS = 2 mod 4 so that
  // 16 lanes reading the same coefficient of 16 rows with 16-byte loads hit
  // 16 distinct groups of four banks
  constexpr int LS = 2 * UP + ((2 * UP) % 4 == 0 ? 2 : 0);
  using ES = EvalStage<P>;
  constexpr int EVAL_ROWS = ES::ROWS;
  static_assert(EVAL_THREADS == 64, "one wave per workgroup");
  __shared__ __attribute__((aligned(16))) double rows[EVAL_ROWS * LS];
  const uint32_t i0 = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = i0 < nq;
  const uint32_t i = valid ? i0 : nq - 1;   // tail lanes repeat the last query and do not store
  const uint32_t src = perm ? perm[i] : i;   // caller's position of query i
  const double x = (double)qx[i], y = (double)qy[i], z = (double)qz[i];
  uint32_t key;
  if (skeys) {
    key = skeys[i];
  } else {
    bool bad = false;
    const uint32_t cmax = (1u << t.D) - 1u;
    key = (spread3(cell_of(x, t.prm.lo[0], t.prm.qscale[0], cmax, &bad)) << 2) |
          (spread3(cell_of(y, t.prm.lo[1], t.prm.qscale[1], cmax, &bad)) << 1) |
          spread3(cell_of(z, t.prm.lo[2], t.prm.qscale[2], cmax, &bad));
  }
  const uint32_t e = t.cells[key >> (3 * (t.D - t.T))];
  uint32_t node = e & 0x0fffffffu;
  int d = (int)(e >> 28);
  if (d == t.T) {
    for (; d < t.D; ++d) {
      const uint32_t m = t.nt.child_mask[node];
      const uint32_t o = (key >> (3 * (t.D - d - 1))) & 7u;
      if (!((m >> o) & 1u)) break;
      node = t.nt.first_child[node] + (uint32_t)__popc(m & ((1u << o) - 1u));
    }
  }
  // frame of the node reached: its cell is the query's cell at level d
  const uint32_t cell = d > 0 ? key >> (3 * (t.D - d)) : 0u;
  const uint32_t ci = compact3(cell >> 2), cj = compact3(cell >> 1), ck = compact3(cell);
  const double* fr = t.lvl + 6 * d;
  const double u = (x - __dadd_rn(t.prm.lo[0], __dmul_rn((double)ci + 0.5, fr[0]))) * fr[3];
  const double v = (y - __dadd_rn(t.prm.lo[1], __dmul_rn((double)cj + 0.5, fr[1]))) * fr[4];
  const double ww = (z - __dadd_rn(t.prm.lo[2], __dmul_rn((double)ck + 0.5, fr[2]))) * fr[5];
  const uint32_t n0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)node);
  double val = 0.0;
  if (__ballot(node != n0) == 0) {
    // read-only constant address space + a wave-uniform address: scalar loads
    typedef const double __attribute__((address_space(4))) cdouble;
    val = poly_eval<P, double>((const cdouble*)(cc + (size_t)n0 * CS), u, v, ww);
  } else {
    constexpr int G = ES::G, BATCH = ES::BATCH, NB = ES::NB;
    constexpr int KS = (UP + G - 1) / G;   // loads per lane per batch
    const int qg = lane / G, part = lane % G;
#pragma unroll 1
    for (int r = 0; r < 64 / EVAL_ROWS; ++r) {
      double2 vals[NB][KS];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        // the group's query: lane EVAL_ROWS r + BATCH b + qg, its row to LDS row BATCH b + qg
        const uint32_t nd = (uint32_t)__shfl((int)node, EVAL_ROWS * r + BATCH * b + qg);
        const double2* srow = reinterpret_cast<const double2*>(cc + (size_t)nd * CS);
#pragma unroll
        for (int k = 0; k < KS; ++k) {
          const int pr = G * k + part;
          vals[b][k] = pr < UP ? srow[pr] : make_double2(0.0, 0.0);
        }
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        double2* drow = reinterpret_cast<double2*>(rows + (BATCH * b + qg) * LS);
#pragma unroll
        for (int k = 0; k < KS; ++k) {
          const int pr = G * k + part;
          if (pr < UP) drow[pr] = vals[b][k];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (lane / EVAL_ROWS == r) val = poly_eval<P, double>(rows + (lane % EVAL_ROWS) * LS, u, v, ww);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  if (valid) out[src] = val;
}

template <int P>
static hipError_t compose_impl(const NodeTable& nt, uint32_t first, uint32_t count, double* cc, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_compose<P>, dim3((count + 3) / 4), dim3(256), 0, s, nt, first, count, cc);
  return hipGetLastError();
}

hipError_t launch_compose(int p, const NodeTable& nt, uint32_t first, uint32_t count, double* cc, hipStream_t s) {
  FMT_DISPATCH_P_ALL(p, compose_impl, nt, first, count, cc, s);
}

hipError_t launch_cell_table(const NodeTable& nt, uint32_t root, int T, const ProblemParams& prm, double* lvl,
                             uint32_t* cells, hipStream_t s) {
  const uint32_t n = 1u << (3 * T);
  const uint32_t threads = n > (uint32_t)FMT_MAX_DEPTH + 1 ? n : (uint32_t)FMT_MAX_DEPTH + 1;
  hipLaunchKernelGGL(k_cell_table, dim3((threads + 255) / 256), dim3(256), 0, s, nt, root, T, prm, lvl, cells);
  return hipGetLastError();
}

template <int P>
static hipError_t eval_impl(int dtype, const EvalTree& t, const double* cc, const void* qx, const void* qy,
                            const void* qz, const uint32_t* perm, const uint32_t* skeys, uint32_t nq, double* out,
                            hipStream_t s) {
  if (nq == 0) return hipSuccess;
  dim3 grid((nq + EVAL_THREADS - 1) / EVAL_THREADS), block(EVAL_THREADS);
  if (dtype == FMT_F32)
    hipLaunchKernelGGL((k_eval<P, float>), grid, block, 0, s, t, cc, (const float*)qx, (const float*)qy,
                       (const float*)qz, perm, skeys, nq, out);
  else
    hipLaunchKernelGGL((k_eval<P, double>), grid, block, 0, s, t, cc, (const double*)qx, (const double*)qy,
                       (const double*)qz, perm, skeys, nq, out);
  return hipGetLastError();
}

hipError_t launch_eval(int p, int dtype, const EvalTree& t, const double* cc, const void* qx, const void* qy,
                       const void* qz, const uint32_t* perm, const uint32_t* skeys, uint32_t nq, double* out,
                       hipStream_t s) {
  FMT_DISPATCH_P_ALL(p, eval_impl, dtype, t, cc, qx, qy, qz, perm, skeys, nq, out, s);
}

}  // namespace fmt
