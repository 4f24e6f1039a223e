// Per-node solve, refinement, residual update and child activation of one
// octree level (Alg. 1 and Alg. 2), plus the topology step that lays out the
// next level's nodes.
#include "k_level.h"

namespace fmt {

// packed lower triangle: element (i, k), k <= i
__device__ __forceinline__ int pk(int i, int k) { return i * (i + 1) / 2 + k; }

size_t factor_doubles(int p) {
  const size_t L = (size_t)basis_size(p);
  return L * (L + 1) / 2 + 2 * L;
}

// Pivots of the equilibrated Gram (unit diagonal) at or below this are
// treated as linear dependence: the column is dropped from the factor.
constexpr double PIVOT_EPS = 1e-13;

// ---------------------------------------------------------------------------
// Triangular solves with a packed factor; one workgroup, one sync per step.
// b: scaled right-hand side (destroyed); z: solution of (L L^T) z = b.
// ---------------------------------------------------------------------------
template <int L>
__device__ void tri_solve(const double* A, const double* diagL, double* b, double* y, double* z) {
  const int tid = threadIdx.x;
  for (int j = 0; j < L; ++j) {
    const double dj = diagL[j];
    const double yj = dj > 0.0 ? b[j] / dj : 0.0;
    const int i = j + 1 + tid;
    if (i < L) b[i] -= A[pk(i, j)] * yj;
    if (tid == 0) y[j] = yj;
    __syncthreads();
  }
  for (int j = L - 1; j >= 0; --j) {
    const double dj = diagL[j];
    const double zj = dj > 0.0 ? y[j] / dj : 0.0;
    if (tid < j) y[tid] -= A[pk(j, tid)] * zj;
    if (tid == 0) z[j] = zj;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// K6: sum a node's chunk partials, equilibrate, Cholesky, solve for F.
// One workgroup per node.  The factor is kept for the refinement sweeps.
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_solve(LevelArgs a, const double* __restrict__ partial,
                                               double* __restrict__ fac) {
  constexpr int L = basis_size(P);
  constexpr int T = pad16(L + 1) / 16;
  constexpr int NPAIR = T * (T + 1) / 2;
  constexpr int NPK = L * (L + 1) / 2;
  __shared__ double A[NPK];
  __shared__ double b[L], y[L], z[L], dg[L], sc[L];
  const int tid = threadIdx.x;
  const uint32_t k = blockIdx.x;
  const uint32_t node = a.node0 + k;
  const uint32_t c0 = a.chunk_off[k], c1 = a.chunk_off[k + 1];

  // assemble: packed lower triangle of Lambda^T Lambda, then Lambda^T r
  for (int e = tid; e < NPK + L; e += 256) {
    int i, kk;
    if (e < NPK) {
      i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      while (pk(i + 1, 0) <= e) ++i;
      while (pk(i, 0) > e) --i;
      kk = e - pk(i, 0);
    } else {
      i = e - NPK;
      kk = L;
    }
    const int lo = i < kk ? i : kk, hi = i < kk ? kk : i;
    const int t1 = lo >> 4, t2 = hi >> 4;
    const int j = t1 * T - t1 * (t1 - 1) / 2 + (t2 - t1);
    const size_t off = (size_t)j * 256 + (lo & 15) * 16 + (hi & 15);
    double s = 0.0;
    for (uint32_t g = c0; g < c1; ++g) s += partial[(size_t)g * NPAIR * 256 + off];
    if (e < NPK) A[e] = s; else b[i] = s;
  }
  __syncthreads();
  // equilibrate to a unit diagonal
  for (int i = tid; i < L; i += 256) {
    const double d = A[pk(i, i)];
    sc[i] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < NPK; e += 256) {
    int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (pk(i + 1, 0) <= e) ++i;
    while (pk(i, 0) > e) --i;
    A[e] *= sc[i] * sc[e - pk(i, 0)];
  }
  for (int i = tid; i < L; i += 256) b[i] *= sc[i];
  __syncthreads();
  // left-looking Cholesky in place; thread t owns row j + t at step j
  for (int j = 0; j < L; ++j) {
    const int i = j + tid;
    if (i < L) {
      double t = A[pk(i, j)];
      const double* ri = A + pk(i, 0);
      const double* rj = A + pk(j, 0);
      for (int q = 0; q < j; ++q) t -= ri[q] * rj[q];
      A[pk(i, j)] = t;
    }
    __syncthreads();
    const double d = A[pk(j, j)];
    const bool ok = d > PIVOT_EPS;
    const double lj = ok ? sqrt(d) : 0.0;
    if (i < L && i > j) A[pk(i, j)] = ok ? A[pk(i, j)] / lj : 0.0;
    if (tid == 0) dg[j] = lj;
    __syncthreads();
  }
  tri_solve<L>(A, dg, b, y, z);
  double* F = a.nt.coef + (size_t)node * L;
  bool deflated = false;
  for (int i = tid; i < L; i += 256) {
    F[i] = sc[i] * z[i];
    if (dg[i] == 0.0) deflated = true;
  }
  if (fac) {
    double* fo = fac + (size_t)k * (NPK + 2 * L);
    for (int e = tid; e < NPK; e += 256) fo[e] = A[e];
    for (int i = tid; i < L; i += 256) {
      fo[NPK + i] = dg[i];
      fo[NPK + L + i] = sc[i];
    }
  }
  if (deflated) atomicOr(a.nt.flags + node, FLAG_DEFLATED);
}

// ---------------------------------------------------------------------------
// K7: refinement.  Sweep: per chunk, r' = r - Lambda F and Lambda^T r' in
// float64.  Solve: delta = G^{-1} (sum of chunk parts) with the kept factor,
// F += delta.
// ---------------------------------------------------------------------------
template <int P, typename TIN>
__global__ void __launch_bounds__(256) k_refine_sweep(LevelArgs a, double* __restrict__ part_b) {
  constexpr int L = basis_size(P);
  constexpr int PB = 64, PS = PB + 4;
  __shared__ double tile[L * PS];
  __shared__ double Fs[L];
  __shared__ double rp[PB];
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
  constexpr Basis<P> B{};
  double acc = 0.0;
  for (uint32_t bs = start; bs < end; bs += PB) {
    const uint32_t pt = bs + lane;
    const bool valid = pt < end;
    double x = 0, y = 0, z = 0;
    if (valid) load_point<TIN>(a.px, a.py, a.pz, pt, x, y, z);
    double pu[P + 1], pv[P + 1], pw[P + 1];
    scaled_powers<P>(valid ? (x - cx) * sx : 0.0, pu);
    scaled_powers<P>(valid ? (y - cy) * sy : 0.0, pv);
    scaled_powers<P>(valid ? (z - cz) * sz : 0.0, pw);
    if (!valid) pu[0] = 0.0;
    __syncthreads();
    // wave w writes basis columns c = w, w+4, ...
#pragma unroll
    for (int c = 0; c < L; ++c)
      if ((c & 3) == w) tile[c * PS + lane] = pu[B.lx[c]] * pv[B.ly[c]] * pw[B.lz[c]];
    __syncthreads();
    if (tid < PB) {
      double s = 0.0;
      for (int c = 0; c < L; ++c) s += tile[c * PS + tid] * Fs[c];
      rp[tid] = (bs + tid < end) ? a.r[bs + tid] - s : 0.0;
    }
    __syncthreads();
    if (tid < L) {
      const double* col = tile + tid * PS;
#pragma unroll 8
      for (int q = 0; q < PB; ++q) acc += col[q] * rp[q];
    }
  }
  if (tid < L) part_b[(size_t)g * L + tid] = acc;
}

template <int P>
__global__ void __launch_bounds__(256) k_refine_solve(LevelArgs a, const double* __restrict__ part_b,
                                                      const double* __restrict__ fac) {
  constexpr int L = basis_size(P);
  constexpr int NPK = L * (L + 1) / 2;
  __shared__ double A[NPK];
  __shared__ double b[L], y[L], z[L], dg[L], sc[L];
  const int tid = threadIdx.x;
  const uint32_t k = blockIdx.x;
  const uint32_t node = a.node0 + k;
  const uint32_t c0 = a.chunk_off[k], c1 = a.chunk_off[k + 1];
  const double* fo = fac + (size_t)k * (NPK + 2 * L);
  for (int e = tid; e < NPK; e += 256) A[e] = fo[e];
  for (int i = tid; i < L; i += 256) {
    dg[i] = fo[NPK + i];
    sc[i] = fo[NPK + L + i];
    double s = 0.0;
    for (uint32_t g = c0; g < c1; ++g) s += part_b[(size_t)g * L + i];
    b[i] = s * fo[NPK + L + i];
  }
  __syncthreads();
  tri_solve<L>(A, dg, b, y, z);
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
  const uint32_t c0 = a.chunk_off[k], c1 = a.chunk_off[k + 1];
  uint32_t mask = 0;
  for (int o = 0; o < 8; ++o) {
    const uint32_t n_o = bnd[o + 1] - bnd[o];
    cbeg[(size_t)k * 8 + o] = bnd[o];
    ccnt[(size_t)k * 8 + o] = n_o;
    if (n_o < L) continue;
    double s = 0.0;
    for (uint32_t gg = c0; gg < c1; ++gg) s += part_ss[(size_t)gg * 8 + o];
    if (sqrt(s / (double)n_o) > a.tol) mask |= 1u << o;
  }
  a.nt.child_mask[node] = mask;
  nact[k] = (uint32_t)__popc(mask);
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
      ++run;
    }
  }
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
static hipError_t sweep_impl(int dtype, const LevelArgs& a, double* part_b, hipStream_t s) {
  if (a.nchunks == 0) return hipSuccess;
  if (dtype == FMT_F32) hipLaunchKernelGGL((k_refine_sweep<P, float>), dim3(a.nchunks), dim3(256), 0, s, a, part_b);
  else hipLaunchKernelGGL((k_refine_sweep<P, double>), dim3(a.nchunks), dim3(256), 0, s, a, part_b);
  return hipGetLastError();
}
hipError_t launch_refine_sweep(int p, int dtype, const LevelArgs& a, double* part_b, hipStream_t s) {
  FMT_DISPATCH_P(p, sweep_impl, dtype, a, part_b, s);
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
