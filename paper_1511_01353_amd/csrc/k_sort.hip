// Morton keys, stable LSD radix sort of (key, index) pairs, and the gather of
// points into key order.
//
// Keys replace the per-node octant ordering of Alg. 1: sorting once by the
// interleaved cell bits puts the points of every octree node, at every
// depth, in one contiguous range, children in octant order.
#include "k_sort.h"

namespace fmt {

__device__ __forceinline__ uint32_t find_problem(const ProblemParams* prm, int nprob, uint32_t g) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prm[mid].offset <= g) lo = mid; else hi = mid - 1;
  }
  return (uint32_t)lo;
}

template <typename T>
__global__ void __launch_bounds__(256) k_keygen(const PtrSet* ptrs, const ProblemParams* prm,
                                                int nprob, int depth, uint32_t total,
                                                uint32_t* keys, uint32_t* status, PtrSet cat) {
  uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  uint32_t k = nprob == 1 ? 0u : find_problem(prm, nprob, g);
  const ProblemParams& P = prm[k];
  uint32_t i = g - P.offset;
  const T* X = (const T*)ptrs[k].x;
  const T* Y = (const T*)ptrs[k].y;
  const T* Z = (const T*)ptrs[k].z;
  double x = (double)X[i], y = (double)Y[i], z = (double)Z[i];
  bool bad = false;
  // domain: finite and inside the closed box
  if (!(x >= P.lo[0] && x <= P.hi[0] && y >= P.lo[1] && y <= P.hi[1] && z >= P.lo[2] && z <= P.hi[2]))
    bad = true;
  uint32_t cmax = (1u << depth) - 1u;
  uint32_t qx = cell_of(x, P.lo[0], P.qscale[0], cmax, &bad);
  uint32_t qy = cell_of(y, P.lo[1], P.qscale[1], cmax, &bad);
  uint32_t qz = cell_of(z, P.lo[2], P.qscale[2], cmax, &bad);
  uint32_t key = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
  if (nprob > 1) key |= k << (3 * depth);
  keys[g] = key;
  if (bad) atomicOr(status, STATUS_DOMAIN);
  if (cat.x) {
    // a batch's inputs, concatenated in global point order (the sort's payload)
    ((T*)cat.x)[g] = X[i];
    ((T*)cat.y)[g] = Y[i];
    ((T*)cat.z)[g] = Z[i];
    ((T*)cat.f)[g] = ((const T*)ptrs[k].f)[i];
  }
}

// Query keys for evaluation of one tree: same cell rule, no domain check
// (outside queries follow the clamped path).
template <typename T>
__global__ void __launch_bounds__(256) k_query_keys(const T* qx, const T* qy, const T* qz, uint32_t nq,
                                                    ProblemParams P, int depth, uint32_t* keys) {
  uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nq) return;
  bool bad = false;
  uint32_t cmax = (1u << depth) - 1u;
  uint32_t a = cell_of((double)qx[g], P.lo[0], P.qscale[0], cmax, &bad);
  uint32_t b = cell_of((double)qy[g], P.lo[1], P.qscale[1], cmax, &bad);
  uint32_t c = cell_of((double)qz[g], P.lo[2], P.qscale[2], cmax, &bad);
  keys[g] = (spread3(a) << 2) | (spread3(b) << 1) | spread3(c);
}

// ---------------------------------------------------------------------------
// Radix sort, one pass per RADIX_BITS digit.
// Tile t of SORT_TILE keys is handled by block t; inside the tile, wave w
// owns the contiguous quarter [w*TILE/4, (w+1)*TILE/4) and walks it in rounds
// of 64 keys.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(SORT_THREADS) k_radix_hist(const uint32_t* __restrict__ keys, uint32_t n,
                                                             int shift, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[RADIX];
  for (int i = threadIdx.x; i < RADIX; i += SORT_THREADS) h[i] = 0;
  __syncthreads();
  uint32_t base = blockIdx.x * SORT_TILE;
#pragma unroll
  for (int j = 0; j < SORT_ITEMS; ++j) {
    uint32_t i = base + j * SORT_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & (RADIX - 1)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < RADIX; d += SORT_THREADS) hist[d * gridDim.x + blockIdx.x] = h[d];
}

// Exclusive scan of one digit's per-tile counts (workgroup d owns digit d:
// hist[d * tiles + t], contiguous, read in coalesced rounds of 256); the
// digit's total goes to tot[d].
__global__ void __launch_bounds__(256) k_digit_scan(uint32_t* __restrict__ hist, uint32_t tiles,
                                                    uint32_t* __restrict__ tot) {
  __shared__ uint32_t s[256];
  const uint32_t tid = threadIdx.x;
  uint32_t* row = hist + (size_t)blockIdx.x * tiles;
  uint32_t run = 0;
  for (uint32_t base = 0; base < tiles; base += 256) {
    const uint32_t i = base + tid;
    const uint32_t v = i < tiles ? row[i] : 0u;
    s[tid] = v;
    __syncthreads();
    for (uint32_t off = 1; off < 256; off <<= 1) {
      const uint32_t t = tid >= off ? s[tid - off] : 0u;
      __syncthreads();
      s[tid] += t;
      __syncthreads();
    }
    if (i < tiles) row[i] = run + s[tid] - v;
    run += s[255];
    __syncthreads();
  }
  if (tid == 0) tot[blockIdx.x] = run;
}

template <bool FIRST>
__global__ void __launch_bounds__(SORT_THREADS) k_radix_scatter(const uint32_t* __restrict__ kin,
                                                                const uint32_t* __restrict__ vin,
                                                                uint32_t* __restrict__ kout,
                                                                uint32_t* __restrict__ vout, uint32_t n,
                                                                int shift,
                                                                const uint32_t* __restrict__ offs,
                                                                const uint32_t* __restrict__ tot) {
  constexpr int WAVES = SORT_THREADS / 64;
  constexpr int QUARTER = SORT_TILE / WAVES;
  constexpr int ROUNDS = QUARTER / 64;
  __shared__ uint32_t wcnt[WAVES][RADIX];
  __shared__ uint32_t lofs[RADIX];
  __shared__ uint32_t goff[RADIX];
  __shared__ uint32_t dbase[RADIX];
  __shared__ uint32_t sk[SORT_TILE];
  __shared__ uint32_t sv[SORT_TILE];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int i = tid; i < WAVES * RADIX; i += SORT_THREADS) (&wcnt[0][0])[i] = 0;
  __syncthreads();

  const uint64_t below_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint32_t base = blockIdx.x * SORT_TILE + w * QUARTER;
  uint32_t key[ROUNDS], val[ROUNDS], rank[ROUNDS];
#pragma unroll
  for (int j = 0; j < ROUNDS; ++j) {
    const uint32_t i = base + j * 64 + lane;
    const bool valid = i < n;
    const uint32_t k = valid ? kin[i] : 0u;
    const uint32_t d = (k >> shift) & (RADIX - 1);
    // lanes of this wave holding the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < RADIX_BITS; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t before = (uint32_t)__popcll(peers & below_mask);
    const uint32_t c = wcnt[w][d];
    rank[j] = c + before;
    // the lowest lane of each digit group advances the wave's running count;
    // every lane of the group read the old value in the load above
    __builtin_amdgcn_wave_barrier();
    if (valid && before == 0) wcnt[w][d] = c + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
    key[j] = k;
    val[j] = FIRST ? i : (valid ? vin[i] : 0u);
  }
  __syncthreads();
  // per digit: wave bases and the tile-local digit start
  if (tid < RADIX) {
    uint32_t run = 0;
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) {
      uint32_t c = wcnt[ww][tid];
      wcnt[ww][tid] = run;
      run += c;
    }
    lofs[tid] = run;   // tile-local digit total for now
    dbase[tid] = tot[tid];
  }
  __syncthreads();
  // exclusive scans of the tile-local and of the global digit totals
  const uint32_t mine = tid < RADIX ? lofs[tid] : 0u;
  const uint32_t mine_g = tid < RADIX ? dbase[tid] : 0u;
  for (int off = 1; off < RADIX; off <<= 1) {
    const uint32_t v = (tid < RADIX && tid >= off) ? lofs[tid - off] : 0u;
    const uint32_t vg = (tid < RADIX && tid >= off) ? dbase[tid - off] : 0u;
    __syncthreads();
    if (tid < RADIX) {
      lofs[tid] += v;
      dbase[tid] += vg;
    }
    __syncthreads();
  }
  if (tid < RADIX) {
    lofs[tid] -= mine;
    goff[tid] = dbase[tid] - mine_g + offs[tid * gridDim.x + blockIdx.x];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ROUNDS; ++j) {
    const uint32_t i = base + j * 64 + lane;
    if (i < n) {
      const uint32_t d = (key[j] >> shift) & (RADIX - 1);
      const uint32_t pos = lofs[d] + wcnt[w][d] + rank[j];
      sk[pos] = key[j];
      sv[pos] = val[j];
    }
  }
  __syncthreads();
  const uint32_t tile0 = blockIdx.x * SORT_TILE;
  const uint32_t tn = min((uint32_t)SORT_TILE, n - tile0);
  for (uint32_t i = tid; i < tn; i += SORT_THREADS) {
    const uint32_t k = sk[i];
    const uint32_t d = (k >> shift) & (RADIX - 1);
    const uint32_t o = goff[d] + (i - lofs[d]);
    kout[o] = k;
    vout[o] = sv[i];
  }
}

// The same pass moving NP payload arrays of PT along with (key, value).
// Ranks and destinations as above; once keys and values are out, their LDS
// staging area is reused for the payload, one array at a time (read
// coalesced at the element's source position, written coalesced at its
// destination), so the payload costs neither registers during ranking nor
// extra LDS.  FIRST: values are source positions (not read).
template <bool FIRST, typename PT, int NP>
__global__ void __launch_bounds__(SORT_THREADS) k_radix_scatter_p(const uint32_t* __restrict__ kin,
                                                                  const uint32_t* __restrict__ vin,
                                                                  PayloadSet<PT, NP> pin,
                                                                  uint32_t* __restrict__ kout,
                                                                  uint32_t* __restrict__ vout,
                                                                  PayloadSet<PT, NP> pout, uint32_t n, int shift,
                                                                  const uint32_t* __restrict__ offs,
                                                                  const uint32_t* __restrict__ tot) {
  constexpr int WAVES = SORT_THREADS / 64;
  constexpr int QUARTER = SORT_TILE / WAVES;
  constexpr int ROUNDS = QUARTER / 64;
  constexpr int OUTS = SORT_TILE / SORT_THREADS;
  static_assert(sizeof(PT) <= 8, "payload elements of at most 8 bytes");
  __shared__ uint32_t wcnt[WAVES][RADIX];
  __shared__ uint32_t lofs[RADIX];
  __shared__ uint32_t goff[RADIX];
  __shared__ uint32_t dbase[RADIX];
  __shared__ __attribute__((aligned(16))) uint32_t stage[2 * SORT_TILE];
  uint32_t* sk = stage;
  uint32_t* sv = stage + SORT_TILE;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int i = tid; i < WAVES * RADIX; i += SORT_THREADS) (&wcnt[0][0])[i] = 0;
  __syncthreads();

  const uint64_t below_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint32_t base = blockIdx.x * SORT_TILE + w * QUARTER;
  // 4-byte payloads are loaded up front so that their latency overlaps the
  // ranking; wider ones are read again at staging time
  constexpr bool PRELOAD = sizeof(PT) == 4;
  PT pre[PRELOAD ? NP : 1][PRELOAD ? ROUNDS : 1];
  if constexpr (PRELOAD) {
#pragma unroll
    for (int a = 0; a < NP; ++a)
#pragma unroll
      for (int j = 0; j < ROUNDS; ++j) {
        const uint32_t i = base + j * 64 + lane;
        pre[a][j] = i < n ? pin.a[a][i] : PT(0);
      }
  }
  uint32_t key[ROUNDS], rank[ROUNDS];
#pragma unroll
  for (int j = 0; j < ROUNDS; ++j) {
    const uint32_t i = base + j * 64 + lane;
    const bool valid = i < n;
    const uint32_t k = valid ? kin[i] : 0u;
    const uint32_t d = (k >> shift) & (RADIX - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < RADIX_BITS; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t before = (uint32_t)__popcll(peers & below_mask);
    const uint32_t c = wcnt[w][d];
    rank[j] = c + before;
    __builtin_amdgcn_wave_barrier();
    if (valid && before == 0) wcnt[w][d] = c + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
    key[j] = k;
  }
  __syncthreads();
  if (tid < RADIX) {
    uint32_t run = 0;
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) {
      uint32_t c = wcnt[ww][tid];
      wcnt[ww][tid] = run;
      run += c;
    }
    lofs[tid] = run;
    dbase[tid] = tot[tid];
  }
  __syncthreads();
  const uint32_t mine = tid < RADIX ? lofs[tid] : 0u;
  const uint32_t mine_g = tid < RADIX ? dbase[tid] : 0u;
  for (int off = 1; off < RADIX; off <<= 1) {
    const uint32_t v = (tid < RADIX && tid >= off) ? lofs[tid - off] : 0u;
    const uint32_t vg = (tid < RADIX && tid >= off) ? dbase[tid - off] : 0u;
    __syncthreads();
    if (tid < RADIX) {
      lofs[tid] += v;
      dbase[tid] += vg;
    }
    __syncthreads();
  }
  if (tid < RADIX) {
    lofs[tid] -= mine;
    goff[tid] = dbase[tid] - mine_g + offs[tid * gridDim.x + blockIdx.x];
  }
  __syncthreads();
  // tile-local position of each of this lane's elements
  uint32_t pos[ROUNDS];
#pragma unroll
  for (int j = 0; j < ROUNDS; ++j) {
    const uint32_t i = base + j * 64 + lane;
    const uint32_t d = (key[j] >> shift) & (RADIX - 1);
    pos[j] = lofs[d] + wcnt[w][d] + rank[j];
    if (i < n) {
      sk[pos[j]] = key[j];
      sv[pos[j]] = FIRST ? i : vin[i];
    }
  }
  __syncthreads();
  const uint32_t tile0 = blockIdx.x * SORT_TILE;
  const uint32_t tn = min((uint32_t)SORT_TILE, n - tile0);
  // global destination of the tile positions this thread writes out
  uint32_t dst[OUTS];
#pragma unroll
  for (int m = 0; m < OUTS; ++m) {
    const uint32_t i = tid + m * SORT_THREADS;
    if (i < tn) {
      const uint32_t k = sk[i];
      const uint32_t d = (k >> shift) & (RADIX - 1);
      dst[m] = goff[d] + (i - lofs[d]);
      kout[dst[m]] = k;
      vout[dst[m]] = sv[i];
    }
  }
  PT* sp = (PT*)stage;
#pragma unroll
  for (int a = 0; a < NP; ++a) {
    __syncthreads();   // the staging area is free again
#pragma unroll
    for (int j = 0; j < ROUNDS; ++j) {
      const uint32_t i = base + j * 64 + lane;
      if (i < n) {
        if constexpr (PRELOAD) sp[pos[j]] = pre[a][j];
        else sp[pos[j]] = pin.a[a][i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < OUTS; ++m) {
      const uint32_t i = tid + m * SORT_THREADS;
      if (i < tn) pout.a[a][dst[m]] = sp[i];
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_keygen(int dtype, const PtrSet* ptrs, const ProblemParams* prm, int nprob, int depth,
                         uint32_t total, uint32_t* keys, uint32_t* status, const PtrSet& cat, hipStream_t s) {
  if (total == 0) return hipSuccess;
  if (dtype == FMT_F32)
    hipLaunchKernelGGL(k_keygen<float>, dim3(blocks_for(total, 256)), dim3(256), 0, s, ptrs, prm, nprob, depth,
                       total, keys, status, cat);
  else
    hipLaunchKernelGGL(k_keygen<double>, dim3(blocks_for(total, 256)), dim3(256), 0, s, ptrs, prm, nprob, depth,
                       total, keys, status, cat);
  return hipGetLastError();
}

hipError_t launch_query_keys(int dtype, const void* qx, const void* qy, const void* qz, uint32_t nq,
                             const ProblemParams& P, int depth, uint32_t* keys, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  if (dtype == FMT_F32)
    hipLaunchKernelGGL(k_query_keys<float>, dim3(blocks_for(nq, 256)), dim3(256), 0, s, (const float*)qx,
                       (const float*)qy, (const float*)qz, nq, P, depth, keys);
  else
    hipLaunchKernelGGL(k_query_keys<double>, dim3(blocks_for(nq, 256)), dim3(256), 0, s, (const double*)qx,
                       (const double*)qy, (const double*)qz, nq, P, depth, keys);
  return hipGetLastError();
}

int radix_sort_passes(int bits) {
  const int p = (bits + RADIX_BITS - 1) / RADIX_BITS;
  return p < 1 ? 1 : p;
}

size_t radix_sort_scratch_words(uint32_t n) {
  uint32_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
  return (size_t)RADIX * tiles + RADIX + 16;
}

hipError_t radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, uint32_t n,
                      int bits, bool vals_are_iota, uint32_t* scratch, hipStream_t s, bool* result_in_alt) {
  *result_in_alt = false;
  if (n == 0) return hipSuccess;
  const uint32_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
  uint32_t* hist = scratch;
  uint32_t* tot = scratch + (size_t)RADIX * tiles;
  int passes = (bits + RADIX_BITS - 1) / RADIX_BITS;
  if (passes < 1) passes = 1;   // at least one pass so that the index array is written
  uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * RADIX_BITS;
    hipLaunchKernelGGL(k_radix_hist, dim3(tiles), dim3(SORT_THREADS), 0, s, ki, n, shift, hist);
    hipLaunchKernelGGL(k_digit_scan, dim3(RADIX), dim3(256), 0, s, hist, tiles, tot);
    if (p == 0 && vals_are_iota)
      hipLaunchKernelGGL(k_radix_scatter<true>, dim3(tiles), dim3(SORT_THREADS), 0, s, ki, vi, ko, vo, n, shift,
                         hist, tot);
    else
      hipLaunchKernelGGL(k_radix_scatter<false>, dim3(tiles), dim3(SORT_THREADS), 0, s, ki, vi, ko, vo, n, shift,
                         hist, tot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t* t = ki; ki = ko; ko = t;
    t = vi; vi = vo; vo = t;
  }
  *result_in_alt = (ki != keys);
  return hipSuccess;
}

template <typename PT, int NP>
static hipError_t radix_sort_payload_t(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                                       const void* const* pin, void* const* pay, void* const* pay_alt, uint32_t n,
                                       int bits, uint32_t* scratch, hipStream_t s, bool* result_in_alt) {
  const uint32_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
  uint32_t* hist = scratch;
  uint32_t* tot = scratch + (size_t)RADIX * tiles;
  const int passes = radix_sort_passes(bits);
  uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
  PayloadSet<PT, NP> src, a, b;
  for (int q = 0; q < NP; ++q) {
    src.a[q] = (PT*)pin[q];
    a.a[q] = (PT*)pay[q];
    b.a[q] = (PT*)pay_alt[q];
  }
  // pass 0 reads the caller's payload and writes the alternate set, then the
  // sets alternate like the keys
  PayloadSet<PT, NP> pi = src, po = b;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * RADIX_BITS;
    hipLaunchKernelGGL(k_radix_hist, dim3(tiles), dim3(SORT_THREADS), 0, s, ki, n, shift, hist);
    hipLaunchKernelGGL(k_digit_scan, dim3(RADIX), dim3(256), 0, s, hist, tiles, tot);
    if (p == 0)
      hipLaunchKernelGGL((k_radix_scatter_p<true, PT, NP>), dim3(tiles), dim3(SORT_THREADS), 0, s, ki, vi, pi, ko,
                         vo, po, n, shift, hist, tot);
    else
      hipLaunchKernelGGL((k_radix_scatter_p<false, PT, NP>), dim3(tiles), dim3(SORT_THREADS), 0, s, ki, vi, pi,
                         ko, vo, po, n, shift, hist, tot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    std::swap(ki, ko);
    std::swap(vi, vo);
    pi = po;
    po = (p % 2 == 0) ? a : b;
  }
  *result_in_alt = ki != keys;
  return hipSuccess;
}

hipError_t radix_sort_payload(int dtype, int np, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                              uint32_t* vals_alt, const void* const* pin, void* const* pay, void* const* pay_alt,
                              uint32_t n, int bits, uint32_t* scratch, hipStream_t s, bool* result_in_alt) {
  *result_in_alt = false;
  if (n == 0) return hipSuccess;
  if (np == 3) {
    if (dtype == FMT_F32)
      return radix_sort_payload_t<float, 3>(keys, vals, keys_alt, vals_alt, pin, pay, pay_alt, n, bits, scratch, s,
                                            result_in_alt);
    return radix_sort_payload_t<double, 3>(keys, vals, keys_alt, vals_alt, pin, pay, pay_alt, n, bits, scratch, s,
                                           result_in_alt);
  }
  if (np == 4) {
    if (dtype == FMT_F32)
      return radix_sort_payload_t<float, 4>(keys, vals, keys_alt, vals_alt, pin, pay, pay_alt, n, bits, scratch, s,
                                            result_in_alt);
    return radix_sort_payload_t<double, 4>(keys, vals, keys_alt, vals_alt, pin, pay, pay_alt, n, bits, scratch, s,
                                           result_in_alt);
  }
  return hipErrorInvalidValue;
}

// residual start: the sorted values, widened to float64
template <typename T>
__global__ void __launch_bounds__(256) k_widen(const T* __restrict__ f, uint32_t n, double* __restrict__ r) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = (double)f[i];
}

hipError_t launch_widen(int dtype, const void* f, uint32_t n, double* r, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (dtype == FMT_F32)
    hipLaunchKernelGGL(k_widen<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, (const float*)f, n, r);
  else
    hipLaunchKernelGGL(k_widen<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, (const double*)f, n, r);
  return hipGetLastError();
}


}  // namespace fmt
