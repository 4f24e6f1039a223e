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
// Radix sort, one pass per BITS-bit digit (BITS = 8, 9 or 10, chosen per
// sort so that the key takes the fewest passes).
// Tile t of SORT_TILE keys is handled by block t; inside the tile, wave w
// owns the contiguous quarter [w*TILE/4, (w+1)*TILE/4) and walks it in rounds
// of 64 keys.
// ---------------------------------------------------------------------------
template <int BITS>
__global__ void __launch_bounds__(SORT_THREADS) k_radix_hist(const uint32_t* __restrict__ keys, uint32_t n,
                                                             int shift, uint32_t* __restrict__ hist) {
  constexpr int R = 1 << BITS;
  __shared__ uint32_t h[R];
  for (int i = threadIdx.x; i < R; i += SORT_THREADS) h[i] = 0;
  __syncthreads();
  uint32_t base = blockIdx.x * SORT_TILE;
#pragma unroll
  for (int j = 0; j < SORT_ITEMS; ++j) {
    uint32_t i = base + j * SORT_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & (R - 1)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < R; d += SORT_THREADS) hist[d * gridDim.x + blockIdx.x] = h[d];
}

// Exclusive scans, in place, of two arrays x and y of R entries (R a
// multiple of SORT_THREADS): thread t owns entries [t E, (t + 1) E); waves
// scan with shuffles, then the wave totals are added in order.  Every
// thread of the workgroup calls it.
template <int R>
__device__ __forceinline__ void exclusive_scan_pair(uint32_t* x, uint32_t* y, uint32_t* wx, uint32_t* wy) {
  static_assert(R % SORT_THREADS == 0, "digit count must be a multiple of the workgroup size");
  constexpr int E = R / SORT_THREADS;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint32_t vx[E], vy[E], sx = 0, sy = 0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    vx[e] = x[tid * E + e];
    vy[e] = y[tid * E + e];
    sx += vx[e];
    sy += vy[e];
  }
  uint32_t ix = sx, iy = sy;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t tx = (uint32_t)__shfl_up((int)ix, off), ty = (uint32_t)__shfl_up((int)iy, off);
    if (lane >= off) {
      ix += tx;
      iy += ty;
    }
  }
  if (lane == 63) {
    wx[w] = ix;
    wy[w] = iy;
  }
  __syncthreads();
  uint32_t rx = ix - sx, ry = iy - sy;
  for (int q = 0; q < w; ++q) {
    rx += wx[q];
    ry += wy[q];
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    x[tid * E + e] = rx;
    rx += vx[e];
    y[tid * E + e] = ry;
    ry += vy[e];
  }
  __syncthreads();
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

template <bool FIRST, int BITS>
__global__ void __launch_bounds__(SORT_THREADS) k_radix_scatter(const uint32_t* __restrict__ kin,
                                                                const uint32_t* __restrict__ vin,
                                                                uint32_t* __restrict__ kout,
                                                                uint32_t* __restrict__ vout, uint32_t n,
                                                                int shift,
                                                                const uint32_t* __restrict__ offs,
                                                                const uint32_t* __restrict__ tot) {
  constexpr int R = 1 << BITS;
  constexpr int WAVES = SORT_THREADS / 64;
  constexpr int QUARTER = SORT_TILE / WAVES;
  constexpr int ROUNDS = QUARTER / 64;
  __shared__ uint32_t wcnt[WAVES][R];
  __shared__ uint32_t lofs[R];
  __shared__ uint32_t goff[R];
  __shared__ uint32_t dbase[R];
  __shared__ uint32_t wsum[2][WAVES];
  __shared__ uint32_t sk[SORT_TILE];
  __shared__ uint32_t sv[SORT_TILE];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int i = tid; i < WAVES * R; i += SORT_THREADS) (&wcnt[0][0])[i] = 0;
  __syncthreads();

  const uint64_t below_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint32_t base = blockIdx.x * SORT_TILE + w * QUARTER;
  uint32_t key[ROUNDS], val[ROUNDS], rank[ROUNDS];
#pragma unroll
  for (int j = 0; j < ROUNDS; ++j) {
    const uint32_t i = base + j * 64 + lane;
    const bool valid = i < n;
    const uint32_t k = valid ? kin[i] : 0u;
    const uint32_t d = (k >> shift) & (R - 1);
    // lanes of this wave holding the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
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
  for (int d = tid; d < R; d += SORT_THREADS) {
    uint32_t run = 0;
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) {
      uint32_t c = wcnt[ww][d];
      wcnt[ww][d] = run;
      run += c;
    }
    lofs[d] = run;   // tile-local digit total for now
    dbase[d] = tot[d];
  }
  __syncthreads();
  // exclusive scans of the tile-local and of the global digit totals
  exclusive_scan_pair<R>(lofs, dbase, wsum[0], wsum[1]);
  for (int d = tid; d < R; d += SORT_THREADS) goff[d] = dbase[d] + offs[d * gridDim.x + blockIdx.x];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ROUNDS; ++j) {
    const uint32_t i = base + j * 64 + lane;
    if (i < n) {
      const uint32_t d = (key[j] >> shift) & (R - 1);
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
    const uint32_t d = (k >> shift) & (R - 1);
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
template <bool FIRST, typename PT, int NP, int BITS>
__global__ void __launch_bounds__(SORT_THREADS) k_radix_scatter_p(const uint32_t* __restrict__ kin,
                                                                  const uint32_t* __restrict__ vin,
                                                                  PayloadSet<PT, NP> pin,
                                                                  uint32_t* __restrict__ kout,
                                                                  uint32_t* __restrict__ vout,
                                                                  PayloadSet<PT, NP> pout, uint32_t n, int shift,
                                                                  const uint32_t* __restrict__ offs,
                                                                  const uint32_t* __restrict__ tot) {
  constexpr int R = 1 << BITS;
  constexpr int WAVES = SORT_THREADS / 64;
  constexpr int QUARTER = SORT_TILE / WAVES;
  constexpr int ROUNDS = QUARTER / 64;
  constexpr int OUTS = SORT_TILE / SORT_THREADS;
  static_assert(sizeof(PT) <= 8, "payload elements of at most 8 bytes");
  __shared__ uint32_t wcnt[WAVES][R];
  __shared__ uint32_t lofs[R];
  __shared__ uint32_t goff[R];
  __shared__ uint32_t dbase[R];
  __shared__ uint32_t wsum[2][WAVES];
  __shared__ __attribute__((aligned(16))) uint32_t stage[2 * SORT_TILE];
  uint32_t* sk = stage;
  uint32_t* sv = stage + SORT_TILE;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int i = tid; i < WAVES * R; i += SORT_THREADS) (&wcnt[0][0])[i] = 0;
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
    const uint32_t d = (k >> shift) & (R - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
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
  for (int d = tid; d < R; d += SORT_THREADS) {
    uint32_t run = 0;
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) {
      uint32_t c = wcnt[ww][d];
      wcnt[ww][d] = run;
      run += c;
    }
    lofs[d] = run;   // tile-local digit total for now
    dbase[d] = tot[d];
  }
  __syncthreads();
  // exclusive scans of the tile-local and of the global digit totals
  exclusive_scan_pair<R>(lofs, dbase, wsum[0], wsum[1]);
  for (int d = tid; d < R; d += SORT_THREADS) goff[d] = dbase[d] + offs[d * gridDim.x + blockIdx.x];
  __syncthreads();
  // tile-local position of each of this lane's elements
  uint32_t pos[ROUNDS];
#pragma unroll
  for (int j = 0; j < ROUNDS; ++j) {
    const uint32_t i = base + j * 64 + lane;
    const uint32_t d = (key[j] >> shift) & (R - 1);
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
      const uint32_t d = (k >> shift) & (R - 1);
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

// Digit width for a sort over `bits` key bits: 8, 9 or 10, the narrowest
// that needs the fewest passes (e.g. 18 bits: two passes of 9).
static int digit_bits(int bits) {
  int best = 8, best_p = (bits + 7) / 8;
  for (int w = 9; w <= MAX_RADIX_BITS; ++w) {
    const int p = (bits + w - 1) / w;
    if (p < best_p) {
      best = w;
      best_p = p;
    }
  }
  return best;
}

int radix_sort_passes(int bits) {
  const int w = digit_bits(bits);
  const int p = (bits + w - 1) / w;
  return p < 1 ? 1 : p;   // at least one pass so that the index array is written
}

size_t radix_sort_scratch_words(uint32_t n) {
  uint32_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
  return ((size_t)tiles + 1) * (1u << MAX_RADIX_BITS) + 16;
}

// One pass (histogram, digit scan, scatter) of the plain sort.
template <int BITS>
static void plain_pass(bool iota, const uint32_t* ki, const uint32_t* vi, uint32_t* ko, uint32_t* vo, uint32_t n,
                       uint32_t tiles, int shift, uint32_t* hist, uint32_t* tot, hipStream_t s) {
  hipLaunchKernelGGL(k_radix_hist<BITS>, dim3(tiles), dim3(SORT_THREADS), 0, s, ki, n, shift, hist);
  hipLaunchKernelGGL(k_digit_scan, dim3(1 << BITS), dim3(256), 0, s, hist, tiles, tot);
  if (iota)
    hipLaunchKernelGGL((k_radix_scatter<true, BITS>), dim3(tiles), dim3(SORT_THREADS), 0, s, ki, vi, ko, vo, n,
                       shift, hist, tot);
  else
    hipLaunchKernelGGL((k_radix_scatter<false, BITS>), dim3(tiles), dim3(SORT_THREADS), 0, s, ki, vi, ko, vo, n,
                       shift, hist, tot);
}

hipError_t radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, uint32_t n,
                      int bits, bool vals_are_iota, uint32_t* scratch, hipStream_t s, bool* result_in_alt) {
  *result_in_alt = false;
  if (n == 0) return hipSuccess;
  const uint32_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
  const int w = digit_bits(bits);
  uint32_t* hist = scratch;
  uint32_t* tot = scratch + ((size_t)tiles << w);
  const int passes = radix_sort_passes(bits);
  uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
  for (int p = 0; p < passes; ++p) {
    const bool iota = p == 0 && vals_are_iota;
    if (w == 8) plain_pass<8>(iota, ki, vi, ko, vo, n, tiles, p * w, hist, tot, s);
    else if (w == 9) plain_pass<9>(iota, ki, vi, ko, vo, n, tiles, p * w, hist, tot, s);
    else plain_pass<10>(iota, ki, vi, ko, vo, n, tiles, p * w, hist, tot, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t* t = ki; ki = ko; ko = t;
    t = vi; vi = vo; vo = t;
  }
  *result_in_alt = (ki != keys);
  return hipSuccess;
}

// One pass of the payload sort.
template <typename PT, int NP, int BITS>
static void payload_pass(bool first, const uint32_t* ki, const uint32_t* vi, const PayloadSet<PT, NP>& pi,
                         uint32_t* ko, uint32_t* vo, const PayloadSet<PT, NP>& po, uint32_t n, uint32_t tiles,
                         int shift, uint32_t* hist, uint32_t* tot, hipStream_t s) {
  hipLaunchKernelGGL(k_radix_hist<BITS>, dim3(tiles), dim3(SORT_THREADS), 0, s, ki, n, shift, hist);
  hipLaunchKernelGGL(k_digit_scan, dim3(1 << BITS), dim3(256), 0, s, hist, tiles, tot);
  if (first)
    hipLaunchKernelGGL((k_radix_scatter_p<true, PT, NP, BITS>), dim3(tiles), dim3(SORT_THREADS), 0, s, ki, vi, pi,
                       ko, vo, po, n, shift, hist, tot);
  else
    hipLaunchKernelGGL((k_radix_scatter_p<false, PT, NP, BITS>), dim3(tiles), dim3(SORT_THREADS), 0, s, ki, vi, pi,
                       ko, vo, po, n, shift, hist, tot);
}

template <typename PT, int NP>
static hipError_t radix_sort_payload_t(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                                       const void* const* pin, void* const* pay, void* const* pay_alt, uint32_t n,
                                       int bits, uint32_t* scratch, hipStream_t s, bool* result_in_alt) {
  const uint32_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
  const int w = digit_bits(bits);
  uint32_t* hist = scratch;
  uint32_t* tot = scratch + ((size_t)tiles << w);
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
    if (w == 8) payload_pass<PT, NP, 8>(p == 0, ki, vi, pi, ko, vo, po, n, tiles, p * w, hist, tot, s);
    else if (w == 9) payload_pass<PT, NP, 9>(p == 0, ki, vi, pi, ko, vo, po, n, tiles, p * w, hist, tot, s);
    else payload_pass<PT, NP, 10>(p == 0, ki, vi, pi, ko, vo, po, n, tiles, p * w, hist, tot, s);
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
__global__ void __launch_bounds__(256) k_widen(const T* __restrict__ f, uint32_t n, double* __restrict__ r,
                                               uint32_t* __restrict__ zero, uint32_t nzero) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = (double)f[i];
  for (uint32_t j = i; j < nzero; j += gridDim.x * blockDim.x) zero[j] = 0u;
}

hipError_t launch_widen(int dtype, const void* f, uint32_t n, double* r, uint32_t* zero, uint32_t nzero,
                        hipStream_t s) {
  if (n == 0 && nzero == 0) return hipSuccess;
  const unsigned grid = blocks_for(n > nzero ? n : nzero, 256);
  if (dtype == FMT_F32)
    hipLaunchKernelGGL(k_widen<float>, dim3(grid), dim3(256), 0, s, (const float*)f, n, r, zero, nzero);
  else
    hipLaunchKernelGGL(k_widen<double>, dim3(grid), dim3(256), 0, s, (const double*)f, n, r, zero, nzero);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) k_refit_gather(const uint32_t* __restrict__ order,
                                                      const uint32_t* __restrict__ skey, uint32_t off, uint32_t n,
                                                      const T* __restrict__ x, const T* __restrict__ y,
                                                      const T* __restrict__ z, ProblemParams P, int depth,
                                                      T* __restrict__ px, T* __restrict__ py, T* __restrict__ pz,
                                                      uint32_t* status) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t j = order[off + i] - off;
  if (j >= n) {
    atomicOr(status, STATUS_MISMATCH);
    return;
  }
  const T vx = x[j], vy = y[j], vz = z[j];
  px[i] = vx;
  py[i] = vy;
  pz[i] = vz;
  const double dx = (double)vx, dy = (double)vy, dz = (double)vz;
  bool bad = !(dx >= P.lo[0] && dx <= P.hi[0] && dy >= P.lo[1] && dy <= P.hi[1] && dz >= P.lo[2] && dz <= P.hi[2]);
  const uint32_t cmax = (1u << depth) - 1u;
  const uint32_t key = (spread3(cell_of(dx, P.lo[0], P.qscale[0], cmax, &bad)) << 2) |
                       (spread3(cell_of(dy, P.lo[1], P.qscale[1], cmax, &bad)) << 1) |
                       spread3(cell_of(dz, P.lo[2], P.qscale[2], cmax, &bad));
  const uint32_t kmask = depth > 0 ? (1u << (3 * depth)) - 1u : 0u;
  if (bad || key != (skey[off + i] & kmask)) atomicOr(status, STATUS_MISMATCH);
}

template <typename T>
__global__ void __launch_bounds__(256) k_gather_fields(const uint32_t* __restrict__ order, uint32_t off, uint32_t n,
                                                       const T* __restrict__ f, uint64_t fstride,
                                                       double* __restrict__ r, uint64_t rstride) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t j = order[off + i] - off;
  if (j < n) r[(uint64_t)blockIdx.y * rstride + i] = (double)f[(uint64_t)blockIdx.y * fstride + j];
}

__global__ void __launch_bounds__(256) k_slice_points(const uint32_t* __restrict__ skey,
                                                      const uint32_t* __restrict__ order, uint32_t off, uint32_t n,
                                                      uint32_t kmask, uint32_t* __restrict__ okey,
                                                      uint32_t* __restrict__ oorder) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  okey[i] = skey[off + i] & kmask;
  oorder[i] = order[off + i] - off;
}

__global__ void __launch_bounds__(256) k_replicate(const uint32_t* __restrict__ src, uint64_t words,
                                                   uint32_t* __restrict__ dst, uint64_t stride_words) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) dst[(uint64_t)blockIdx.y * stride_words + i] = src[i];
}

hipError_t launch_replicate(const void* src, size_t bytes, void* dst, size_t stride, int rows, hipStream_t s) {
  if (rows <= 0 || bytes == 0) return hipSuccess;
  if ((bytes | stride | (uintptr_t)src | (uintptr_t)dst) & 3) return hipErrorInvalidValue;
  const uint64_t words = bytes / 4;
  hipLaunchKernelGGL(k_replicate, dim3(blocks_for(words, 256), (unsigned)rows), dim3(256), 0, s,
                     (const uint32_t*)src, words, (uint32_t*)dst, (uint64_t)(stride / 4));
  return hipGetLastError();
}

hipError_t launch_refit_gather(int dtype, const uint32_t* order, const uint32_t* skey, uint32_t off, uint32_t n,
                               const void* x, const void* y, const void* z, const ProblemParams& P, int depth,
                               void* px, void* py, void* pz, uint32_t* status, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (dtype == FMT_F32)
    hipLaunchKernelGGL(k_refit_gather<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, order, skey, off, n,
                       (const float*)x, (const float*)y, (const float*)z, P, depth, (float*)px, (float*)py,
                       (float*)pz, status);
  else
    hipLaunchKernelGGL(k_refit_gather<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, order, skey, off, n,
                       (const double*)x, (const double*)y, (const double*)z, P, depth, (double*)px, (double*)py,
                       (double*)pz, status);
  return hipGetLastError();
}

hipError_t launch_gather_fields(int dtype, const uint32_t* order, uint32_t off, uint32_t n, const void* f, int m,
                                uint64_t fstride, double* r, uint64_t rstride, hipStream_t s) {
  if (n == 0 || m <= 0) return hipSuccess;
  const dim3 grid(blocks_for(n, 256), (unsigned)m);
  if (dtype == FMT_F32)
    hipLaunchKernelGGL(k_gather_fields<float>, grid, dim3(256), 0, s, order, off, n, (const float*)f, fstride, r,
                       rstride);
  else
    hipLaunchKernelGGL(k_gather_fields<double>, grid, dim3(256), 0, s, order, off, n, (const double*)f, fstride, r,
                       rstride);
  return hipGetLastError();
}

hipError_t launch_slice_points(const uint32_t* skey, const uint32_t* order, uint32_t off, uint32_t n, uint32_t kmask,
                               uint32_t* okey, uint32_t* oorder, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_slice_points, dim3(blocks_for(n, 256)), dim3(256), 0, s, skey, order, off, n, kmask, okey,
                     oorder);
  return hipGetLastError();
}

}  // namespace fmt
