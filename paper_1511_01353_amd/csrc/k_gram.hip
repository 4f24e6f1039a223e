// Gram reduction of one (node, chunk) work item on the matrix cores.
//
// Alg. 2 factors the node's Vandermonde matrix Lambda (n x calL).  Here the
// least-squares system is formed as normal equations: the augmented Gram
// [Lambda | r]^T [Lambda | r] holds Lambda^T Lambda, the right-hand side
// Lambda^T r and r^T r.  Points are the reduction dimension of a 16x16x4 MFMA:
// a batch of 64 points is turned into basis values in LDS (column-major, one
// column per basis function, point index fastest), and every 16x16 block
// (t1 <= t2) of the padded augmented matrix accumulates over the batch in
// registers.  The four waves of a workgroup own disjoint blocks, so the
// partial of a chunk needs no cross-wave reduction.
#include "k_level.h"

namespace fmt {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename TT>
struct Mfma;

template <>
struct Mfma<double> {
  typedef d4_t acc_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of output element i held by `lane` (column is lane % 16)
  static __device__ __forceinline__ int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};

template <>
struct Mfma<float> {
  typedef f4_t acc_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

template <int P>
struct GramShape {
  static constexpr int L = basis_size(P);
  static constexpr int LA = L + 1;          // augmented with the residual column
  static constexpr int LP = pad16(LA);
  static constexpr int T = LP / 16;         // 16-wide block rows
  static constexpr int NPAIR = T * (T + 1) / 2;
  static constexpr int PB = 64;             // points per LDS batch
  static constexpr int PS = PB + 4;         // LDS column stride (spreads banks)
  static constexpr int MAXPW = (NPAIR + 3) / 4;
};

size_t gram_partial_doubles(int p) {
  int T = pad16(basis_size(p) + 1) / 16;
  return (size_t)T * (T + 1) / 2 * 256;
}

// Columns [C0, C1) of the batch tile for this lane's point: basis values,
// then the residual column, then zero padding.
template <int P, int C0, int C1, typename TT>
__device__ __forceinline__ void write_cols(TT* tile, int lane, const double (&pu)[P + 1],
                                           const double (&pv)[P + 1], const double (&pw)[P + 1], double rv) {
  constexpr Basis<P> B{};
  constexpr int L = basis_size(P);
  constexpr int PS = GramShape<P>::PS;
#pragma unroll
  for (int c = C0; c < C1; ++c) {
    double val;
    if (c < L) {
      val = pu[B.lx[c < L ? c : 0]] * pv[B.ly[c < L ? c : 0]] * pw[B.lz[c < L ? c : 0]];
    } else if (c == L) {
      val = rv;
    } else {
      val = 0.0;
    }
    tile[c * PS + lane] = (TT)val;
  }
}

// Partial Gram of points [start, end) of a node into `out`, basis values and
// products in TT.  Float32 products accumulate in float32 over one batch of 64
// points and are then added into float64 registers.
template <int P, typename TIN, typename TT>
__device__ __forceinline__ void gram_body(const LevelArgs& a, TT* tile, uint32_t start, uint32_t end,
                                          const double* geo, double* __restrict__ out) {
  using S = GramShape<P>;
  using M = Mfma<TT>;
  constexpr bool NARROW = sizeof(TT) < sizeof(double);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const double cx = geo[0], cy = geo[1], cz = geo[2], sx = geo[3], sy = geo[4], sz = geo[5];

  // blocks (t1, t2), t1 <= t2, enumerated row by row; wave w owns j = w + 4*jj
  int t1s[S::MAXPW], t2s[S::MAXPW];
#pragma unroll
  for (int jj = 0; jj < S::MAXPW; ++jj) {
    int rem = w + 4 * jj, t1 = 0;
    while (t1 < S::T && rem >= S::T - t1) { rem -= S::T - t1; ++t1; }
    t1s[jj] = t1;
    t2s[jj] = t1 + rem;
  }
  typename M::acc_t acc[S::MAXPW];
  double wide[NARROW ? S::MAXPW : 1][4];
#pragma unroll
  for (int jj = 0; jj < S::MAXPW; ++jj) {
    acc[jj] = typename M::acc_t{0, 0, 0, 0};
    if constexpr (NARROW) {
#pragma unroll
      for (int i = 0; i < 4; ++i) wide[jj][i] = 0.0;
    }
  }

  // the next batch's point is loaded before this batch's products, so its
  // memory latency overlaps the matrix-core work
  double nx = 0, ny = 0, nz = 0, nr = 0;
  if (start + lane < end) {
    load_point<TIN>(a.px, a.py, a.pz, start + lane, nx, ny, nz);
    nr = a.r[start + lane];
  }
  for (uint32_t bs = start; bs < end; bs += S::PB) {
    const uint32_t pt = bs + lane;
    const bool valid = pt < end;
    const double x = nx, y = ny, z = nz, rv = valid ? nr : 0.0;
    if (pt + S::PB < end) {
      load_point<TIN>(a.px, a.py, a.pz, pt + S::PB, nx, ny, nz);
      nr = a.r[pt + S::PB];
    }
    double u = valid ? (x - cx) * sx : 0.0;
    double v = valid ? (y - cy) * sy : 0.0;
    double ww = valid ? (z - cz) * sz : 0.0;
    double pu[P + 1], pv[P + 1], pw[P + 1];
    scaled_powers<P>(u, pu);
    scaled_powers<P>(v, pv);
    scaled_powers<P>(ww, pw);
    if (!valid) pu[0] = 0.0;
    __syncthreads();   // the previous batch's operand reads are done
    constexpr int Q = S::LP / 4;
    switch (w) {
      case 0: write_cols<P, 0, Q>(tile, lane, pu, pv, pw, rv); break;
      case 1: write_cols<P, Q, 2 * Q>(tile, lane, pu, pv, pw, rv); break;
      case 2: write_cols<P, 2 * Q, 3 * Q>(tile, lane, pu, pv, pw, rv); break;
      default: write_cols<P, 3 * Q, S::LP>(tile, lane, pu, pv, pw, rv); break;
    }
    __syncthreads();
    const int c = lane & 15;
#pragma unroll 4
    for (int ks = 0; ks < S::PB / 4; ++ks) {
      const int prow = ks * 4 + (lane >> 4);
#pragma unroll
      for (int jj = 0; jj < S::MAXPW; ++jj) {
        if (w + 4 * jj < S::NPAIR) {
          const TT av = tile[(16 * t1s[jj] + c) * S::PS + prow];
          const TT bv = tile[(16 * t2s[jj] + c) * S::PS + prow];
          acc[jj] = M::run(av, bv, acc[jj]);
        }
      }
    }
    if constexpr (NARROW) {
#pragma unroll
      for (int jj = 0; jj < S::MAXPW; ++jj) {
#pragma unroll
        for (int i = 0; i < 4; ++i) wide[jj][i] += (double)acc[jj][i];
        acc[jj] = typename M::acc_t{0, 0, 0, 0};
      }
    }
  }
#pragma unroll
  for (int jj = 0; jj < S::MAXPW; ++jj) {
    const int j = w + 4 * jj;
    if (j < S::NPAIR) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double val;
        if constexpr (NARROW) val = wide[jj][i]; else val = (double)acc[jj][i];
        out[j * 256 + M::row(lane, i) * 16 + (lane & 15)] = val;
      }
    }
  }
}

// Float64 path: float64 basis values and products.  Mixed path: float32
// products, except for nodes with fewer than MIXED_WIDE_RATIO * calL points
// (near-interpolating nodes whose Gram is too ill-conditioned for a float32
// preconditioner), which take the float64 route.
constexpr int MIXED_WIDE_RATIO = 4;

// ROUTE 0: every chunk, float64 products.  ROUTE 1 / 2 (mixed path): only
// the chunks of nodes that take the float32 / float64 route; the two launches
// cover the level between them, and each sizes its LDS tile and registers for
// one element type.  Up to p = 6 the registers are held to 4 waves per SIMD
// for the float32 route and 3 for the float64 routes, which their LDS tiles
// allow: more waves in flight hide the batch loads and barriers behind other
// waves' matrix-core work.  Larger bases keep the compiler's allocation
// (held to 3 waves they would spill).
template <int P, typename TIN, typename TT, int ROUTE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P <= 6 ? (ROUTE == 1 ? 4 : 3) : 1)))
k_gram(LevelArgs a, double* __restrict__ partial) {
  using S = GramShape<P>;
  __shared__ TT tile[S::LP * S::PS];
  const uint32_t g = blockIdx.x;
  const uint32_t k = chunk_node(a.chunk_off, a.nnodes, g);
  const uint32_t node = a.node0 + k;
  const uint32_t nb = a.nt.begin[node], nc = a.nt.count[node];
  if (ROUTE != 0 && (nc >= (uint32_t)(MIXED_WIDE_RATIO * S::L)) != (ROUTE == 1)) return;   // the other launch's chunk
  const uint32_t start = nb + (g - a.chunk_off[k]) * CHUNK;
  const uint32_t end = min(nb + nc, start + (uint32_t)CHUNK);
  const double* geo = a.nt.geo + 6 * (size_t)node;
  double* out = partial + (size_t)g * S::NPAIR * 256;
  gram_body<P, TIN, TT>(a, tile, start, end, geo, out);
}

template <int P, typename TIN>
static void gram_launch(int path, const LevelArgs& a, double* partial, hipStream_t s) {
  dim3 grid(a.nchunks), block(256);
  if (path == FMT_PATH_MIXED) {
    hipLaunchKernelGGL((k_gram<P, TIN, float, 1>), grid, block, 0, s, a, partial);
    hipLaunchKernelGGL((k_gram<P, TIN, double, 2>), grid, block, 0, s, a, partial);
  } else {
    hipLaunchKernelGGL((k_gram<P, TIN, double, 0>), grid, block, 0, s, a, partial);
  }
}

template <int P>
static hipError_t gram_impl(int path, int dtype, const LevelArgs& a, double* partial, hipStream_t s) {
  if (a.nchunks == 0) return hipSuccess;
  if (dtype == FMT_F32) gram_launch<P, float>(path, a, partial, s);
  else gram_launch<P, double>(path, a, partial, s);
  return hipGetLastError();
}

hipError_t launch_gram(int p, int path, int dtype, const LevelArgs& a, double* partial, hipStream_t s) {
  FMT_DISPATCH_P(p, gram_impl, path, dtype, a, partial, s);
}

}  // namespace fmt
