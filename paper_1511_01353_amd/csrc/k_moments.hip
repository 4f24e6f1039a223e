// Power moments of one (node, chunk) work item on the float64 vector ALUs.
//
// The least-squares normal equations of Alg. 2 need G = Lambda^T Lambda and
// b = Lambda^T r.  With Lambda_alpha(u) = u^alpha / alpha!, every Gram entry
// is a power moment, G_{alpha beta} = M_{alpha+beta} / (alpha! beta!) with
// M_gamma = sum_i u_i^gamma over |gamma| <= 2p, and b_alpha =
// B_alpha / alpha! with B_alpha = sum_i r_i u_i^alpha.  There are only
// C(2p+3, 3) distinct moments (455 for p = 6) against calL(calL+1)/2 Gram
// entries (3570), so accumulating the moments takes several times fewer
// float64 operations per point than forming the Gram, and stays in float64.
//
// Layout of the work: a workgroup of NW waves takes one chunk; each wave owns
// a group of moment "runs" (fixed a, b; c = 0..cmax) chosen at compile time
// to balance the accumulator count.  A lane walks the chunk's points lane,
// lane+64, ... keeping its accumulators in registers; the 64 lanes are then
// summed through LDS in rounds of 16 accumulators, in a fixed order.
#include <utility>

#include "k_level.h"

namespace fmt {

// Position of (a, b, c) in the graded order (same rule as the basis).
__host__ __device__ constexpr int gidx(int a, int b, int c) {
  const int k = a + b + c;
  return k * (k + 1) * (k + 2) / 6 + (k - a) * (k - a + 1) / 2 + (k - a - b);
}

// MODE 0 (fit): moments M (|gamma| <= 2p), r-weighted moments B (|alpha| <= p)
// and sum r^2.  MODE 1 (refinement): B only, weighted by r' = r - Lambda F.
template <int P, int MODE>
struct MomentPlan {
  static constexpr int P2 = 2 * P;
  static constexpr int NM = MODE == 0 ? basis_size(P2) : 0;
  static constexpr int NB = basis_size(P);
  static constexpr int NOUT = NM + NB + (MODE == 0 ? 1 : 0);
  static constexpr int NI_M = MODE == 0 ? (P2 + 1) * (P2 + 2) / 2 : 0;
  static constexpr int NI_B = (P + 1) * (P + 2) / 2;
  static constexpr int NI = NI_M + NI_B + (MODE == 0 ? 1 : 0);
  static constexpr int CAP = 64;   // accumulators per lane budget
  static constexpr int NW_MAX = MODE == 0 ? 8 : 2;
  static constexpr int NG_MIN = (NOUT + CAP - 1) / CAP;
  static constexpr int NW = NG_MIN < NW_MAX ? (NG_MIN < 1 ? 1 : NG_MIN) : NW_MAX;
  static constexpr int NPASS = (NG_MIN + NW - 1) / NW;
  static constexpr int NG = NW * NPASS;

  // items: kind 0 = M run, 1 = B run, 2 = sum r^2
  int kind[NI], ia[NI], ib[NI], len[NI], slot[NI], out0[NI];
  int gcount[NG], gitem[NG][NI], load[NG];
  static constexpr int OUTW = CAP + 2 * P + 8;
  int outmap[NG][OUTW];   // output position of each accumulator slot (-1: none)

  constexpr MomentPlan() : kind(), ia(), ib(), len(), slot(), out0(), gcount(), gitem(), load(), outmap() {
    int n = 0;
    if (MODE == 0) {
      for (int a = 0; a <= P2; ++a)
        for (int b = 0; a + b <= P2; ++b) {
          kind[n] = 0; ia[n] = a; ib[n] = b; len[n] = P2 - a - b + 1; out0[n] = 0; ++n;
        }
    }
    for (int a = 0; a <= P; ++a)
      for (int b = 0; a + b <= P; ++b) {
        kind[n] = 1; ia[n] = a; ib[n] = b; len[n] = P - a - b + 1; out0[n] = NM; ++n;
      }
    if (MODE == 0) { kind[n] = 2; ia[n] = 0; ib[n] = 0; len[n] = 1; out0[n] = NM + NB; ++n; }
    // longest runs first, each to the least loaded group
    int order[NI] = {};
    for (int i = 0; i < NI; ++i) order[i] = i;
    for (int i = 1; i < NI; ++i) {
      int v = order[i], j = i;
      while (j > 0 && len[order[j - 1]] < len[v]) { order[j] = order[j - 1]; --j; }
      order[j] = v;
    }
    for (int g = 0; g < NG; ++g) { load[g] = 0; gcount[g] = 0; }
    for (int t = 0; t < NI; ++t) {
      const int i = order[t];
      int best = 0;
      for (int g = 1; g < NG; ++g)
        if (load[g] < load[best]) best = g;
      slot[i] = load[best];
      load[best] += len[i];
      gitem[best][gcount[best]++] = i;
    }
    for (int g = 0; g < NG; ++g)
      for (int q = 0; q < OUTW; ++q) outmap[g][q] = -1;
    for (int g = 0; g < NG; ++g)
      for (int t = 0; t < gcount[g]; ++t) {
        const int i = gitem[g][t];
        for (int c = 0; c < len[i]; ++c) {
          const int k = ia[i] + ib[i] + c;
          const int pos = k * (k + 1) * (k + 2) / 6 + (k - ia[i]) * (k - ia[i] + 1) / 2 + (k - ia[i] - ib[i]);
          outmap[g][slot[i] + c] = kind[i] == 2 ? out0[i] : out0[i] + pos;
        }
      }
  }
};

template <int P, int MODE>
struct Plan {
  static constexpr MomentPlan<P, MODE> v{};
};

size_t moment_partial_doubles(int p) { return basis_size(2 * p) + basis_size(p) + 1; }
size_t moment_refine_doubles(int p) { return basis_size(p); }

// Accumulate item I (compile-time) for one point: a run acc[s + c] += h w^c.
template <int S, int NA, int P2, size_t... C>
__device__ __forceinline__ void acc_run(std::index_sequence<C...>, double h, const double (&pw)[P2 + 1],
                                        double (&acc)[NA]) {
  ((acc[S + (int)C] += h * pw[C]), ...);
}

template <int P, int MODE, int I, int NA>
__device__ __forceinline__ void accumulate_item(const double (&pu)[2 * P + 1], const double (&pv)[2 * P + 1],
                                                const double (&pw)[2 * P + 1], double wt, double (&acc)[NA]) {
  constexpr const MomentPlan<P, MODE>& M = Plan<P, MODE>::v;
  constexpr int k = M.kind[I], s = M.slot[I], n = M.len[I], ea = M.ia[I], eb = M.ib[I];
  if constexpr (k == 2) {
    acc[s] += wt * wt;
  } else {
    double h = pu[ea] * pv[eb];
    if constexpr (k == 1) h *= wt;
    acc_run<s, NA, 2 * P>(std::make_index_sequence<n>{}, h, pw, acc);
  }
}

template <int P, int MODE, int G, int NA, size_t... T>
__device__ __forceinline__ void accumulate(std::index_sequence<T...>, const double (&pu)[2 * P + 1],
                                           const double (&pv)[2 * P + 1], const double (&pw)[2 * P + 1], double wt,
                                           double (&acc)[NA]) {
  (accumulate_item<P, MODE, Plan<P, MODE>::v.gitem[G][T], NA>(pu, pv, pw, wt, acc), ...);
}

// red: 16 x 65 doubles of LDS owned by this wave.
template <int P, int MODE, int G, typename TIN>
__device__ __forceinline__ void moments_group(const LevelArgs& a, uint32_t start, uint32_t end, const double* geo,
                                              const double* rp, double* red, double* out) {
  constexpr const MomentPlan<P, MODE>& M = Plan<P, MODE>::v;
  constexpr int NA = M.load[G] > 0 ? M.load[G] : 1;
  static_assert(NA <= MomentPlan<P, MODE>::OUTW, "a moment group exceeds the output map");
  constexpr int P2 = 2 * P;
  const int lane = threadIdx.x & 63;
  const double cx = geo[0], cy = geo[1], cz = geo[2], sx = geo[3], sy = geo[4], sz = geo[5];
  double acc[NA];
#pragma unroll
  for (int s = 0; s < NA; ++s) acc[s] = 0.0;
  // the next point's data is loaded one iteration ahead (index clamped into
  // the chunk), so its latency overlaps this point's arithmetic
  double nx = 0.0, ny = 0.0, nz = 0.0, nw = 0.0;
  if (start + lane < end) {
    load_point<TIN>(a.px, a.py, a.pz, start + lane, nx, ny, nz);
    nw = MODE == 1 ? rp[lane] : a.r[start + lane];
  }
#pragma unroll 1
  for (uint32_t i = start + lane; i < end; i += 64) {
    const double x = nx, y = ny, z = nz, wt = nw;
    {
      const uint32_t j = min(i + 64, end - 1);
      load_point<TIN>(a.px, a.py, a.pz, j, nx, ny, nz);
      nw = MODE == 1 ? rp[j - start] : a.r[j];
    }
    const double u = (x - cx) * sx, v = (y - cy) * sy, w = (z - cz) * sz;
    double pu[P2 + 1], pv[P2 + 1], pw[P2 + 1];
    pu[0] = pv[0] = pw[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= P2; ++k) {
      pu[k] = pu[k - 1] * u;
      pv[k] = pv[k - 1] * v;
      pw[k] = pw[k - 1] * w;
    }
    accumulate<P, MODE, G, NA>(std::make_index_sequence<M.gcount[G]>{}, pu, pv, pw, wt, acc);
  }
  // sum over the 64 lanes: rounds of 16 accumulators through LDS; lane l
  // adds column block (l / 16) of row (l % 16), then the 4 partials combine
#pragma unroll
  for (int s0 = 0; s0 < NA; s0 += 16) {
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (s0 + q < NA) red[q * 65 + lane] = acc[s0 + q];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int row = lane & 15, cb = lane >> 4;
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) t += red[row * 65 + cb * 16 + c];
    t += __shfl_xor(t, 16);
    t += __shfl_xor(t, 32);
    if (cb == 0 && s0 + row < NA) {
      const int o = Plan<P, MODE>::v.outmap[G][s0 + row];
      if (o >= 0) out[o] = t;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <int P, int MODE, typename TIN, int G = 0>
__device__ __forceinline__ void dispatch_group(int g, const LevelArgs& a, uint32_t start, uint32_t end,
                                               const double* geo, const double* rp, double* red, double* out) {
  if constexpr (G < MomentPlan<P, MODE>::NG) {
    if (g == G) moments_group<P, MODE, G, TIN>(a, start, end, geo, rp, red, out);
    else dispatch_group<P, MODE, TIN, G + 1>(g, a, start, end, geo, rp, red, out);
  }
}

template <int P, int MODE, typename TIN>
__global__ void __launch_bounds__((MomentPlan<P, MODE>::NW * 64)) k_moments(LevelArgs a, double* __restrict__ part) {
  using MP = MomentPlan<P, MODE>;
  constexpr int L = basis_size(P);
  __shared__ double rp[MODE == 1 ? CHUNK : 1];   // r' = r - Lambda F of the chunk's points
  __shared__ double red[MP::NW][16 * 65];
  const uint32_t g = blockIdx.x;
  const uint32_t k = chunk_node(a.chunk_off, a.nnodes, g);
  const uint32_t node = a.node0 + k;
  const uint32_t nb = a.nt.begin[node], nc = a.nt.count[node];
  const uint32_t start = nb + (g - a.chunk_off[k]) * CHUNK;
  const uint32_t end = min(nb + nc, start + (uint32_t)CHUNK);
  const double* geo = a.nt.geo + 6 * (size_t)node;
  if constexpr (MODE == 1) {
    if (!(a.nt.flags[node] & FLAG_REFINE)) return;   // whole workgroup: its node needs no refinement
    // r' once per point, four points per thread at a time; the node's
    // coefficients are wave-uniform and read with scalar loads (read-only
    // constant address space), so they take no vector registers
    typedef const double __attribute__((address_space(4))) cdouble;
    const cdouble* F = (const cdouble*)(a.nt.coef + (size_t)node * L);
    const double cx = geo[0], cy = geo[1], cz = geo[2], sx = geo[3], sy = geo[4], sz = geo[5];
    constexpr int NT = MP::NW * 64, NPT = 4;
    for (uint32_t i0 = start + threadIdx.x; i0 < end; i0 += NPT * NT) {
      double u[NPT], v[NPT], w[NPT], val[NPT];
#pragma unroll
      for (int q = 0; q < NPT; ++q) {
        const uint32_t i = min(i0 + q * NT, end - 1);   // tail lanes repeat a point and do not store
        double x, y, z;
        load_point<TIN>(a.px, a.py, a.pz, i, x, y, z);
        u[q] = (x - cx) * sx;
        v[q] = (y - cy) * sy;
        w[q] = (z - cz) * sz;
      }
      poly_eval_multi<P, NPT>(F, u, v, w, val);
#pragma unroll
      for (int q = 0; q < NPT; ++q) {
        const uint32_t i = i0 + q * NT;
        if (i < end) rp[i - start] = a.r[i] - val[q];
      }
    }
    __syncthreads();
  }
  double* out = part + (size_t)g * MP::NOUT;
  const int w = threadIdx.x >> 6;
  for (int pass = 0; pass < MP::NPASS; ++pass)
    dispatch_group<P, MODE, TIN>(pass * MP::NW + w, a, start, end, geo, rp, red[w], out);
}

template <int P>
static hipError_t moments_impl(int mode, int dtype, const LevelArgs& a, double* part, hipStream_t s) {
  if (a.nchunks == 0) return hipSuccess;
  dim3 grid(a.nchunks);
  if (mode == 0) {
    dim3 block(MomentPlan<P, 0>::NW * 64);
    if (dtype == FMT_F32) hipLaunchKernelGGL((k_moments<P, 0, float>), grid, block, 0, s, a, part);
    else hipLaunchKernelGGL((k_moments<P, 0, double>), grid, block, 0, s, a, part);
  } else {
    dim3 block(MomentPlan<P, 1>::NW * 64);
    if (dtype == FMT_F32) hipLaunchKernelGGL((k_moments<P, 1, float>), grid, block, 0, s, a, part);
    else hipLaunchKernelGGL((k_moments<P, 1, double>), grid, block, 0, s, a, part);
  }
  return hipGetLastError();
}

hipError_t launch_moments(int p, int mode, int dtype, const LevelArgs& a, double* part, hipStream_t s) {
  FMT_DISPATCH_P(p, moments_impl, mode, dtype, a, part, s);
}

}  // namespace fmt
