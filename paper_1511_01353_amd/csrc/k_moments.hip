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
// Layout of the work: a workgroup of NW * SPLIT waves takes one chunk,
// whose points (coordinates and weight) it first stages in LDS with all of
// its loads in flight at once.  Each wave owns a group of moment "runs"
// (fixed a, b; c = 0..cmax) chosen at compile time to balance the
// accumulator count, and one of SPLIT slices of the chunk's points.  A lane
// walks its slice's points keeping its accumulators in registers; the 64
// lanes are then summed through LDS in rounds of RROWS accumulators, and the
// slices in a fixed order.
//
// Modes: 0 = M, B and sum r^2 of a level's nodes; 1 = B of the refinement
// residual r' = r - Lambda F; 2 = B only (the power moments M of the node come
// from the moment pyramid); 3 = M only, over the cells of the pyramid's
// finest level; 4 = B only as mode 2 for the nodes with fewer than
// SMALL_NODE points (mode 2 takes the others): two waves per chunk reading
// their points straight from memory (no staging, so many more workgroups
// share a compute unit); 5 = mode 0 for the nodes with fewer than
// SMALL_NODE points (mode 0 then takes the others; p <= SMALL_M_P): a
// staging buffer for SMALL_NODE points and reduction rounds of 8
// accumulators, 20 KB of LDS against mode 0's 40 KB (levels of tens of
// thousands of small nodes in a batch; measured with mode 0 in eight-wave
// workgroups, when it fitted one workgroup per compute unit).  At p = 5
// and 6 the split cost more than it saved, and mode 0 keeps every node.
#include <utility>

#include "k_level.h"

namespace fmt {

// Position of (a, b, c) in the graded order (same rule as the basis).
__host__ __device__ constexpr int gidx(int a, int b, int c) {
  const int k = a + b + c;
  return k * (k + 1) * (k + 2) / 6 + (k - a) * (k - a + 1) / 2 + (k - a - b);
}

// highest order whose small nodes take mode 5
constexpr int SMALL_M_P = 4;

template <int P, int MODE>
struct MomentPlan {
  static constexpr bool HAS_M = MODE == 0 || MODE == 3 || MODE == 5;
  static constexpr bool HAS_B = MODE != 3;
  static constexpr bool HAS_RR = MODE == 0 || MODE == 5;
  static constexpr int P2 = 2 * P;
  static constexpr int NM = HAS_M ? basis_size(P2) : 0;
  static constexpr int NB = HAS_B ? basis_size(P) : 0;
  static constexpr int NOUT = NM + NB + (HAS_RR ? 1 : 0);
  static constexpr int NI_M = HAS_M ? (P2 + 1) * (P2 + 2) / 2 : 0;
  static constexpr int NI_B = HAS_B ? (P + 1) * (P + 2) / 2 : 0;
  static constexpr int NI = NI_M + NI_B + (HAS_RR ? 1 : 0);
  static constexpr int CAP = 64;   // accumulators per lane budget
  // waves per workgroup, measured up to p = 8: four (mode 4: two).
  // Workgroups of eight waves were ~1% slower per float64 fit in the B
  // passes (modes 1 and 2: four point slices of two groups of runs instead
  // of two), 6% slower per mixed fit (whose refinement sweeps every node)
  // and 2% slower per batch in mode 0 (whose 70 KB tile then left one
  // workgroup per compute unit); sixteen were 7% slower.  Mode 3 runs over
  // many small cells, where small workgroups let more of them share a
  // compute unit.  The large bases (p > 8) keep eight waves.
  static constexpr int WAVES = MODE == 4 ? 2 : (P > 8 ? 8 : 4);
  static constexpr int NW_MAX = HAS_M ? WAVES : 2;
  static constexpr int NG_MIN = (NOUT + CAP - 1) / CAP;
  static constexpr int NW = NG_MIN < NW_MAX ? (NG_MIN < 1 ? 1 : NG_MIN) : NW_MAX;
  static constexpr int NPASS = (NG_MIN + NW - 1) / NW;
  static constexpr int NG = NW * NPASS;
  // with few groups, point slices keep the workgroup's waves busy
  static constexpr int SPLIT = NW >= WAVES ? 1 : WAVES / NW;
  static constexpr int NTHR = NW * SPLIT * 64;
  // accumulators per reduction round: 16 when the reduction buffer can
  // share the LDS of the staged points (one pass over the groups), else 8
  static constexpr int RROWS = HAS_M && NPASS == 1 && MODE != 5 ? 16 : 8;
  static constexpr int PMAX = HAS_M ? P2 : P;    // highest power used

  // items: kind 0 = M run, 1 = B run, 2 = sum r^2
  int kind[NI], ia[NI], ib[NI], len[NI], slot[NI], out0[NI];
  int gcount[NG], gitem[NG][NI], load[NG];
  static constexpr int OUTW = CAP + 2 * P + 8;
  int outmap[NG][OUTW];   // output position of each accumulator slot (-1: none)

  constexpr MomentPlan() : kind(), ia(), ib(), len(), slot(), out0(), gcount(), gitem(), load(), outmap() {
    int n = 0;
    if (HAS_M) {
      for (int a = 0; a <= P2; ++a)
        for (int b = 0; a + b <= P2; ++b) {
          kind[n] = 0; ia[n] = a; ib[n] = b; len[n] = P2 - a - b + 1; out0[n] = 0; ++n;
        }
    }
    if (HAS_B) {
      for (int a = 0; a <= P; ++a)
        for (int b = 0; a + b <= P; ++b) {
          kind[n] = 1; ia[n] = a; ib[n] = b; len[n] = P - a - b + 1; out0[n] = NM; ++n;
        }
    }
    if (HAS_RR) { kind[n] = 2; ia[n] = 0; ib[n] = 0; len[n] = 1; out0[n] = NM + NB; ++n; }
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

#ifndef FMT_MOMENTS_WIDE_P
size_t moment_partial_doubles(int p) { return basis_size(2 * p) + basis_size(p) + 1; }
size_t moment_refine_doubles(int p) { return basis_size(p); }
size_t moment_base_doubles(int p) { return basis_size(2 * p); }
#endif

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
    if constexpr (k == 1 && MomentPlan<P, MODE>::HAS_M) h *= wt;
    acc_run<s, NA, 2 * P>(std::make_index_sequence<n>{}, h, pw, acc);
  }
}

template <int P, int MODE, int G, int NA, size_t... T>
__device__ __forceinline__ void accumulate(std::index_sequence<T...>, const double (&pu)[2 * P + 1],
                                           const double (&pv)[2 * P + 1], const double (&pw)[2 * P + 1], double wt,
                                           double (&acc)[NA]) {
  (accumulate_item<P, MODE, Plan<P, MODE>::v.gitem[G][T], NA>(pu, pv, pw, wt, acc), ...);
}

// The chunk's points staged in LDS: coordinates in the input type, and the
// weight (r, or r' in mode 1) in float64 except in mode 3; room for CAP
// points (a chunk; mode 5's nodes have fewer than SMALL_NODE).
template <int MODE, typename TIN>
struct Staged {
  static constexpr bool HAS_W = MODE != 3;
  static constexpr bool IN_LDS = MODE != 4;   // mode 4 reads the points where they are
  static constexpr uint32_t CAP = MODE == 5 ? (uint32_t)SMALL_NODE : (uint32_t)CHUNK;
  static constexpr size_t BYTES = IN_LDS ? (size_t)CAP * (3 * sizeof(TIN) + (HAS_W ? sizeof(double) : 0)) : 0;
  const TIN* x;
  const TIN* y;
  const TIN* z;
  const double* w;
  __device__ Staged(char* base) {
    TIN* p = reinterpret_cast<TIN*>(base);
    x = p;
    y = p + CAP;
    z = p + 2 * CAP;
    w = reinterpret_cast<const double*>(p + 3 * CAP);
  }
  __device__ Staged(const TIN* gx, const TIN* gy, const TIN* gz, const double* gw) : x(gx), y(gy), z(gz), w(gw) {}
};

// One wave's share of a chunk: group G of the runs over slice `slice` of the
// n staged points.  red: RROWS x 65 doubles of LDS owned by this wave; with
// ALIAS it overlays the staged points, so every wave first finishes its
// points (workgroup barrier).  The lane sums go to out[] (one slice) or to
// comb[slice][] (several slices, summed by the caller).
template <int P, int MODE, int G, typename TIN, bool ALIAS>
__device__ __forceinline__ void moments_group(const Staged<MODE, TIN>& st, uint32_t n, int slice, const double* geo,
                                              double* red, double* out) {
  using MP = MomentPlan<P, MODE>;
  constexpr const MP& M = Plan<P, MODE>::v;
  constexpr int NA = M.load[G] > 0 ? M.load[G] : 1;
  static_assert(NA <= MP::OUTW, "a moment group exceeds the output map");
  constexpr int P2 = 2 * P, R = MP::RROWS, STEP = 64 * MP::SPLIT;
  const int lane = threadIdx.x & 63;
  const double cx = geo[0], cy = geo[1], cz = geo[2], sx = geo[3], sy = geo[4], sz = geo[5];
  double acc[NA];
#pragma unroll
  for (int s = 0; s < NA; ++s) acc[s] = 0.0;
#pragma unroll 1
  for (uint32_t j = (uint32_t)(slice * 64 + lane); j < n; j += STEP) {
    const double u = ((double)st.x[j] - cx) * sx, v = ((double)st.y[j] - cy) * sy, w = ((double)st.z[j] - cz) * sz;
    double wt = 0.0;
    if constexpr (Staged<MODE, TIN>::HAS_W) wt = st.w[j];
    double pu[P2 + 1], pv[P2 + 1], pw[P2 + 1];
    // the B-only modes fold the weight into the w powers (one product per
    // run fewer); the others weight the B runs' leading product
    pu[0] = pv[0] = 1.0;
    pw[0] = MP::HAS_M ? 1.0 : wt;
#pragma unroll
    for (int k = 1; k <= MP::PMAX; ++k) {
      pu[k] = pu[k - 1] * u;
      pv[k] = pv[k - 1] * v;
      pw[k] = pw[k - 1] * w;
    }
    accumulate<P, MODE, G, NA>(std::make_index_sequence<M.gcount[G]>{}, pu, pv, pw, wt, acc);
  }
  if constexpr (ALIAS) __syncthreads();
  // sum over the 64 lanes: rounds of R accumulators through LDS; lane l adds
  // column block (l / R) of row (l % R), then the 64 / R partials combine
#pragma unroll
  for (int s0 = 0; s0 < NA; s0 += R) {
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (s0 + q < NA) red[q * 65 + lane] = acc[s0 + q];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int row = lane % R, cb = lane / R;
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < R; ++c) t += red[row * 65 + cb * R + c];
#pragma unroll
    for (int off = R; off < 64; off <<= 1) t += __shfl_xor(t, off);
    if (cb == 0 && s0 + row < NA) {
      const int o = Plan<P, MODE>::v.outmap[G][s0 + row];
      if (o >= 0) out[(MP::SPLIT > 1 ? slice * MP::NOUT : 0) + o] = t;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <int P, int MODE, typename TIN, bool ALIAS, int G = 0>
__device__ __forceinline__ void dispatch_group(int g, const Staged<MODE, TIN>& st, uint32_t n, int slice,
                                               const double* geo, double* red, double* out) {
  if constexpr (G < MomentPlan<P, MODE>::NG) {
    if (g == G) moments_group<P, MODE, G, TIN, ALIAS>(st, n, slice, geo, red, out);
    else dispatch_group<P, MODE, TIN, ALIAS, G + 1>(g, st, n, slice, geo, red, out);
  }
}

// The base-moment pass (mode 3) holds its registers to 3 waves per SIMD up
// to p = 6 (its LDS tile allows 3 workgroups per CU; the compiler's own
// allocation gives 2): 18% faster at p = 6.
template <int P, int MODE, typename TIN>
__global__ void __launch_bounds__((MomentPlan<P, MODE>::NTHR))
__attribute__((amdgpu_waves_per_eu(MODE == 3 && P <= 6 ? 3 : 1)))
k_moments(LevelArgs a, double* __restrict__ part) {
  using MP = MomentPlan<P, MODE>;
  using ST = Staged<MODE, TIN>;
  constexpr int L = basis_size(P), NT = MP::NTHR;
  // one pass over the groups: the reduction buffers overlay the staged points
  constexpr bool ALIAS = MP::NPASS == 1;
  constexpr size_t RED_B = (size_t)MP::NW * MP::SPLIT * MP::RROWS * 65 * sizeof(double);
  constexpr size_t SMEM_B = ALIAS ? (ST::BYTES > RED_B ? ST::BYTES : RED_B) : ST::BYTES + RED_B;
  __shared__ __attribute__((aligned(16))) char smem[SMEM_B];
  __shared__ double comb[MP::SPLIT > 1 ? MP::SPLIT * MP::NOUT : 1];
  uint32_t g = blockIdx.x, k;
  if (MODE == 1 && a.sel) {
    // the late refinement's sweep over the listed nodes
    if (!listed_chunk(a, blockIdx.x, k, g)) return;
  } else {
    // the grid may be an upper bound on the chunk count (pyramid cells)
    if (g >= a.chunk_off[a.nnodes]) return;
    k = chunk_node(a.chunk_off, a.nnodes, g);
  }
  const uint32_t node = a.node0 + k;
  const uint32_t nb = a.nt.begin[node], nc = a.nt.count[node];
  const uint32_t start = nb + (g - a.chunk_off[k]) * CHUNK;
  const uint32_t n = min(nb + nc, start + (uint32_t)CHUNK) - start;
  const double* geo = a.nt.geo + 6 * (size_t)node;
  const uint32_t fj = blockIdx.y;   // field of a multi-field launch
  const double* rin = a.r + (size_t)fj * a.rstride;
  if constexpr (MODE == 0 || MODE == 2 || MODE == 4 || MODE == 5) {
    // a level split between the pyramid's nodes (modes 2, 4) and the others
    constexpr bool PYR_NODES = MODE == 2 || MODE == 4;
    if (a.pyr_tab && pyramid_covers(a.pyr_tab[PYR_TAB_WORDS * a.nt.problem[node] + 1], a.level) != PYR_NODES) return;
  }
  if constexpr (MODE == 0 || MODE == 5) {
    if (a.only_flag && !(a.nt.flags[node] & a.only_flag)) return;   // not this pass's node
  }
  // modes 2 and 4, and 0 and 5 (p <= SMALL_M_P), split the nodes by size
  if constexpr (MODE == 2 || (MODE == 0 && P <= SMALL_M_P)) {
    if (nc < SMALL_NODE) return;
  }
  if constexpr (MODE == 4 || MODE == 5) {
    if (nc >= SMALL_NODE) return;
  }
  if constexpr (MODE == 1) {
    if (!(a.nt.flags[node] & FLAG_REFINE)) return;   // whole workgroup: its node needs no refinement
  }
  TIN* sxw = reinterpret_cast<TIN*>(smem);
  double* sww = reinterpret_cast<double*>(sxw + 3 * ST::CAP);
  const TIN* gx = (const TIN*)a.px + start;
  const TIN* gy = (const TIN*)a.py + start;
  const TIN* gz = (const TIN*)a.pz + start;
  constexpr int NPT = 4;   // points per thread per round: all their loads are issued together
  if constexpr (MODE == 1) {
    // r' = r - Lambda F once per point; the node's coefficients are
    // wave-uniform and read with scalar loads (read-only constant address
    // space), so they take no vector registers
    typedef const double __attribute__((address_space(4))) cdouble;
    const cdouble* F = (const cdouble*)(a.nt.coef + (size_t)fj * a.cstride + (size_t)node * L);
    const double cx = geo[0], cy = geo[1], cz = geo[2], sx = geo[3], sy = geo[4], sz = geo[5];
    for (uint32_t i0 = threadIdx.x; i0 < n; i0 += NPT * NT) {
      TIN vx[NPT], vy[NPT], vz[NPT];
      double u[NPT], v[NPT], w[NPT], val[NPT], r[NPT];
#pragma unroll
      for (int q = 0; q < NPT; ++q) {
        const uint32_t i = min(i0 + q * NT, n - 1);   // tail lanes repeat a point and do not store
        vx[q] = gx[i];
        vy[q] = gy[i];
        vz[q] = gz[i];
        r[q] = rin[start + i];
      }
#pragma unroll
      for (int q = 0; q < NPT; ++q) {
        u[q] = ((double)vx[q] - cx) * sx;
        v[q] = ((double)vy[q] - cy) * sy;
        w[q] = ((double)vz[q] - cz) * sz;
      }
      if (a.sweep_current) {
        // the residual update already subtracted Lambda F
#pragma unroll
        for (int q = 0; q < NPT; ++q) val[q] = 0.0;
      } else {
        poly_eval_multi<P, NPT>(F, u, v, w, val);
      }
#pragma unroll
      for (int q = 0; q < NPT; ++q) {
        const uint32_t i = i0 + q * NT;
        if (i < n) {
          sxw[i] = vx[q];
          sxw[ST::CAP + i] = vy[q];
          sxw[2 * ST::CAP + i] = vz[q];
          sww[i] = r[q] - val[q];
        }
      }
    }
  } else if constexpr (ST::IN_LDS) {
    for (uint32_t i0 = threadIdx.x; i0 < n; i0 += NPT * NT) {
      TIN vx[NPT], vy[NPT], vz[NPT];
      double r[NPT];
#pragma unroll
      for (int q = 0; q < NPT; ++q) {
        const uint32_t i = min(i0 + q * NT, n - 1);
        vx[q] = gx[i];
        vy[q] = gy[i];
        vz[q] = gz[i];
        if constexpr (ST::HAS_W) r[q] = rin[start + i];
      }
#pragma unroll
      for (int q = 0; q < NPT; ++q) {
        const uint32_t i = i0 + q * NT;
        if (i < n) {
          sxw[i] = vx[q];
          sxw[ST::CAP + i] = vy[q];
          sxw[2 * ST::CAP + i] = vz[q];
          if constexpr (ST::HAS_W) sww[i] = r[q];
        }
      }
    }
  }
  __syncthreads();
  const ST st = [&] {
    if constexpr (ST::IN_LDS) return ST(smem);
    else return ST(gx, gy, gz, rin + start);
  }();
  double* out = part + ((size_t)fj * a.nchunks + g) * MP::NOUT;
  const int w = threadIdx.x >> 6;
  const int grp = w % MP::NW, slice = w / MP::NW;
  double* red = reinterpret_cast<double*>(smem + (ALIAS ? 0 : ST::BYTES)) + (size_t)w * MP::RROWS * 65;
  double* dst = MP::SPLIT > 1 ? comb : out;
  for (int pass = 0; pass < MP::NPASS; ++pass)
    dispatch_group<P, MODE, TIN, ALIAS>(pass * MP::NW + grp, st, n, slice, geo, red, dst);
  if constexpr (MP::SPLIT > 1) {
    __syncthreads();
    for (int o = threadIdx.x; o < MP::NOUT; o += NT) {
      double t = comb[o];
#pragma unroll
      for (int q = 1; q < MP::SPLIT; ++q) t += comb[q * MP::NOUT + o];
      out[o] = t;
    }
  }
}

template <int P, int MODE>
static void launch_mode(int dtype, const LevelArgs& a, double* part, hipStream_t s) {
  dim3 grid(MODE == 1 && a.sel ? a.nsel_chunks : a.nchunks, field_rows(a)), block(MomentPlan<P, MODE>::NTHR);
  if (grid.x == 0) return;
  if (dtype == FMT_F32) hipLaunchKernelGGL((k_moments<P, MODE, float>), grid, block, 0, s, a, part);
  else hipLaunchKernelGGL((k_moments<P, MODE, double>), grid, block, 0, s, a, part);
}

template <int P>
static hipError_t moments_impl(int mode, int dtype, const LevelArgs& a, double* part, hipStream_t s) {
  if (a.nchunks == 0) return hipSuccess;
  if constexpr (P > 8) {
    // large bases: per-level moments (mode 0) and the refinement sweep (mode 1)
    switch (mode) {
      case 0: launch_mode<P, 0>(dtype, a, part, s); break;
      case 1: launch_mode<P, 1>(dtype, a, part, s); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (mode) {
      case 0:
        // up to SMALL_M_P the larger nodes in mode 0, those under SMALL_NODE
        // points in mode 5
        if (P > SMALL_M_P || a.nsmall == UINT32_MAX || a.nsmall < a.nnodes) launch_mode<P, 0>(dtype, a, part, s);
        if (P <= SMALL_M_P && a.nsmall > 0) launch_mode<P, 5>(dtype, a, part, s);
        break;
      case 1: launch_mode<P, 1>(dtype, a, part, s); break;
      case 2: launch_mode<P, 2>(dtype, a, part, s); break;
      case 3: launch_mode<P, 3>(dtype, a, part, s); break;
      case 4: launch_mode<P, 4>(dtype, a, part, s); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

#ifndef FMT_MOMENTS_WIDE_P
hipError_t launch_moments(int p, int mode, int dtype, const LevelArgs& a, double* part, hipStream_t s) {
  switch (p) {
    case 10: return launch_moments_p10(mode, dtype, a, part, s);
    case 12: return launch_moments_p12(mode, dtype, a, part, s);
    case 14: return launch_moments_p14(mode, dtype, a, part, s);
    default: break;
  }
  FMT_DISPATCH_P(p, moments_impl, mode, dtype, a, part, s);
}
#else
// this translation unit: the kernels of one large order only
#define FMT_MOMENTS_CAT2(a, b) a##b
#define FMT_MOMENTS_CAT(a, b) FMT_MOMENTS_CAT2(a, b)
hipError_t FMT_MOMENTS_CAT(launch_moments_p, FMT_MOMENTS_WIDE_P)(int mode, int dtype, const LevelArgs& a,
                                                                  double* part, hipStream_t s) {
  return moments_impl<FMT_MOMENTS_WIDE_P>(mode, dtype, a, part, s);
}
#endif

}  // namespace fmt
