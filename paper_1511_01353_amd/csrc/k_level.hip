// Per-node solve, refinement, residual update and child activation of one
// octree level (Alg. 1 and Alg. 2), plus the topology step that lays out the
// next level's nodes.
#include "k_level.h"
#include "k_ldl.h"

namespace fmt {

size_t factor_doubles(int p) {
  const int L = basis_size(p);
  const int T = (L + 15) / 16;
  return (size_t)T * (T + 1) / 2 * 256 + 3 * (size_t)L;
}

// ---------------------------------------------------------------------------
// Right-looking blocked LDL^T factorisation of the unit-diagonal matrix A
// (blocked storage, padding rows/columns set to the identity), in place, by
// all 256 threads.  Afterwards the strictly lower part of A holds the unit
// lower factor L; the diagonal and the strict upper part of every diagonal
// block hold 0, and D lives in dv (with iv = D^-1, 0 where deflated).  The
// zeros let the triangular solves run without per-step masks.  The 16 words
// after the blocked storage, A[WORDS .. WORDS + 15], are a zero row (the
// caller zeroes them).  Per block column J:
//   (a) the diagonal block and the panel below it in one right-looking pass:
//       each wave that holds panel rows (up to 48, in lanes 16..63) also
//       holds the block's 16 rows in lanes 0..15 and factors the block
//       alongside (redundantly; wave 0 stores it once the other waves have
//       read it).  At step k lanes 0..15 publish column k of the block in
//       LDS and every lane reads the pivot and the entries A(c, k), c > k, as
//       broadcasts; each lane scales its entry k by 1/d_k (its L(row, k)) and
//       updates its entries c > k.  Entries above the diagonal of a block row
//       collect values that are never read, so the updates need no mask;
//   (b) the trailing blocks take A_IK -= (L_IJ D_J) L_KJ^T on float64 MFMA,
//       with lookahead: block column J+1 right away, the blocks right of it
//       by the waves that do not take part in (a) for column J+1, while the
//       others factor it.
// Pivots at or below PIVOT_EPS are deflated: their inverse is 0, so their
// column of L is 0 and the solve gives that unknown 0.
// ---------------------------------------------------------------------------

// A_IK -= (L_IJ D_J) L_KJ^T for one block pair, by one wave on MFMA.
__device__ __forceinline__ void trailing_block(double* A, const double* dv, int J, int I, int K, int lane) {
  double* out = A + bidx(I, K);
  const double* li = A + bidx(I, J);
  const double* lk = A + bidx(K, J);
  solve_d4 acc;
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = out[bel((lane >> 4) + 4 * q, lane & 15)];
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) {
    const int kk = 4 * s4 + (lane >> 4);
    const double av = -li[bel(lane & 15, kk)] * dv[16 * J + kk];
    const double bv = lk[bel(lane & 15, kk)];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) out[bel((lane >> 4) + 4 * q, lane & 15)] = acc[q];
}

// Block pair number p (0-based) of the lower triangle of block columns
// K0 .. T-1, column by column: (I, K) with K0 <= K <= I < T.
__device__ __forceinline__ void pair_of(int p, int K0, int T, int& I, int& K) {
  K = K0;
  while (p >= T - K) {
    p -= T - K;
    ++K;
  }
  I = K + p;
}

template <int L>
__device__ __forceinline__ void ldl_blocked(double* A, double* dv, double* iv) {
  using S = BlockShape<L>;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  static_assert(S::LP - 16 <= 4 * 48, "the panel rows exceed the lanes of four waves");
  __shared__ double colbuf[4 * 16];
  for (int J = 0; J < S::T; ++J) {
    // waves 0 .. nbusy-1 factor column J (wave w > 0 only if it holds panel rows)
    int nbusy = 1;
    while (nbusy < 4 && 16 * (J + 1) + 48 * nbusy < S::LP) ++nbusy;
    const bool busy = w < nbusy;
    // trailing pairs of column J-1 right of column J: (I, K), J+1 <= K <= I
    const int mrest = S::T - J - 1;
    const int nrest = J >= 1 ? mrest * (mrest + 1) / 2 : 0;
    if (nbusy == 4 && nrest > 0) {
      for (int p = w; p < nrest; p += 4) {
        int I, K;
        pair_of(p, J + 1, S::T, I, K);
        trailing_block(A, dv, J - 1, I, K, lane);
      }
      __syncthreads();
    }
    // (a) diagonal block (lanes 0..15) and panel rows 16 (J + 1) + 48 w +
    // lane - 16 (lanes 16..63) of the busy waves
    const int r = lane;
    const int i0 = lane < 16 ? 16 * J + lane : 16 * (J + 1) + 48 * w + (lane - 16);
    const bool live = i0 < S::LP;
    const int i = live ? i0 : 16 * J;   // lanes past the last row point at a valid row, unused
    double* row = A + bidx(i >> 4, J) + (i & 15) * 16;   // row i of block column J
    const int sw = (i & 15) >> 1;
    double a[16];
    if (busy) {
#pragma unroll
      for (int c = 0; c < 16; ++c) a[c] = (live && (r >= 16 || c <= r)) ? row[c ^ sw] : 0.0;
      // steps past the last real row of the block change nothing (the
      // padding is the identity) and are skipped
      const int kmax = L - 16 * J < 16 ? L - 16 * J : 16;
      double* col = colbuf + 16 * w;   // this wave's copy of column k
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (k < kmax) {
          // lanes 0..15 publish column k of the block; every lane then reads
          // the pivot and the entries below it as broadcasts
          if (r < 16) col[r] = a[k];
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          const double d = col[k];
          const double inv = d > PIVOT_EPS ? pivot_recip(d) : 0.0;
          const double lk = a[k] * inv;                  // L[row][k] for rows below k
#pragma unroll
          for (int c = k + 1; c < 16; ++c) a[c] = fma(-lk, col[c], a[c]);
          a[k] = r > k ? lk : a[k];                      // lane k keeps its pivot
        }
      }
      if (r < 16) {
        if (w == 0) {
          // lane r's diagonal entry is its pivot; the inverse is recomputed
          // from it exactly as in the step
          double dr = a[0];
#pragma unroll
          for (int c = 1; c < 16; ++c) dr = c == r ? a[c] : dr;
          dv[16 * J + r] = dr;
          iv[16 * J + r] = dr > PIVOT_EPS ? pivot_recip(dr) : 0.0;
        }
      } else if (live) {
#pragma unroll
        for (int c = 0; c < 16; ++c) row[c ^ sw] = a[c];
      }
    } else {
      // the other waves meanwhile apply column J-1 to the blocks right of
      // column J (column J itself was updated before this step)
      for (int p = w - nbusy; p < nrest; p += 4 - nbusy) {
        int I, K;
        pair_of(p, J + 1, S::T, I, K);
        trailing_block(A, dv, J - 1, I, K, lane);
      }
    }
    __syncthreads();
    // every wave has read the diagonal block: wave 0 stores its factor
    if (w == 0 && r < 16) {
#pragma unroll
      for (int c = 0; c < 16; ++c) row[c ^ sw] = c < r ? a[c] : 0.0;
    }
    if (J + 1 == S::T) break;
    // (b) lookahead: column J+1 now, (I, J+1) for I > J
    for (int p = w; p < S::T - J - 1; p += 4) trailing_block(A, dv, J, J + 1 + p, J + 1, lane);
    __syncthreads();
  }
  __syncthreads();   // the last diagonal block's factor is in place
}

// ---------------------------------------------------------------------------
// L D L^T z = b with the blocked factor of ldl_blocked, run by wave 0 alone:
// lane l owns rows l, l+64, l+128 in registers; the value of each step is
// read from its owner lane with v_readlane, so a step is one FMA deep.  The
// zero diagonal and upper parts of the diagonal blocks, and the zero row for
// blocks that do not exist, make every update unconditional: a row that is
// already final, or a padding row, only ever adds 0 * y.  Deflated unknowns
// (iv = 0) come out 0.  The caller synchronises the workgroup before reading
// z.
// ---------------------------------------------------------------------------
template <int L>
__device__ __forceinline__ void tri_solve_wave(const double* A, const double* iv, const double* b, double* z) {
  using S = BlockShape<L>;
  constexpr int NS = (L + 63) / 64;
  constexpr int ZROW = S::WORDS;
  const int lane = threadIdx.x & 63;
  int rI[NS], rlo[NS], rsw[NS];
  double bb[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = lane + 64 * s;
    const int ic = i < S::LP ? i : S::LP - 1;   // rows past the padding read in bounds
    rI[s] = ic >> 4;
    rlo[s] = ic & 15;
    rsw[s] = (ic & 15) >> 1;
    bb[s] = i < L ? b[i] : 0.0;
  }
  // forward: L y = b.  Row j is final once step j starts, so bb ends holding y.
#pragma unroll
  for (int s0 = 0; s0 < NS; ++s0) {
#pragma unroll
    for (int jj = 0; jj < 64; ++jj) {
      const int j = 64 * s0 + jj;
      if (j < L) {
        const int J = j >> 4;
        const double yj = lane_value(bb[s0], jj);
#pragma unroll
        for (int s = s0; s < NS; ++s) {
          // element (i, j): block (I, J) if I >= J, else the zero row
          const int rowbase = s > s0 ? (rI[s] * (rI[s] + 1) / 2 + J) * 256 + 16 * rlo[s]
                                     : (rI[s] >= J ? (rI[s] * (rI[s] + 1) / 2 + J) * 256 + 16 * rlo[s] : ZROW);
          bb[s] = fma(-A[rowbase + ((j & 15) ^ rsw[s])], yj, bb[s]);
        }
      }
    }
  }
  // diagonal: w = D^-1 y
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = lane + 64 * s;
    bb[s] *= iv[i < L ? i : 0];
  }
  // backward: L^T z = w; element (j, i) of L for i < j lies in block row
  // J = j >> 4; bb ends holding z.
#pragma unroll
  for (int s0 = NS - 1; s0 >= 0; --s0) {
#pragma unroll
    for (int jj = 63; jj >= 0; --jj) {
      const int j = 64 * s0 + jj;
      if (j < L) {
        const int J = j >> 4;
        const int jsw = (j & 15) >> 1;
        const double zj = lane_value(bb[s0], jj);
#pragma unroll
        for (int s = 0; s <= s0; ++s) {
          const int base = s < s0 ? (J * (J + 1) / 2 + rI[s]) * 256 + 16 * (j & 15)
                                  : (rI[s] <= J ? (J * (J + 1) / 2 + rI[s]) * 256 + 16 * (j & 15) : ZROW);
          bb[s] = fma(-A[base + (rlo[s] ^ jsw)], zj, bb[s]);
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = lane + 64 * s;
    if (i < L) z[i] = bb[s];
  }
}

// Factor, solve, write F and (optionally) the factor; shared tail of both
// K6 variants.  A holds the equilibrated matrix (blocked, padding = identity),
// b the scaled right-hand side, sc the equilibration scales.  The kept factor
// is [blocked L and D | D | D^-1 | sc].


// refine: 0 none, 1 where the estimate asks (flags the node), 2 every node.
// coef: the node's coefficient row; flag: its flag word; fout: where the
// factor goes (null: nowhere).  With SOLVE false only the factor is made (no
// right-hand side; b, z and coef may be null) and it is always stored.
// With regram (float32 Gram partials): a node whose estimate exceeds
// REGRAM_KAPPA or that deflates a pivot gets FLAG_REGRAM and nothing else
// (no coefficients, flags or factor): the float64 re-solve takes it.
template <int L, bool SOLVE = true>
__device__ __forceinline__ void factor_solve_store(double* A, double* b, double* z, double* dv, double* iv,
                                                   const double* sc, double (*xv)[L], double (*yv)[L], int refine,
                                                   double* coef, uint32_t* flag, double* fout,
                                                   uint32_t* status = nullptr, bool regram = false) {
  using S = BlockShape<L>;
  __shared__ int need_factor;   // the refinement sweeps will apply to this node
  __shared__ int any_deflated, to_regram;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const bool estimate = refine == 1 || regram;
  if (tid == 0) {
    need_factor = !SOLVE || refine == 2;
    any_deflated = 0;
    to_regram = 0;
  }
  if (estimate)
    for (int e = tid; e < 2 * L; e += 256) xv[e / L][e % L] = probe_entry(e % L, e / L, L);
  ldl_blocked<L>(A, dv, iv);
  // wave 0 solves for the coefficients; waves 1 and 2 meanwhile apply the
  // inverse to the two probe vectors (|G^-1 x| <= 1 / lambda_min, close to
  // it for all but exceptional x), a condition estimate at no extra latency
  if (w == 0) {
    if constexpr (SOLVE) tri_solve_wave<L>(A, iv, b, z);
  } else if (estimate && w <= 2) {
    tri_solve_wave<L>(A, iv, xv[w - 1], yv[w - 1]);
  }
  __syncthreads();
  bool deflated = false;
  for (int i = tid; i < L; i += 256)
    if (iv[i] == 0.0) deflated = true;
  if (deflated) any_deflated = 1;
  if (estimate && (w == 1 || w == 2)) {
    double ss = 0.0;
    for (int i = lane; i < L; i += 64) ss += yv[w - 1][i] * yv[w - 1][i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) ss += __shfl_xor(ss, off);
    const double kappa = (double)L * sqrt(ss);
    if (lane == 0 && regram && !(kappa <= REGRAM_KAPPA)) to_regram = 1;
    if (lane == 0 && refine == 1 && kappa > REFINE_KAPPA) {
      atomicOr(flag, FLAG_REFINE);
      need_factor = 1;
    }
  }
  __syncthreads();
  if (regram && (to_regram || any_deflated)) {
    if (tid == 0) atomicOr(flag, FLAG_REGRAM);
    return;   // uniform: the whole workgroup leaves the node to the float64 re-solve
  }
  if constexpr (SOLVE) {
    bool bad = false;
    for (int i = tid; i < L; i += 256) {
      const double c = sc[i] * z[i];
      coef[i] = c;
      bad |= !__builtin_isfinite(c);
    }
    mark_nonfinite(bad, flag, status);
  }
  deflated = any_deflated != 0;
  if (refine == 2) {
    if (tid == 0) atomicOr(flag, FLAG_REFINE);
  } else if (estimate && deflated) {
    if (tid == 0) atomicOr(flag, FLAG_REFINE);
    need_factor = 1;
  }
  __syncthreads();
  // the factor is kept only for the nodes the refinement sweeps will visit
  if (fout && need_factor) {
    double* fo = fout;
    for (int e = tid; e < S::WORDS; e += 256) fo[e] = A[e];
    for (int i = tid; i < L; i += 256) {
      fo[S::WORDS + i] = dv[i];
      fo[S::WORDS + L + i] = iv[i];
      fo[S::WORDS + 2 * L + i] = sc[i];
    }
  }
  if (deflated && tid == 0) atomicOr(flag, FLAG_DEFLATED);
}

// Fill the blocked matrix in storage order: thread t writes word t of every
// block, i.e. element (r, c) with r = t >> 4 and c = (t & 15) ^ (r >> 1), so
// the LDS writes are contiguous and the block indices are compile-time.
// value(i, q) gives the entry for i, q < L; the padding is the identity.
// Diagonal blocks get both triangles (the factor reads only the lower one).
// The zero row after the blocks is cleared too.
template <int L, typename V>
__device__ __forceinline__ void assemble_blocked(double* A, V value) {
  using S = BlockShape<L>;
  const int tid = threadIdx.x;
  const int r = tid >> 4, c = (tid & 15) ^ (r >> 1);
#pragma unroll
  for (int I = 0; I < S::T; ++I) {
    const int i = 16 * I + r;
#pragma unroll
    for (int J = 0; J <= I; ++J) {
      const int q = 16 * J + c;
      A[bidx(I, J) + tid] = (i < L && q < L) ? value(i, q) : (i == q ? 1.0 : 0.0);
    }
  }
  if (tid < 16) A[S::WORDS + tid] = 0.0;
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
  __shared__ double A[S::WORDS + 16];   // + the zero row
  __shared__ double b[L], z[L], dv[S::LP], iv[S::LP], sc[L];   // pivots cover the padding too
  __shared__ double xv[2][L], yv[2][L];                           // condition-estimate probes
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
    const double s = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    sc[i] = s;
    b[i] = gram(i, L) * s;
  }
  __syncthreads();
  assemble_blocked<L>(A, [&](int i, int q) { return (i <= q ? gram(i, q) : gram(q, i)) * sc[i] * sc[q]; });
  __syncthreads();
  factor_solve_store<L>(A, b, z, dv, iv, sc, xv, yv, a.refine, a.nt.coef + (size_t)node * L, a.nt.flags + node,
                        fac ? fac + (size_t)k * factor_words<L>() : nullptr, a.status, a.regram != 0);
}

// Equilibrated normal equations from power moments in LDS: mom[0 .. NM) the
// power moments M (graded order up to degree 2p); with bm, the r-weighted
// moments B (calL of them) give the scaled right-hand side b.  Fills the
// exponent table ex, the scales sc (1 / sqrt(G_ii)) and weights wv
// (sc / alpha!), then the blocked matrix A_ik = M[alpha_i + alpha_k] w_i w_k
// in storage order (padding = identity, zero row cleared).  All 256 threads;
// the workgroup's stores of mom (and bm) before the call are published by
// the first barrier inside; the caller synchronises before reading A.
template <int P>
__device__ __forceinline__ void assemble_moments(double* A, const double* mom, const double* bm, double* b,
                                                 double* sc, double* wv, int (*ex)[3]) {
  constexpr int L = basis_size(P);
  constexpr Basis<P> B{};
  using S = BlockShape<L>;
  const int tid = threadIdx.x;
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
    if (bm) b[i] = bm[i] * s * f;
  }
  __syncthreads();
  // storage-order fill (as assemble_blocked) with this thread's row and
  // column exponents (packed a | b << 8 | c << 16) and weights in registers
  const int r = tid >> 4, c = (tid & 15) ^ (r >> 1);
  uint32_t er[S::T], ec[S::T];
  double wr[S::T], wc[S::T];
#pragma unroll
  for (int I = 0; I < S::T; ++I) {
    const int i = 16 * I + r, q = 16 * I + c;
    er[I] = i < L ? (uint32_t)ex[i][0] | ((uint32_t)ex[i][1] << 8) | ((uint32_t)ex[i][2] << 16) : 0u;
    ec[I] = q < L ? (uint32_t)ex[q][0] | ((uint32_t)ex[q][1] << 8) | ((uint32_t)ex[q][2] << 16) : 0u;
    wr[I] = i < L ? wv[i] : 0.0;
    wc[I] = q < L ? wv[q] : 0.0;
  }
#pragma unroll
  for (int I = 0; I < S::T; ++I) {
    const int i = 16 * I + r;
#pragma unroll
    for (int J = 0; J <= I; ++J) {
      const int q = 16 * J + c;
      const uint32_t e = er[I] + ec[J];
      const double m = mom[graded((int)(e & 255u), (int)((e >> 8) & 255u), (int)(e >> 16))];
      A[bidx(I, J) + tid] = (i < L && q < L) ? m * wr[I] * wc[J] : (i == q ? 1.0 : 0.0);
    }
  }
  if (tid < 16) A[S::WORDS + tid] = 0.0;
}

// ---------------------------------------------------------------------------
// K6 from power moments: G_ik = M[alpha_i + alpha_k] / (alpha_i! alpha_k!),
// b_i = B[alpha_i] / alpha_i!.  Equilibration is folded into the assembly:
// with s_i = 1 / sqrt(G_ii) and w_i = s_i / alpha_i!, the scaled matrix is
// A_ik = M[alpha_i + alpha_k] w_i w_k and the scaled right-hand side
// B[alpha_i] w_i.  M and B come from the node's mode-0 partial, or, where
// the moment pyramid covers the node, M from its pyramid cell and B from the
// node's B-only partial.
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_solve_m(LevelArgs a, const double* __restrict__ part_m,
                                                 const double* __restrict__ part_b, const double* __restrict__ pyr,
                                                 double* __restrict__ fac) {
  constexpr int L = basis_size(P);
  constexpr int NM = basis_size(2 * P);
  constexpr int NOUT = NM + L + 1;
  using S = BlockShape<L>;
  __shared__ double A[S::WORDS + 16];   // + the zero row
  __shared__ double mom[NOUT > 4 * L ? NOUT : 4 * L];
  __shared__ double b[L], z[L], dv[S::LP], iv[S::LP], sc[L], wv[L];   // pivots cover the padding too
  __shared__ int ex[L][3];
  // the condition-estimate probes reuse the moments' space (dead after assembly)
  double(*xv)[L] = reinterpret_cast<double(*)[L]>(mom);
  double(*yv)[L] = reinterpret_cast<double(*)[L]>(mom + 2 * L);
  const int tid = threadIdx.x;
  const uint32_t k = blockIdx.x;
  const uint32_t node = a.node0 + k;
  const uint32_t c0 = a.chunk_off[k];   // chunks of the node were summed into this one
  if (a.only_flag && !(a.nt.flags[node] & a.only_flag)) return;   // whole workgroup: not this pass's node
  const uint32_t* pt = a.pyr_tab ? a.pyr_tab + PYR_TAB_WORDS * a.nt.problem[node] : nullptr;
  if (pt && a.fac_up && (pt[3] >> 28) > (uint32_t)a.level) return;   // factored ahead: k_solve_ahead
  if (pt && pyramid_covers(pt[1], a.level)) {
    // M from the pyramid cell, B from the node's B-only partial; all loads
    // issued before the first store
    const size_t cell = (size_t)pt[0] + level_first(a.level) + a.nt.prefix[node];
    const double* ms = pyr + cell * NM;
    const double* bs = part_b + (size_t)c0 * L;
    constexpr int RM = (NM + 255) / 256, RB = (L + 255) / 256;
    double vm[RM], vb[RB];
#pragma unroll
    for (int q = 0; q < RM; ++q) vm[q] = tid + 256 * q < NM ? ms[tid + 256 * q] : 0.0;
#pragma unroll
    for (int q = 0; q < RB; ++q) vb[q] = tid + 256 * q < L ? bs[tid + 256 * q] : 0.0;
#pragma unroll
    for (int q = 0; q < RM; ++q)
      if (tid + 256 * q < NM) mom[tid + 256 * q] = vm[q];
#pragma unroll
    for (int q = 0; q < RB; ++q)
      if (tid + 256 * q < L) mom[NM + tid + 256 * q] = vb[q];
  } else {
    copy_to_lds<256, NM + L>(mom, part_m + (size_t)c0 * NOUT, tid);
  }
  assemble_moments<P>(A, mom, mom + NM, b, sc, wv, ex);
  __syncthreads();
  factor_solve_store<L>(A, b, z, dv, iv, sc, xv, yv, a.refine, a.nt.coef + (size_t)node * L, a.nt.flags + node,
                        fac ? fac + (size_t)k * factor_words<L>() : nullptr, a.status);
}

// ---------------------------------------------------------------------------
// K6 for the nodes whose factor was made ahead of the level loop
// (k_factor_cells): B from the node's mode-2 partial, scaled as the
// assembly scales it, and the two triangular solves with the kept factor;
// the factor's flags go to the node, and the factor itself to the level's
// refinement slot where the estimate asked for refinement.  Other nodes exit.
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_solve_ahead(LevelArgs a, const double* __restrict__ part_b,
                                                     double* __restrict__ fac) {
  constexpr int L = basis_size(P);
  constexpr size_t FW = factor_words<L>();
  constexpr Basis<P> B{};
  using S = BlockShape<L>;
  __shared__ double A[S::WORDS + 16];   // + the zero row
  __shared__ double b[L], z[L], iv[S::LP], sc[L];
  const int tid = threadIdx.x;
  const uint32_t k = blockIdx.x;
  const uint32_t node = a.node0 + k;
  const uint32_t* pt = a.pyr_tab + PYR_TAB_WORDS * a.nt.problem[node];
  if (!((pt[3] >> 28) > (uint32_t)a.level)) return;   // whole workgroup: factored in this level's solve
  const uint32_t c0 = a.chunk_off[k];   // chunks of the node were summed into this one
  const uint32_t slot = (pt[3] & 0x0FFFFFFFu) + level_first(a.level) + a.nt.prefix[node];
  const double* fo = a.fac_up + (size_t)slot * FW;
  const double* bs = part_b + (size_t)c0 * L;
  copy_to_lds<256, S::WORDS>(A, fo, tid);
  if (tid < 16) A[S::WORDS + tid] = 0.0;
  for (int i = tid; i < L; i += 256) {
    iv[i] = fo[S::WORDS + L + i];
    sc[i] = fo[S::WORDS + 2 * L + i];
    b[i] = bs[i] * sc[i] * B.inv_fact[i];   // as assemble_moments scales it
  }
  __syncthreads();
  if (tid < 64) tri_solve_wave<L>(A, iv, b, z);
  __syncthreads();
  bool bad = false;
  for (int i = tid; i < L; i += 256) {
    const double c = sc[i] * z[i];
    a.nt.coef[(size_t)node * L + i] = c;
    bad |= !__builtin_isfinite(c);
  }
  mark_nonfinite(bad, a.nt.flags + node, a.status);
  const uint32_t fl = a.up_flags[slot];
  if (tid == 0 && fl) atomicOr(a.nt.flags + node, fl);
  // keep the factor where the refinement looks for it
  if (fac && (fl & FLAG_REFINE)) {
    double* fk = fac + (size_t)k * FW;
    for (size_t e = tid; e < FW; e += 256) fk[e] = fo[e];
  }
}

// ---------------------------------------------------------------------------
// Factor only, from the mode-3 partials (M alone): the same equilibrated
// matrix as k_solve_m, factored and stored for every node, with the
// condition estimate and flags.  One workgroup per node; used where several
// right-hand sides share one node set (the fixed-topology transform).
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_factor_m(LevelArgs a, const double* __restrict__ part_m,
                                                  double* __restrict__ fac) {
  constexpr int L = basis_size(P);
  constexpr int NM = basis_size(2 * P);
  using S = BlockShape<L>;
  __shared__ double A[S::WORDS + 16];   // + the zero row
  __shared__ double mom[NM > 4 * L ? NM : 4 * L];
  __shared__ double dv[S::LP], iv[S::LP], sc[L], wv[L];
  __shared__ int ex[L][3];
  double(*xv)[L] = reinterpret_cast<double(*)[L]>(mom);
  double(*yv)[L] = reinterpret_cast<double(*)[L]>(mom + 2 * L);
  const int tid = threadIdx.x;
  const uint32_t k = blockIdx.x;
  const uint32_t node = a.node0 + k;
  copy_to_lds<256, NM>(mom, part_m + (size_t)a.chunk_off[k] * NM, tid);
  assemble_moments<P>(A, mom, nullptr, nullptr, sc, wv, ex);
  __syncthreads();
  factor_solve_store<L, false>(A, nullptr, nullptr, dv, iv, sc, xv, yv, a.refine, nullptr, a.nt.flags + node,
                               fac + (size_t)k * factor_words<L>());
}

// ---------------------------------------------------------------------------
// Factors made ahead of the level loop: one workgroup per listed pyramid
// entry (a cell of a level above the pyramid's finest), its M taken from
// the pyramid, the factor and the flags of its condition estimate stored in
// slot g.  The level's solve then only applies them (k_solve_ahead).
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_factor_cells(const double* __restrict__ pyr,
                                                      const uint32_t* __restrict__ list, int refine,
                                                      double* __restrict__ fac_up, uint32_t* __restrict__ up_flags) {
  constexpr int L = basis_size(P);
  constexpr int NM = basis_size(2 * P);
  using S = BlockShape<L>;
  __shared__ double A[S::WORDS + 16];   // + the zero row
  __shared__ double mom[NM > 4 * L ? NM : 4 * L];
  __shared__ double dv[S::LP], iv[S::LP], sc[L], wv[L];
  __shared__ int ex[L][3];
  double(*xv)[L] = reinterpret_cast<double(*)[L]>(mom);
  double(*yv)[L] = reinterpret_cast<double(*)[L]>(mom + 2 * L);
  const int tid = threadIdx.x;
  const uint32_t g = blockIdx.x;
  copy_to_lds<256, NM>(mom, pyr + (size_t)list[g] * NM, tid);
  assemble_moments<P>(A, mom, nullptr, nullptr, sc, wv, ex);
  __syncthreads();
  factor_solve_store<L, false>(A, nullptr, nullptr, dv, iv, sc, xv, yv, refine, nullptr, up_flags + g,
                               fac_up + (size_t)g * factor_words<L>());
}

// ---------------------------------------------------------------------------
// K7: refinement.  The sweep (power moments of r' = r - Lambda F, float64,
// in k_moments.hip) gives B'[alpha] = sum r' u^alpha per chunk; the solve
// sums its node's chunks, takes delta = G^{-1} Lambda^T r' with the kept
// factor and sets F += delta.
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_refine_solve(LevelArgs a, const double* __restrict__ part_b,
                                                      const double* __restrict__ fac) {
  constexpr int L = basis_size(P);
  constexpr Basis<P> B{};
  using S = BlockShape<L>;
  __shared__ double A[S::WORDS + 16];   // + the zero row
  __shared__ double b[L], z[L], iv[L], sc[L];
  const int tid = threadIdx.x;
  const uint32_t k = a.sel ? a.sel[blockIdx.x] : blockIdx.x;
  const uint32_t node = a.node0 + k;
  if (!(a.nt.flags[node] & FLAG_REFINE)) return;   // whole workgroup: its node needs no refinement
  // with a.refine == 2 (every node refined) the chunk partials were summed
  // into the first chunk's slot beforehand; otherwise they are summed here
  const uint32_t c0 = a.chunk_off[k], c1 = a.refine == 2 ? c0 + 1 : a.chunk_off[k + 1];
  part_b += (size_t)blockIdx.y * a.nchunks * L;   // the field's partials
  const double* fo = fac + (size_t)k * (S::WORDS + 3 * L);
  copy_to_lds<256, S::WORDS>(A, fo, tid);
  if (tid < 16) A[S::WORDS + tid] = 0.0;
  // B' of the node: its chunks' partials summed here (G interleaved groups of
  // chunks per moment, then the groups in order)
  constexpr int G = 256 / L > 0 ? 256 / L : 1;
  __shared__ double bsum[G][L];
  if (tid < G * L) {
    const int i = tid % L, q = tid / L;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    uint32_t g = c0 + (uint32_t)q;
    for (; g + 7 * G < c1; g += 8 * G) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += part_b[(size_t)(g + u * G) * L + i];
    }
    for (; g < c1; g += G) acc[0] += part_b[(size_t)g * L + i];
    bsum[q][i] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  __syncthreads();
  for (int i = tid; i < L; i += 256) {
    double t = bsum[0][i];
#pragma unroll
    for (int q = 1; q < G; ++q) t += bsum[q][i];
    iv[i] = fo[S::WORDS + L + i];
    sc[i] = fo[S::WORDS + 2 * L + i];
    b[i] = t * B.inv_fact[i] * fo[S::WORDS + 2 * L + i];
  }
  __syncthreads();
  if (tid < 64) tri_solve_wave<L>(A, iv, b, z);
  __syncthreads();
  double* F = a.nt.coef + (size_t)blockIdx.y * a.cstride + (size_t)node * L;
  bool bad = false;
  for (int i = tid; i < L; i += 256) {
    const double dl = sc[i] * z[i];
    const double c = F[i] + dl;
    F[i] = c;
    if (a.delta) a.delta[(size_t)k * L + i] = dl;
    bad |= !__builtin_isfinite(c);
  }
  mark_nonfinite(bad, a.nt.flags + node, a.status);
}


// The first solve of every field against the kept factors: one workgroup
// per node loads the node's factor into LDS once, and its four waves take
// the fields in turn (each wave scales its field's B, runs the two
// triangular solves on the shared factor and writes F).  The chunk partials
// were summed beforehand.
template <int P>
__global__ void __launch_bounds__(256) k_factor_solve(LevelArgs a, const double* __restrict__ part_b,
                                                      const double* __restrict__ fac) {
  constexpr int L = basis_size(P);
  constexpr Basis<P> B{};
  using S = BlockShape<L>;
  __shared__ double A[S::WORDS + 16];   // + the zero row
  __shared__ double iv[L], sc[L];
  __shared__ double bw[4][L], zw[4][L];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const uint32_t k = blockIdx.x;
  const uint32_t node = a.node0 + k;
  const uint32_t c0 = a.chunk_off[k];
  const double* fo = fac + (size_t)k * factor_words<L>();
  copy_to_lds<256, S::WORDS>(A, fo, tid);
  if (tid < 16) A[S::WORDS + tid] = 0.0;
  for (int i = tid; i < L; i += 256) {
    iv[i] = fo[S::WORDS + L + i];
    sc[i] = fo[S::WORDS + 2 * L + i];
  }
  __syncthreads();
  const uint32_t nf = a.nfields > 1 ? a.nfields : 1u;
  for (uint32_t j = (uint32_t)w; j < nf; j += 4) {
    const double* bs = part_b + ((size_t)j * a.nchunks + c0) * L;
    for (int i = lane; i < L; i += 64) bw[w][i] = bs[i] * B.inv_fact[i] * sc[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    tri_solve_wave<L>(A, iv, bw[w], zw[w]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double* F = a.nt.coef + (size_t)j * a.cstride + (size_t)node * L;
    for (int i = lane; i < L; i += 64) F[i] = sc[i] * zw[w][i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// ---------------------------------------------------------------------------
// K8: residual update r <- r - Lambda F (Alg. 2) and, per chunk and child
// octant, the sum of r^2 (Alg. 1's E_RMS numerator) and the point count,
// reduced in a fixed order so that results do not depend on scheduling.
// part_ss holds 16 doubles per chunk: 8 sums of r^2, then 8 counts (exact).
// ---------------------------------------------------------------------------
// Threads of a residual workgroup (one chunk of up to CHUNK points): 1024
// up to p = 3 (sixteen waves in flight per chunk hide the load latency of
// the few chunks of the top levels; the polynomial fits the registers of
// four waves per SIMD), 256 above (more threads per workgroup would make the
// compiler spill the polynomial's coefficients).  Above p = 3 the nodes
// under SMALL_NODE points (one chunk of at most 1023 points) take a launch
// of one-wave workgroups instead (SMALL): a lane then walks several points
// instead of most lanes one or none, and more chunks share a compute unit
// (the batched workload's deep levels of 10^4 small nodes: 9.0 -> 8.7 ms
// per batch when every chunk took one wave, but the 2 048-point chunks of
// the large nodes lost as much).  The choice depends on the node alone.
template <int P, bool SMALL = false>
struct ResidualShape {
  static constexpr bool SPLIT = P > 3;   // launches split by node size
  static constexpr int THREADS = SMALL ? 64 : (P <= 3 ? 1024 : 256);
  static constexpr int WAVES = THREADS / 64;
};

// LISTED: the launch covers the listed nodes' chunks (a.sel); SMALL: the
// nodes under SMALL_NODE points (where ResidualShape splits; else the others)
template <int P, typename TIN, bool LISTED, bool SMALL>
__global__ void __launch_bounds__((ResidualShape<P, SMALL>::THREADS))
k_residual(LevelArgs a, double* __restrict__ part_ss) {
  constexpr int L = basis_size(P);
  constexpr int NT = ResidualShape<P, SMALL>::THREADS, NW = ResidualShape<P, SMALL>::WAVES;
  __shared__ double Fs[L];
  __shared__ double red[NW][8];
  __shared__ uint32_t redc[NW][8];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  uint32_t g = blockIdx.x, k;
  if constexpr (LISTED) {
    if (!listed_chunk(a, blockIdx.x, k, g)) return;
  } else {
    k = chunk_node(a.chunk_off, a.nnodes, g);
  }
  const uint32_t node = a.node0 + k;
  if (a.only_flag && !(a.nt.flags[node] & a.only_flag)) return;   // whole workgroup: not this pass's node
  const uint32_t nb = a.nt.begin[node], nc = a.nt.count[node];
  if constexpr (ResidualShape<P>::SPLIT && !LISTED) {
    if ((nc < (uint32_t)SMALL_NODE) != SMALL) return;   // the other launch's node
  }
  const uint32_t start = nb + (g - a.chunk_off[k]) * CHUNK;
  const uint32_t end = min(nb + nc, start + (uint32_t)CHUNK);
  const double* geo = a.nt.geo + 6 * (size_t)node;
  const double cx = geo[0], cy = geo[1], cz = geo[2], sx = geo[3], sy = geo[4], sz = geo[5];
  const uint32_t fj = blockIdx.y;   // field of a multi-field launch
  double* rr = a.r + (size_t)fj * a.rstride;
  // the polynomial to subtract: the node's coefficients, or (correction
  // pass) its refinement's delta
  const double* Fsrc = a.delta ? a.delta + (size_t)k * L : a.nt.coef + (size_t)fj * a.cstride + (size_t)node * L;
  for (int i = tid; i < L; i += NT) Fs[i] = Fsrc[i];
  __syncthreads();
  const bool stats = a.level < a.D;
  const int shift = stats ? 3 * (a.D - a.level - 1) : 0;
  double ss[8];
  uint32_t cn[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    ss[q] = 0.0;
    cn[q] = 0u;
  }
  auto tally = [&](double rn, uint32_t key) {
    const uint32_t o = (key >> shift) & 7u;
    const double r2 = rn * rn;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      ss[q] += (o == (uint32_t)q) ? r2 : 0.0;
      cn[q] += (o == (uint32_t)q) ? 1u : 0u;
    }
  };
  if constexpr (P <= 6) {
    // the next point's inputs are loaded before this point's polynomial, so
    // their latency overlaps it (larger bases would lose occupancy)
    TIN nx = 0, ny = 0, nz = 0;
    double nr = 0.0;
    uint32_t nk = 0;
    if (start + tid < end) {
      const uint32_t i0 = start + tid;
      nx = ((const TIN*)a.px)[i0];
      ny = ((const TIN*)a.py)[i0];
      nz = ((const TIN*)a.pz)[i0];
      nr = rr[i0];
      nk = a.skey[i0];
    }
    for (uint32_t i = start + tid; i < end; i += NT) {
      const double x = (double)nx, y = (double)ny, z = (double)nz, rold = nr;
      const uint32_t key = nk;
      if (i + NT < end) {
        nx = ((const TIN*)a.px)[i + NT];
        ny = ((const TIN*)a.py)[i + NT];
        nz = ((const TIN*)a.pz)[i + NT];
        nr = rr[i + NT];
        nk = a.skey[i + NT];
      }
      const double val = poly_eval<P, double>(Fs, (x - cx) * sx, (y - cy) * sy, (z - cz) * sz);
      const double rn = rold - val;
      rr[i] = rn;
      tally(rn, key);
    }
  } else {
    for (uint32_t i = start + tid; i < end; i += NT) {
      double x, y, z;
      load_point<TIN>(a.px, a.py, a.pz, i, x, y, z);
      const double val = poly_eval<P, double>(Fs, (x - cx) * sx, (y - cy) * sy, (z - cz) * sz);
      const double rn = rr[i] - val;
      rr[i] = rn;
      tally(rn, a.skey[i]);
    }
  }
  if (!stats) return;
  // fixed-order reduction: butterfly inside the wave, then waves in order
#pragma unroll
  for (int q = 0; q < 8; ++q) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      ss[q] += __shfl_xor(ss[q], off);
      cn[q] += __shfl_xor(cn[q], off);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      red[w][q] = ss[q];
      redc[w][q] = cn[q];
    }
  }
  __syncthreads();
  part_ss += (size_t)fj * a.nchunks * 16;
  // the waves in order (a fixed summation order)
  if (tid < 8) {
    double t = red[0][tid];
#pragma unroll
    for (int q = 1; q < NW; ++q) t += red[q][tid];
    part_ss[(size_t)g * 16 + tid] = t;
  } else if (tid < 16) {
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) c += redc[q][tid - 8];
    part_ss[(size_t)g * 16 + tid] = (double)c;
  }
}

// Exclusive prefix sum of one value per thread over a workgroup of NT
// threads: inclusive scans inside each wave (shuffles), then the wave totals
// from LDS.  Returns the thread's exclusive prefix and sets total; wsum holds
// NT / 64 words.  Every thread must call it (two barriers inside).
template <uint32_t NT>
__device__ __forceinline__ uint32_t scan_block(uint32_t x, uint32_t* wsum, uint32_t& total) {
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  uint32_t v = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)v, o);
    if (lane >= (uint32_t)o) v += y;
  }
  if (lane == 63) wsum[w] = v;
  __syncthreads();
  uint32_t base = 0, all = 0;
#pragma unroll
  for (uint32_t q = 0; q < NT / 64; ++q) {
    const uint32_t t = wsum[q];
    base += q < w ? t : 0u;
    all += t;
  }
  __syncthreads();   // wsum may be reused after this
  total = all;
  return base + v - x;
}
__device__ __forceinline__ uint32_t scan_1024(uint32_t x, uint32_t* wsum, uint32_t& total) {
  return scan_block<1024>(x, wsum, total);
}

// ---------------------------------------------------------------------------
// Residual update of every field of a multi-field launch (the fixed-topology
// refit), without octant statistics: one workgroup per chunk reads the
// chunk's points once per group of up to RF_GROUP fields and takes each
// field's r <- r - Lambda F with that field's coefficients (the arithmetic of
// k_residual, point by point).
// ---------------------------------------------------------------------------
constexpr int RF_GROUP = 8;

template <int P, typename TIN>
__global__ void __launch_bounds__(256) k_residual_fields(LevelArgs a) {
  constexpr int L = basis_size(P);
  __shared__ double Fs[RF_GROUP][L];
  const int tid = threadIdx.x;
  const uint32_t g = blockIdx.x;
  const uint32_t k = chunk_node(a.chunk_off, a.nnodes, g);
  const uint32_t node = a.node0 + k;
  const uint32_t nb = a.nt.begin[node], nc = a.nt.count[node];
  const uint32_t start = nb + (g - a.chunk_off[k]) * CHUNK;
  const uint32_t end = min(nb + nc, start + (uint32_t)CHUNK);
  const double* geo = a.nt.geo + 6 * (size_t)node;
  const double cx = geo[0], cy = geo[1], cz = geo[2], sx = geo[3], sy = geo[4], sz = geo[5];
  const uint32_t nf = a.nfields > 1 ? a.nfields : 1u;
  for (uint32_t f0 = 0; f0 < nf; f0 += RF_GROUP) {
    const uint32_t ng = min((uint32_t)RF_GROUP, nf - f0);
    __syncthreads();   // the previous group's coefficients are no longer read
    for (uint32_t e = tid; e < ng * L; e += 256)
      Fs[e / L][e % L] = a.nt.coef[(size_t)(f0 + e / L) * a.cstride + (size_t)node * L + e % L];
    __syncthreads();
    for (uint32_t i = start + tid; i < end; i += 256) {
      double x, y, z;
      load_point<TIN>(a.px, a.py, a.pz, i, x, y, z);
      const double u = (x - cx) * sx, v = (y - cy) * sy, w = (z - cz) * sz;
      for (uint32_t j = 0; j < ng; ++j) {
        double* rr = a.r + (size_t)(f0 + j) * a.rstride;
        const double val = poly_eval<P, double>(Fs[j], u, v, w);
        rr[i] = rr[i] - val;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Child activation (Alg. 1): octant o of a node at depth d becomes a node iff
// d + 1 <= D, n_o >= calL (tested first) and sqrt(sum r^2 / n_o) > tol.
// One thread per node.  The octant counts come from the residual pass (exact
// integers); points are sorted by key, so octant o's points follow those of
// octants 0..o-1 inside the node.
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
  const uint32_t c0 = a.chunk_off[k];   // chunks of the node were summed into this one
  const double* st = part_ss + (size_t)c0 * 16;
  uint32_t pos = a.nt.begin[node], mask = 0;
  for (int o = 0; o < 8; ++o) {
    const uint32_t n_o = (uint32_t)st[8 + o];
    cbeg[(size_t)k * 8 + o] = pos;
    ccnt[(size_t)k * 8 + o] = n_o;
    pos += n_o;
    if (n_o < L) continue;
    if (sqrt(st[o] / (double)n_o) > a.tol) mask |= 1u << o;
  }
  a.nt.child_mask[node] = mask;
  nact[k] = (uint32_t)__popc(mask);
}

// Sum the per-chunk partials of every multi-chunk node into the node's first
// chunk slot (deterministic).  `width` doubles per chunk.  A workgroup covers
// 64 elements of one node with 16 lane groups; group q sums chunks
// q, q+16, ... into eight interleaved accumulators (eight loads in flight per
// thread), and the sixteen group sums are added in a fixed tree.
// Single-chunk nodes exit at once; with the level's list of multi-chunk
// nodes (multi, nmulti entries) only those are launched.
__global__ void __launch_bounds__(1024) k_chunk_reduce(const uint32_t* __restrict__ chunk_off, uint32_t nnodes,
                                                       double* __restrict__ buf, uint32_t width, uint32_t eblocks,
                                                       uint64_t fstride, const uint32_t* __restrict__ flags,
                                                       uint32_t only_flag, const uint32_t* __restrict__ multi,
                                                       uint32_t nmulti) {
  __shared__ double part[16][64];
  buf += (size_t)blockIdx.y * fstride;   // the field's partials
  const uint32_t q0 = blockIdx.x / eblocks;
  if (q0 >= (multi ? nmulti : nnodes)) return;
  const uint32_t k = multi ? multi[q0] : q0;
  if (k >= nnodes) return;
  const uint32_t c0 = chunk_off[k], c1 = chunk_off[k + 1];
  if (c1 - c0 < 2) return;
  if (only_flag && !(flags[k] & only_flag)) return;   // not this pass's node
  const uint32_t lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const uint32_t e = (blockIdx.x % eblocks) * 64 + lane;
  double acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = 0.0;
  if (e < width) {
    uint32_t g = c0 + q;
    for (; g + 16 * 7 < c1; g += 16 * 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += buf[(size_t)(g + 16 * u) * width + e];
    }
    for (; g < c1; g += 16) acc[0] += buf[(size_t)g * width + e];
  }
  part[q][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (q == 0 && e < width) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = part[2 * u][lane] + part[2 * u + 1][lane];
    buf[(size_t)c0 * width + e] = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
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
                                               uint32_t* __restrict__ counters, uint32_t* __restrict__ hostc,
                                               uint32_t seq, uint32_t* __restrict__ next_multi,
                                               uint32_t* __restrict__ sel) {
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t nmulti;   // children spanning more than one chunk, listed in next_multi
  const uint32_t tid = threadIdx.x;
  if (tid == 0) nmulti = 0;
  const uint32_t m = a.nnodes;
  const uint32_t seg = (m + 1023u) / 1024u;
  const uint32_t b = min(m, tid * seg), e = min(m, b + seg);
  // Every loop below issues the loads of EB iterations before using any:
  // one workgroup walks a level of tens of thousands of nodes (batches of
  // problems), and a load latency per iteration would dominate.
  constexpr uint32_t EB = 8;
  uint32_t sum = 0, flagged = 0;
  for (uint32_t i0 = b; i0 < e; i0 += EB) {
    uint32_t v[EB], f[EB];
#pragma unroll
    for (uint32_t u = 0; u < EB; ++u) {
      const uint32_t i = min(i0 + u, e - 1);
      v[u] = nact[i];
      f[u] = a.nt.flags[a.node0 + i];
    }
#pragma unroll
    for (uint32_t u = 0; u < EB; ++u)
      if (i0 + u < e) {
        sum += v[u];
        flagged += (f[u] & FLAG_REFINE) ? 1u : 0u;
      }
  }
  uint32_t total, level_flagged, flagged_chunks = 0;
  uint32_t fpos = scan_1024(flagged, wsum, level_flagged);
  if (level_flagged) {   // (uniform) flagged nodes are rare
    // the flagged nodes in order and their first chunk numbers among them,
    // for the late refinement's launches
    uint32_t fchunks = 0;
    if (flagged)
      for (uint32_t i = b; i < e; ++i)
        if (a.nt.flags[a.node0 + i] & FLAG_REFINE) fchunks += a.chunk_off[i + 1] - a.chunk_off[i];
    uint32_t cpos = scan_1024(fchunks, wsum, flagged_chunks);
    if (sel && flagged) {
      uint32_t* sel_off = sel + m + 1;
      for (uint32_t i = b; i < e; ++i)
        if (a.nt.flags[a.node0 + i] & FLAG_REFINE) {
          sel[fpos] = i;
          sel_off[fpos] = cpos;
          ++fpos;
          cpos += a.chunk_off[i + 1] - a.chunk_off[i];
        }
    }
  }
  if (sel && tid == 0) sel[m + 1 + level_flagged] = flagged_chunks;
  // each node's first child index (exclusive prefix of the active counts),
  // in place of its count
  uint32_t run = scan_1024(sum, wsum, total);
  for (uint32_t i0 = b; i0 < e; i0 += EB) {
    uint32_t v[EB];
#pragma unroll
    for (uint32_t u = 0; u < EB; ++u) v[u] = nact[min(i0 + u, e - 1)];
#pragma unroll
    for (uint32_t u = 0; u < EB; ++u)
      if (i0 + u < e) {
        nact[i0 + u] = run;
        run += v[u];
      }
  }
  __syncthreads();
  // one thread per (node, octant): the octant's child, if active; four
  // strided iterations' loads at a time (children are laid out after the
  // level's nodes, so none of these loads reads what the iterations write)
  uint32_t pts = 0, small = 0;
  constexpr uint32_t CB = 4;
  const uint32_t npr = 8u * m;
  for (uint32_t pr0 = tid; pr0 < npr; pr0 += 1024u * CB) {
    uint32_t mk[CB], fi[CB], pb[CB], px[CB], cb[CB], cc[CB];
#pragma unroll
    for (uint32_t u = 0; u < CB; ++u) {
      const uint32_t pr = min(pr0 + 1024u * u, npr - 1), node = a.node0 + (pr >> 3);
      mk[u] = a.nt.child_mask[node];
      fi[u] = nact[pr >> 3];
      pb[u] = a.nt.problem[node];
      px[u] = a.nt.prefix[node];
      cb[u] = cbeg[pr];
      cc[u] = ccnt[pr];
    }
#pragma unroll
    for (uint32_t u = 0; u < CB; ++u) {
      const uint32_t pr = pr0 + 1024u * u;
      if (pr >= npr) continue;
      const uint32_t i = pr >> 3, o = pr & 7u;
      const uint32_t node = a.node0 + i;
      const uint32_t mask = mk[u];
      const uint32_t first = next0 + fi[u];
      if (o == 0 && mask) a.nt.first_child[node] = first;
      if (!((mask >> o) & 1u)) continue;
      const uint32_t crun = fi[u] + (uint32_t)__popc(mask & ((1u << o) - 1u));
      const uint32_t cid = next0 + crun;
      const uint32_t prob = pb[u];
      const uint32_t cpre = (px[u] << 3) | o;
      a.nt.begin[cid] = cb[u];
      const uint32_t cn = cc[u];
      a.nt.count[cid] = cn;
      a.nt.prefix[cid] = cpre;
      a.nt.level[cid] = (uint32_t)(a.level + 1);
      a.nt.problem[cid] = prob;
      a.nt.parent[cid] = node;
      a.nt.first_child[cid] = 0;
      a.nt.child_mask[cid] = 0;
      a.nt.flags[cid] = 0;
      node_geo(prm[prob], a.level + 1, cpre, a.nt.geo + 6 * (size_t)cid);
      next_chunk_off[crun] = (cn + CHUNK - 1) / CHUNK;
      if (cn > CHUNK) next_multi[atomicAdd(&nmulti, 1u)] = crun;   // the list's order does not matter
      pts += cn;
      small += cn < (uint32_t)SMALL_NODE ? 1u : 0u;
    }
  }
  __syncthreads();
  // total points of the next level (integer sum: exact in any order)
  uint32_t next_points, next_small;
  (void)scan_1024(pts, wsum, next_points);
  (void)scan_1024(small, wsum, next_small);
  // exclusive scan of the children's chunk counts
  const uint32_t seg2 = (total + 1023u) / 1024u;
  const uint32_t b2 = min(total, tid * seg2), e2 = min(total, b2 + seg2);
  uint32_t sum2 = 0;
  for (uint32_t i0 = b2; i0 < e2; i0 += EB) {
    uint32_t v[EB];
#pragma unroll
    for (uint32_t u = 0; u < EB; ++u) v[u] = next_chunk_off[min(i0 + u, e2 - 1)];
#pragma unroll
    for (uint32_t u = 0; u < EB; ++u) sum2 += i0 + u < e2 ? v[u] : 0u;
  }
  uint32_t nchunks_next;
  uint32_t run2 = scan_1024(sum2, wsum, nchunks_next);
  for (uint32_t i0 = b2; i0 < e2; i0 += EB) {
    uint32_t v[EB];
#pragma unroll
    for (uint32_t u = 0; u < EB; ++u) v[u] = next_chunk_off[min(i0 + u, e2 - 1)];
#pragma unroll
    for (uint32_t u = 0; u < EB; ++u)
      if (i0 + u < e2) {
        next_chunk_off[i0 + u] = run2;
        run2 += v[u];
      }
  }
  if (tid == 1023) {
    next_chunk_off[total] = nchunks_next;
    counters[0] = total;
    counters[1] = nchunks_next;
    counters[2] = next_points;
    counters[4] = next_small;
    counters[5] = level_flagged;
    counters[6] = nmulti;
    counters[7] = flagged_chunks;
    if (hostc) {
      // the same counters into host-visible (fine-grained) memory, then the
      // sequence number with a system-scope release: the host waits on it
      hostc[0] = total;
      hostc[1] = nchunks_next;
      hostc[2] = next_points;
      hostc[4] = next_small;
      hostc[5] = level_flagged;
      hostc[6] = nmulti;
      hostc[7] = flagged_chunks;
      __hip_atomic_store(hostc + 3, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// ---------------------------------------------------------------------------
// The same layout for a level of more than EMIT_TILED_MIN nodes, in three
// launches over tiles of EMIT_TILE nodes instead of one workgroup walking
// them all: the tiles' sums (k_emit_count), their exclusive scan and the
// counters (k_emit_scan, one workgroup), then every tile's records from its
// offsets (k_emit_write).  The records, offsets and counters are those of
// k_emit; the multi-chunk list comes out ascending.
// ---------------------------------------------------------------------------
constexpr uint32_t EMIT_TILE = 256;
constexpr uint32_t EMIT_TILED_MIN = 4096;
// per tile: children, their chunks, their points, small children,
// multi-chunk children, flagged nodes, the flagged nodes' chunks
constexpr int EMIT_SUMS = 7;

__device__ __forceinline__ void emit_node_sums(const LevelArgs& a, const uint32_t* __restrict__ ccnt, uint32_t i,
                                               uint32_t mask, uint32_t flags, uint32_t s[EMIT_SUMS]) {
#pragma unroll
  for (int q = 0; q < EMIT_SUMS; ++q) s[q] = 0;
  s[0] = (uint32_t)__popc(mask);
#pragma unroll
  for (uint32_t o = 0; o < 8u; ++o)
    if ((mask >> o) & 1u) {
      const uint32_t cn = ccnt[(size_t)i * 8 + o];
      s[1] += (cn + CHUNK - 1) / CHUNK;
      s[2] += cn;
      s[3] += cn < (uint32_t)SMALL_NODE ? 1u : 0u;
      s[4] += cn > (uint32_t)CHUNK ? 1u : 0u;
    }
  if (flags & FLAG_REFINE) {
    s[5] = 1;
    s[6] = a.chunk_off[i + 1] - a.chunk_off[i];
  }
}

__global__ void __launch_bounds__(EMIT_TILE) k_emit_count(LevelArgs a, const uint32_t* __restrict__ ccnt,
                                                          uint32_t* __restrict__ tsum) {
  __shared__ uint32_t wsum[EMIT_TILE / 64];
  const uint32_t i = blockIdx.x * EMIT_TILE + threadIdx.x;
  uint32_t mask = 0, flags = 0;
  if (i < a.nnodes) {
    mask = a.nt.child_mask[a.node0 + i];
    flags = a.nt.flags[a.node0 + i];
  }
  uint32_t s[EMIT_SUMS];
  emit_node_sums(a, ccnt, i, mask, flags, s);
#pragma unroll
  for (int q = 0; q < EMIT_SUMS; ++q) {
    uint32_t t;
    (void)scan_block<EMIT_TILE>(s[q], wsum, t);
    if (threadIdx.x == 0) tsum[(size_t)blockIdx.x * 8 + q] = t;
  }
}

// tsum: the tiles' sums in, their exclusive prefixes out (in place);
// counters as k_emit's, and counters[8] = 0 for k_emit_write's count of
// finished workgroups
// (a workgroup of four waves: on a device busy with other streams' kernels
// it finds room on a compute unit sooner than one of sixteen)
__global__ void __launch_bounds__(EMIT_TILE) k_emit_scan(uint32_t ntiles, uint32_t m, uint32_t* __restrict__ tsum,
                                                         uint32_t* __restrict__ next_chunk_off,
                                                         uint32_t* __restrict__ sel, uint32_t* __restrict__ counters) {
  __shared__ uint32_t wsum[EMIT_TILE / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t seg = (ntiles + EMIT_TILE - 1) / EMIT_TILE;
  const uint32_t b = min(ntiles, tid * seg), e = min(ntiles, b + seg);
  uint32_t tot[EMIT_SUMS];
#pragma unroll
  for (int q = 0; q < EMIT_SUMS; ++q) {
    uint32_t x = 0;
    for (uint32_t t = b; t < e; ++t) x += tsum[(size_t)t * 8 + q];
    uint32_t run = scan_block<EMIT_TILE>(x, wsum, tot[q]);
    for (uint32_t t = b; t < e; ++t) {
      const uint32_t v = tsum[(size_t)t * 8 + q];
      tsum[(size_t)t * 8 + q] = run;
      run += v;
    }
  }
  if (tid == 0) {
    next_chunk_off[tot[0]] = tot[1];
    if (sel) sel[m + 1 + tot[5]] = tot[6];
    counters[0] = tot[0];
    counters[1] = tot[1];
    counters[2] = tot[2];
    counters[4] = tot[3];
    counters[5] = tot[5];
    counters[6] = tot[4];
    counters[7] = tot[6];
    counters[8] = 0;
  }
}

__global__ void __launch_bounds__(EMIT_TILE) k_emit_write(LevelArgs a, const ProblemParams* __restrict__ prm,
                                                          const uint32_t* __restrict__ cbeg,
                                                          const uint32_t* __restrict__ ccnt, uint32_t next0,
                                                          const uint32_t* __restrict__ toff, uint32_t ntiles,
                                                          uint32_t* __restrict__ next_chunk_off,
                                                          uint32_t* __restrict__ next_multi, uint32_t* __restrict__ sel,
                                                          uint32_t* __restrict__ counters, uint32_t* __restrict__ hostc,
                                                          uint32_t seq) {
  __shared__ uint32_t wsum[EMIT_TILE / 64];
  __shared__ uint32_t last;
  const uint32_t tile = blockIdx.x, i = tile * EMIT_TILE + threadIdx.x;
  const bool in = i < a.nnodes;
  const uint32_t node = a.node0 + i;
  uint32_t mask = 0, flags = 0;
  if (in) {
    mask = a.nt.child_mask[node];
    flags = a.nt.flags[node];
  }
  uint32_t s[EMIT_SUMS];
  emit_node_sums(a, ccnt, i, mask, flags, s);
  // the node's first child, first child chunk, first multi-chunk list entry,
  // flagged-list entry and first flagged chunk
  uint32_t ex[EMIT_SUMS] = {};
#pragma unroll
  for (int q = 0; q < EMIT_SUMS; ++q) {
    if (q == 2 || q == 3) continue;   // totals only
    uint32_t t;
    ex[q] = scan_block<EMIT_TILE>(s[q], wsum, t) + toff[(size_t)tile * 8 + q];
  }
  if (in && mask) {
    a.nt.first_child[node] = next0 + ex[0];
    const uint32_t prob = a.nt.problem[node], pre = a.nt.prefix[node];
    uint32_t crun = ex[0], chunk = ex[1], mrun = ex[4];
    for (uint32_t o = 0; o < 8u; ++o) {
      if (!((mask >> o) & 1u)) continue;
      const uint32_t cid = next0 + crun;
      const uint32_t cpre = (pre << 3) | o;
      const uint32_t cn = ccnt[(size_t)i * 8 + o];
      a.nt.begin[cid] = cbeg[(size_t)i * 8 + o];
      a.nt.count[cid] = cn;
      a.nt.prefix[cid] = cpre;
      a.nt.level[cid] = (uint32_t)(a.level + 1);
      a.nt.problem[cid] = prob;
      a.nt.parent[cid] = node;
      a.nt.first_child[cid] = 0;
      a.nt.child_mask[cid] = 0;
      a.nt.flags[cid] = 0;
      node_geo(prm[prob], a.level + 1, cpre, a.nt.geo + 6 * (size_t)cid);
      next_chunk_off[crun] = chunk;
      chunk += (cn + CHUNK - 1) / CHUNK;
      if (cn > (uint32_t)CHUNK) next_multi[mrun++] = crun;
      ++crun;
    }
  }
  if (sel && in && (flags & FLAG_REFINE)) {
    sel[ex[5]] = i;
    sel[a.nnodes + 1 + ex[5]] = ex[6];
  }
  // the last workgroup to finish hands the counters to the host (after it,
  // this launch writes nothing the host could release)
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(counters + 8, 1u) == ntiles - 1 ? 1u : 0u;
  __syncthreads();
  if (last && threadIdx.x == 0 && hostc) {
    __threadfence();
    hostc[0] = counters[0];
    hostc[1] = counters[1];
    hostc[2] = counters[2];
    hostc[4] = counters[4];
    hostc[5] = counters[5];
    hostc[6] = counters[6];
    hostc[7] = counters[7];
    __hip_atomic_store(hostc + 3, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
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
static hipError_t solve_m_impl(const LevelArgs& a, const double* part_m, const double* part_b, const double* pyr,
                               double* fac, hipStream_t s) {
  if (a.nnodes == 0) return hipSuccess;
  hipLaunchKernelGGL(k_solve_m<P>, dim3(a.nnodes), dim3(256), 0, s, a, part_m, part_b, pyr, fac);
  return hipGetLastError();
}
hipError_t launch_solve_moments(int p, const LevelArgs& a, const double* part_m, const double* part_b,
                                const double* pyr, double* fac, hipStream_t s) {
  if (solve_reg_order(p)) return launch_solve_reg(p, a, part_m, part_b, pyr, fac, s);
  FMT_DISPATCH_P(p, solve_m_impl, a, part_m, part_b, pyr, fac, s);
}

template <int P>
static hipError_t rsolve_impl(const LevelArgs& a, const double* part_b, const double* fac, hipStream_t s) {
  const uint32_t n = a.sel ? a.nsel : a.nnodes;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_refine_solve<P>, dim3(n, field_rows(a)), dim3(256), 0, s, a, part_b, fac);
  return hipGetLastError();
}
hipError_t launch_refine_solve(int p, const LevelArgs& a, const double* part_b, const double* fac, hipStream_t s) {
  FMT_DISPATCH_P(p, rsolve_impl, a, part_b, fac, s);
}

template <int P>
static hipError_t factor_m_impl(const LevelArgs& a, const double* part_m, double* fac, hipStream_t s) {
  if (a.nnodes == 0) return hipSuccess;
  hipLaunchKernelGGL(k_factor_m<P>, dim3(a.nnodes), dim3(256), 0, s, a, part_m, fac);
  return hipGetLastError();
}
hipError_t launch_factor_moments(int p, const LevelArgs& a, const double* part_m, double* fac, hipStream_t s) {
  FMT_DISPATCH_P(p, factor_m_impl, a, part_m, fac, s);
}

template <int P>
static hipError_t ahead_impl(const LevelArgs& a, const double* part_b, double* fac, hipStream_t s) {
  if (a.nnodes == 0 || !a.fac_up || !a.pyr_tab) return hipSuccess;
  hipLaunchKernelGGL(k_solve_ahead<P>, dim3(a.nnodes), dim3(256), 0, s, a, part_b, fac);
  return hipGetLastError();
}
hipError_t launch_solve_ahead(int p, const LevelArgs& a, const double* part_b, double* fac, hipStream_t s) {
  FMT_DISPATCH_P(p, ahead_impl, a, part_b, fac, s);
}

template <int P>
static hipError_t fcells_impl(const double* pyr, const uint32_t* list, uint32_t n, int refine, double* fac_up,
                              uint32_t* up_flags, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_factor_cells<P>, dim3(n), dim3(256), 0, s, pyr, list, refine, fac_up, up_flags);
  return hipGetLastError();
}
hipError_t launch_factor_cells(int p, const double* pyr, const uint32_t* list, uint32_t n, int refine,
                               double* fac_up, uint32_t* up_flags, hipStream_t s) {
  FMT_DISPATCH_P(p, fcells_impl, pyr, list, n, refine, fac_up, up_flags, s);
}

template <int P>
static hipError_t fsolve_impl(const LevelArgs& a, const double* part_b, const double* fac, hipStream_t s) {
  if (a.nnodes == 0) return hipSuccess;
  hipLaunchKernelGGL(k_factor_solve<P>, dim3(a.nnodes), dim3(256), 0, s, a, part_b, fac);
  return hipGetLastError();
}
hipError_t launch_factor_solve(int p, const LevelArgs& a, const double* part_b, const double* fac, hipStream_t s) {
  FMT_DISPATCH_P(p, fsolve_impl, a, part_b, fac, s);
}

template <int P>
static hipError_t resid_impl(int dtype, const LevelArgs& a, double* part_ss, hipStream_t s) {
  const uint32_t n = a.sel ? a.nsel_chunks : a.nchunks;
  if (n == 0) return hipSuccess;
  const dim3 grid(n, field_rows(a));
  const dim3 block(ResidualShape<P>::THREADS);
  if (a.sel) {
    if (dtype == FMT_F32) hipLaunchKernelGGL((k_residual<P, float, true, false>), grid, block, 0, s, a, part_ss);
    else hipLaunchKernelGGL((k_residual<P, double, true, false>), grid, block, 0, s, a, part_ss);
    return hipGetLastError();
  }
  // the larger nodes, then (p > 3) those under SMALL_NODE points; a level
  // whose small-node count is known skips a launch it has no node for
  const bool split = ResidualShape<P>::SPLIT;
  if (!split || a.nsmall == UINT32_MAX || a.nsmall < a.nnodes) {
    if (dtype == FMT_F32) hipLaunchKernelGGL((k_residual<P, float, false, false>), grid, block, 0, s, a, part_ss);
    else hipLaunchKernelGGL((k_residual<P, double, false, false>), grid, block, 0, s, a, part_ss);
  }
  if (split && a.nsmall > 0) {
    const dim3 sblock(ResidualShape<P, true>::THREADS);
    if (dtype == FMT_F32) hipLaunchKernelGGL((k_residual<P, float, false, true>), grid, sblock, 0, s, a, part_ss);
    else hipLaunchKernelGGL((k_residual<P, double, false, true>), grid, sblock, 0, s, a, part_ss);
  }
  return hipGetLastError();
}
hipError_t launch_residual(int p, int dtype, const LevelArgs& a, double* part_ss, hipStream_t s) {
  FMT_DISPATCH_P_ALL(p, resid_impl, dtype, a, part_ss, s);
}

template <int P>
static hipError_t residf_impl(int dtype, const LevelArgs& a, hipStream_t s) {
  if (a.nchunks == 0) return hipSuccess;
  if (dtype == FMT_F32) hipLaunchKernelGGL((k_residual_fields<P, float>), dim3(a.nchunks), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_residual_fields<P, double>), dim3(a.nchunks), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_residual_fields(int p, int dtype, const LevelArgs& a, hipStream_t s) {
  FMT_DISPATCH_P(p, residf_impl, dtype, a, s);
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
  FMT_DISPATCH_P_ALL(p, children_impl, a, part_ss, cbeg, ccnt, nact, s);
}

hipError_t launch_emit(const LevelArgs& a, const ProblemParams* prm, const uint32_t* cbeg, const uint32_t* ccnt,
                       uint32_t* nact, uint32_t next0, uint32_t* next_chunk_off, uint32_t* counters, uint32_t* hostc,
                       uint32_t seq, uint32_t* next_multi, uint32_t* sel, uint32_t* tiles, hipStream_t s) {
  if (a.nnodes <= EMIT_TILED_MIN) {
    hipLaunchKernelGGL(k_emit, dim3(1), dim3(1024), 0, s, a, prm, cbeg, ccnt, nact, next0, next_chunk_off, counters,
                       hostc, seq, next_multi, sel);
    return hipGetLastError();
  }
  if (!tiles) return hipErrorInvalidValue;
  const uint32_t ntiles = (a.nnodes + EMIT_TILE - 1) / EMIT_TILE;
  hipLaunchKernelGGL(k_emit_count, dim3(ntiles), dim3(EMIT_TILE), 0, s, a, ccnt, tiles);
  hipLaunchKernelGGL(k_emit_scan, dim3(1), dim3(EMIT_TILE), 0, s, ntiles, a.nnodes, tiles, next_chunk_off, sel,
                     counters);
  hipLaunchKernelGGL(k_emit_write, dim3(ntiles), dim3(EMIT_TILE), 0, s, a, prm, cbeg, ccnt, next0, tiles, ntiles,
                     next_chunk_off, next_multi, sel, counters, hostc, seq);
  return hipGetLastError();
}

size_t emit_tile_words(uint32_t nnodes) {
  return nnodes <= EMIT_TILED_MIN ? 0 : 8ull * ((nnodes + EMIT_TILE - 1) / EMIT_TILE);
}

hipError_t launch_chunk_reduce(const LevelArgs& a, double* buf, uint32_t width, hipStream_t s) {
  if (a.nnodes == 0 || a.nchunks <= a.nnodes) return hipSuccess;
  const uint32_t nlaunch = a.multi ? a.nmulti : a.nnodes;
  if (nlaunch == 0) return hipSuccess;
  const uint32_t eblocks = (width + 63) / 64;
  hipLaunchKernelGGL(k_chunk_reduce, dim3(nlaunch * eblocks, field_rows(a)), dim3(1024), 0, s, a.chunk_off,
                     a.nnodes, buf, width, eblocks, (uint64_t)a.nchunks * width, a.nt.flags + a.node0, a.only_flag,
                     a.multi, a.nmulti);
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
  FMT_DISPATCH_P_ALL(p, check_impl, nt, nnodes, status, s);
}

}  // namespace fmt
