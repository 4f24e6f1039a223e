// Per-node solve of the normal equations (Alg. 2 on the equilibrated normal
// equations, as k_solve_m) for the small bases, p <= 6 (calL <= 84), with the
// whole matrix held in the registers of one wave.
//
// The LDS-resident factor of k_solve_m keeps 53 KB per node at p = 6 and
// needs four waves per node.  Here one wave owns a node: the upper block
// triangle of the padded matrix (T = ceil(calL / 16) blocks a side,
// T (T + 1) / 2 blocks of 16 x 16) lives in the wave's registers in the
// layout of the float64 MFMA accumulator, so lane l, register j of block
// (J, I) holds element (16 J + 4 j + (l >> 4), 16 I + (l & 15)).  In that
// layout register s of a block of rows of U is at the same time the A operand
// (transposed) and the B operand of a 16 x 16 x 4 MFMA step, so the trailing
// updates need no data movement at all.  LDS holds only vectors and the
// node's moments (10 KB at p = 6).  Up to p = 4 two or more such waves share
// a SIMD; at p = 5 and 6 the matrix and the solve's vectors take the whole
// register file of a SIMD (one wave each, four nodes a compute unit), and the
// kernel is about as fast as the LDS one at p = 6 (one wave issues most of
// its instructions back to back: the work per node, ~90 k SIMD cycles, is
// about what the four waves of the LDS factor spend), faster below.
//
// The factor is an upper-form LDL^T, S = U^T D U, right-looking by block rows:
//   (a) block row J: 16 pivot steps; the pivot comes from its lane with
//       v_readlane, row k of the block row from its row of lanes and the
//       multipliers S(k, m) / d_k of the lane's rows from row k as well
//       (ds_bpermute, all at once); rows m <= k keep their values
//       (multiplier 0: the rows of U, unscaled).  Every update reads the
//       upper triangle only, so the elimination stays symmetric however the
//       rounding falls (with the multipliers taken from column k instead,
//       the two triangles drift apart by rounding, and on nearly singular
//       nodes that moves which pivots fall under the deflation threshold);
//   (b) the blocks right of and below: S_KI -= S_JK^T diag(1 / d_J) S_JI,
//       J < K <= I, on float64 MFMA straight from the registers.
// Pivots at or below PIVOT_EPS are deflated (inverse 0), as in k_solve_m.
// The right-hand side and the two condition-estimate probes ride along as
// three extra columns in the padding (calL + 3 <= 16 T for every p <= 6), so
// the elimination performs the forward substitution; the back substitution
// z_m = (y_m - sum_{n > m} S(m, n) z_n) / d_m runs block by block, with the
// products of the blocks right of the diagonal reduced across each row of
// 16 lanes.  Coefficients, flags and the kept factor (for the refinement) are
// those of k_solve_m, in the same formats.
#include <utility>

#include "k_ldl.h"
#include "k_level.h"

namespace fmt {

typedef double reg_d4 __attribute__((ext_vector_type(4)));

// f(0), f(1), ..., f(E - 1 - B) as compile-time constants
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

template <int L>
struct RegShape {
  static constexpr int T = (L + 15) / 16;
  static constexpr int LP = 16 * T;
  static constexpr int NB = T * (T + 1) / 2;
  // waves per SIMD the register allocation aims at: two or more while the
  // matrix (8 NB registers a lane) leaves room for the solve's vectors
  // (p <= 4), one above
  static constexpr int WAVES = NB <= 6 ? 2 : 1;
};

// Number of the upper block (J, I), J <= I, counted row by row.
template <int T>
__host__ __device__ constexpr int ub(int J, int I) {
  return J * T - J * (J - 1) / 2 + (I - J);
}

__device__ __forceinline__ double join_d(int lo, int hi) {
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// x of lane K of the lane's row of 16 lanes (DPP row_newbcast).
template <int K>
__device__ __forceinline__ double row_bcast(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x150 + K, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x150 + K, 0xf, 0xf, false);
  return join_d(lo, hi);
}

// x of the lane in row G of lanes (lanes 16 G .. 16 G + 15) at the lane's own
// position in its row.
template <int G>
__device__ __forceinline__ double from_row(double x, int lane) {
  const int addr = ((G << 4) | (lane & 15)) << 2;
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
  return join_d(lo, hi);
}

// x of lane src (any lane index, lane-dependent).
__device__ __forceinline__ double from_lane(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
  return join_d(lo, hi);
}

// Sum over the lane's row of 16 lanes by butterflies: every lane of the row
// ends with the same bits (each stage adds the same two values, commuted).
__device__ __forceinline__ double row_sum(double x) {
  x += __shfl_xor(x, 8, 16);
  x += __shfl_xor(x, 4, 16);
  x += __shfl_xor(x, 2, 16);
  x += __shfl_xor(x, 1, 16);
  return x;
}

template <int P>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(RegShape<basis_size(P)>::WAVES)))
k_solve_reg(LevelArgs a, const double* __restrict__ part_m, const double* __restrict__ part_b,
            const double* __restrict__ pyr, double* __restrict__ fac) {
  constexpr int L = basis_size(P);
  constexpr int NM = basis_size(2 * P);
  constexpr int NOUT = NM + L + 1;
  using R = RegShape<L>;
  constexpr int T = R::T, LP = R::LP;
  static_assert(LP - L >= 3, "the right-hand side and the probes need three padding columns");
  constexpr Basis<P> B{};
  __shared__ double wv[LP], sc[LP], dv[LP], iv[LP];
  __shared__ uint32_t ex[LP];                    // exponents, packed a | b << 8 | c << 16 (0 on the padding)
  __shared__ int tet[2 * P + 1], tri[2 * P + 1];   // k (k+1) (k+2) / 6 and k (k+1) / 2: graded() in two lookups
  __shared__ double rhs[3][LP];   // right-hand sides, then (as zs) their solutions
  __shared__ double mom[NM + L];  // M, then B
  double(*zs)[LP] = rhs;
  const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
  const uint32_t k = blockIdx.x;
  const uint32_t node = a.node0 + k;
  if (a.only_flag && !(a.nt.flags[node] & a.only_flag)) return;   // not this pass's node
  const uint32_t* pt = a.pyr_tab ? a.pyr_tab + PYR_TAB_WORDS * a.nt.problem[node] : nullptr;
  if (pt && a.fac_up && (pt[3] >> 28) > (uint32_t)a.level) return;   // factored ahead: k_solve_ahead
  const uint32_t c0 = a.chunk_off[k];   // chunks of the node were summed into this one
  const double* ms;
  const double* bs;
  if (pt && pyramid_covers(pt[1], a.level)) {
    ms = pyr + ((size_t)pt[0] + level_first(a.level) + a.nt.prefix[node]) * NM;
    bs = part_b + (size_t)c0 * L;
  } else {
    ms = part_m + (size_t)c0 * NOUT;
    bs = ms + NM;
  }
  const int refine = a.refine;
  const bool estimate = refine == 1;
  // the moments into LDS (all loads in flight before the first store): the
  // assembly gathers from them with 32-bit addresses
  {
    constexpr int RM = (NM + 63) / 64, RB = (L + 63) / 64;
    double vm[RM], vb[RB];
#pragma unroll
    for (int q = 0; q < RM; ++q) vm[q] = lane + 64 * q < NM ? ms[lane + 64 * q] : 0.0;
#pragma unroll
    for (int q = 0; q < RB; ++q) vb[q] = lane + 64 * q < L ? bs[lane + 64 * q] : 0.0;
#pragma unroll
    for (int q = 0; q < RM; ++q)
      if (lane + 64 * q < NM) mom[lane + 64 * q] = vm[q];
#pragma unroll
    for (int q = 0; q < RB; ++q)
      if (lane + 64 * q < L) mom[NM + lane + 64 * q] = vb[q];
  }
  __syncthreads();

  // equilibration s_i = 1 / sqrt(G_ii), w_i = s_i / alpha_i!, the scaled
  // right-hand side and the probes; padding entries 0
  if (lane <= 2 * P) {
    tet[lane] = lane * (lane + 1) * (lane + 2) / 6;
    tri[lane] = lane * (lane + 1) / 2;
  }
  for (int i = lane; i < LP; i += 64) {
    uint32_t e = 0u;
    double s = 0.0, w = 0.0, bb = 0.0, x0 = 0.0, x1 = 0.0;
    if (i < L) {
      e = (uint32_t)B.lx[i] | ((uint32_t)B.ly[i] << 8) | ((uint32_t)B.lz[i] << 16);
      const double f = B.inv_fact[i];
      const double gii = mom[graded(2 * B.lx[i], 2 * B.ly[i], 2 * B.lz[i])] * f * f;
      s = gii > 0.0 ? 1.0 / sqrt(gii) : 0.0;
      w = s * f;
      bb = mom[NM + i] * s * f;
      if (estimate) {
        x0 = probe_entry(i, 0, L);
        x1 = probe_entry(i, 1, L);
      }
    }
    ex[i] = e;
    sc[i] = s;
    wv[i] = w;
    rhs[0][i] = bb;
    rhs[1][i] = x0;
    rhs[2][i] = x1;
  }
  __syncthreads();

  // S(m, n) = M[alpha_m + alpha_n] w_m w_n; padding rows and columns the
  // identity, except the three right-hand-side columns calL .. calL + 2
  reg_d4 blk[R::NB];
  sfor<0, T>([&](auto Jc) {
    constexpr int J = Jc;
    double wr[4];
    uint32_t er[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      wr[j] = wv[16 * J + 4 * j + g];
      er[j] = ex[16 * J + 4 * j + g];
    }
    sfor<J, T>([&](auto Ic) {
      constexpr int I = Ic;
      const int n = 16 * I + c;
      const double wc = wv[n];
      const uint32_t ec = ex[n];
      const int rr = (n >= L && n < L + 3) ? n - L : 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = 16 * J + 4 * j + g;
        const uint32_t e = er[j] + ec;   // alpha_m + alpha_n, packed a | b << 8 | c << 16
        const int ea = (int)(e & 255u), eb = (int)((e >> 8) & 255u), ek = ea + eb + (int)(e >> 16);
        const double mv = mom[tet[ek] + tri[ek - ea] + (ek - ea - eb)];
        const double rv = rhs[rr][m < L ? m : 0];   // read unconditionally: no branch in the assembly
        const double pad = (m < L && n >= L && n < L + 3) ? rv : (m == n ? 1.0 : 0.0);
        blk[ub<T>(J, I)][j] = (m < L && n < L) ? mv * wr[j] * wc : pad;
      }
    });
  });

  // factor, block row by block row
  bool defl = false;
  sfor<0, T>([&](auto Jc) {
    constexpr int J = Jc;
    constexpr int KMAX = L - 16 * J < 16 ? L - 16 * J : 16;   // pivots of this block row (the rest is padding)
    double ivj[4] = {0.0, 0.0, 0.0, 0.0};                    // 1 / d of the lane's rows 4 j + g
    double dc = 1.0, ivc = 1.0;                              // d and 1 / d of pivot c (stored after the panel)
    sfor<0, KMAX>([&](auto Kc) {
      constexpr int kk = Kc, kr = kk >> 2, kg = kk & 3;
      // row k of the block row, S(k, 16 I + c): all of its broadcasts in
      // flight together, alongside the pivot's reciprocal
      double rk[T];
      sfor<J, T>([&](auto Ic) {
        constexpr int I = Ic;
        rk[I] = from_row<kg>(blk[ub<T>(J, I)][kr], lane);
      });
      // and S(k, m) for the lane's rows m = 16 J + 4 j + g: the multipliers
      // come from row k too, so that every update reads the upper triangle
      // alone and stays symmetric (the lower triangle of the diagonal block
      // takes rounding of its own and is never read)
      double skm[4];
      sfor<kr, 4>([&](auto jc) {
        constexpr int j = jc;
        skm[j] = from_lane(blk[ub<T>(J, J)][kr], (kg << 4) | (4 * j + g));
      });
      const double d = lane_value(blk[ub<T>(J, J)][kr], 16 * kg + kk);
      const double inv = d > PIVOT_EPS ? pivot_recip(d) : 0.0;
      defl |= inv == 0.0;
      dc = c == kk ? d : dc;
      ivc = c == kk ? inv : ivc;
      if (g == kg) ivj[kr] = inv;
      // multipliers S(k, m) / d_k of the lane's rows m = 4 j + g > k
      double mu[4];
      sfor<kr, 4>([&](auto jc) {
        constexpr int j = jc;
        mu[j] = (j > kr || g > kg) ? skm[j] * inv : 0.0;
      });
      sfor<J, T>([&](auto Ic) {
        constexpr int I = Ic;
        sfor<kr, 4>([&](auto jc) {
          constexpr int j = jc;
          // rows m <= k of register kr have mu = 0 and stay as they are
          blk[ub<T>(J, I)][j] = fma(-mu[j], rk[I], blk[ub<T>(J, I)][j]);
        });
      });
    });
    if (g == 0) {
      dv[16 * J + c] = dc;
      iv[16 * J + c] = ivc;
    }
    // S_KI -= S_JK^T diag(1 / d_J) S_JI for J < K <= I
    // (k-step outermost, so that consecutive MFMAs are independent)
    sfor<J + 1, T>([&](auto Kc) {
      constexpr int K = Kc;
      double av[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) av[s] = -blk[ub<T>(J, K)][s] * ivj[s];
#pragma unroll
      for (int s = 0; s < 4; ++s)
        sfor<K, T>([&](auto Ic) {
          constexpr int I = Ic;
          blk[ub<T>(K, I)] =
              __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], blk[ub<T>(J, I)][s], blk[ub<T>(K, I)], 0, 0, 0);
        });
    });
  });
  __syncthreads();   // dv and iv in LDS

  // back substitution for the first NR right-hand sides (columns calL ..
  // calL + NR - 1) together, so that each broadcast of a column of S serves
  // all of them; the solutions go to zs[r][0 .. LP) (0 on the padding)
  auto back = [&](auto NRc) {
    constexpr int NR = NRc;
    sfor<0, T>([&](auto Jr) {
      constexpr int J = T - 1 - (int)Jr;
      constexpr int KMAX = L - 16 * J < 16 ? L - 16 * J : 16;
      // t = y - (blocks right of the diagonal) z, for the lane's rows 4 j + g
      double t[NR][4];
      sfor<0, NR>([&](auto rc) {
        constexpr int r = rc;
        constexpr int CA = (L + r) & 15;   // the right-hand side's column in the last block column
        double zr[T];
#pragma unroll
        for (int I = J + 1; I < T; ++I) zr[I] = zs[r][16 * I + c];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          double p = 0.0;
          sfor<J + 1, T>([&](auto Ic) {
            constexpr int I = Ic;
            p = fma(blk[ub<T>(J, I)][j], zr[I], p);
          });
          if constexpr (J + 1 < T) p = row_sum(p);
          t[r][j] = row_bcast<CA>(blk[ub<T>(J, T - 1)][j]) - p;
        }
      });
      double zcur[NR];   // z_{16 J + c} of this block, as the steps find them
#pragma unroll
      for (int r = 0; r < NR; ++r) zcur[r] = 0.0;
      double ivb[16];   // the block's 1 / d, loaded together
#pragma unroll
      for (int q = 0; q < 16; ++q) ivb[q] = iv[16 * J + q];
      sfor<0, KMAX>([&](auto Kr) {
        constexpr int kk = KMAX - 1 - (int)Kr, kr = kk >> 2, kg = kk & 3;
        const double ivk = ivb[kk];
        double zk[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          zk[r] = lane_value(t[r][kr], 16 * kg) * ivk;
          zcur[r] = c == kk ? zk[r] : zcur[r];
        }
        // rows above k in this block (rows at or below k are solved: their t
        // is no longer read)
        sfor<0, kr + 1>([&](auto jc) {
          constexpr int j = jc;
          const double sv = row_bcast<kk>(blk[ub<T>(J, J)][j]);
#pragma unroll
          for (int r = 0; r < NR; ++r) t[r][j] = fma(-sv, zk[r], t[r][j]);
        });
      });
      if (g == 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r) zs[r][16 * J + c] = zcur[r];
      }
      __syncthreads();
    });
  };

  uint32_t* flag = a.nt.flags + node;
  if (estimate) back(std::integral_constant<int, 3>{});
  else back(std::integral_constant<int, 1>{});
  {
    bool bad = false;
    double* coef = a.nt.coef + (size_t)node * L;
    for (int i = lane; i < L; i += 64) {
      const double cf = sc[i] * zs[0][i];
      coef[i] = cf;
      bad |= !__builtin_isfinite(cf);
    }
    mark_nonfinite(bad, flag, a.status);
  }
  bool need_factor = refine == 2;
  if (estimate) {
    // |G^-1 x| for the two probes (x of norm 1): close to 1 / lambda_min
    double s1 = 0.0, s2 = 0.0;
    for (int i = lane; i < L; i += 64) {
      s1 = fma(zs[1][i], zs[1][i], s1);
      s2 = fma(zs[2][i], zs[2][i], s2);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      s1 += __shfl_xor(s1, off);
      s2 += __shfl_xor(s2, off);
    }
    const double k1 = (double)L * sqrt(s1), k2 = (double)L * sqrt(s2);
    if (k1 > REFINE_KAPPA || k2 > REFINE_KAPPA) {
      if (lane == 0) atomicOr(flag, FLAG_REFINE);
      need_factor = true;
    }
  }
  if (refine == 2) {
    if (lane == 0) atomicOr(flag, FLAG_REFINE);
  } else if (estimate && defl) {
    if (lane == 0) atomicOr(flag, FLAG_REFINE);
    need_factor = true;
  }
  // the factor is kept only for the nodes the refinement sweeps will visit,
  // in k_solve_m's blocked lower storage: L(n, m) = S(m, n) / d_m below the
  // diagonal, zero on and above it and on the padding
  if (fac && need_factor) {
    double* fo = fac + (size_t)k * factor_words<L>();
    sfor<0, T>([&](auto Jc) {
      constexpr int J = Jc;
      sfor<J, T>([&](auto Ic) {
        constexpr int I = Ic;
        const int n = 16 * I + c;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int m = 16 * J + 4 * j + g;
          const double v = (m < n && n < L) ? blk[ub<T>(J, I)][j] * iv[m] : 0.0;
          fo[(uint32_t)(bidx(I, J) + 16 * c + ((4 * j + g) ^ (c >> 1)))] = v;
        }
        __builtin_amdgcn_sched_barrier(0);
      });
    });
    constexpr int WORDS = BlockShape<L>::WORDS;
    for (int i = lane; i < L; i += 64) {
      fo[WORDS + i] = dv[i];
      fo[WORDS + L + i] = iv[i];
      fo[WORDS + 2 * L + i] = sc[i];
    }
  }
  if (defl && lane == 0) atomicOr(flag, FLAG_DEFLATED);
}

template <int P>
static hipError_t solve_reg_impl(const LevelArgs& a, const double* part_m, const double* part_b, const double* pyr,
                                 double* fac, hipStream_t s) {
  if constexpr (P <= 6) {
    if (a.nnodes == 0) return hipSuccess;
    hipLaunchKernelGGL(k_solve_reg<P>, dim3(a.nnodes), dim3(64), 0, s, a, part_m, part_b, pyr, fac);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

bool solve_reg_order(int p) { return p >= 0 && p <= 6; }

hipError_t launch_solve_reg(int p, const LevelArgs& a, const double* part_m, const double* part_b, const double* pyr,
                            double* fac, hipStream_t s) {
  FMT_DISPATCH_P(p, solve_reg_impl, a, part_m, part_b, pyr, fac, s);
  return hipErrorInvalidValue;
}

}  // namespace fmt
