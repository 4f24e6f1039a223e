// Gaussian-RBF factorisation (Section 2, eq. fullyfactored).
//
// The Gaussian kernel between query points x_q and points x_i, expanded in
// Taylor series and truncated to the calL monomials of degree <= p on each
// side, is a product of three dense factors:
//   phi'_{q i} = Lambda(x_q) . C . Lambda(x_i)^T,  C = E T E,
// with E = diag(eps^|alpha|) and T the matrix of Hermite numbers.  Both
// products are dense contractions over the basis, so they run on float64
// MFMA: first B = Lambda(X) C (one row of calL per point), then
// phi' = Lambda(X_q) B^T, an nq x n block written row by row.  One kernel
// does either product: out[q][i] = sum_k Lambda_k(x_q) R[i][k] for the rows R
// (C's rows, or B's).
#include "k_level.h"

namespace fmt {

typedef double rbf_d4 __attribute__((ext_vector_type(4)));

constexpr int RBF_TILE = 64;   // output tile edge (queries and rows)
constexpr int RBF_K = 64;      // basis entries staged per round
constexpr int RBF_LD = RBF_K + 1;

// out[q * ostride + i] = sum_{k < L} Lambda_k(x_q) R[i * LS + k] for q < nq,
// i < nr.  Workgroup: a 64 x 64 tile of (q, i); its four waves take 32 x 32
// quadrants as 2 x 2 blocks of 16 x 16 on MFMA (float64, k = 4 per step).
// Per round the 64 queries' basis values for 64 entries of k (from their
// scaled powers t^k / k!, held in LDS) and the 64 rows' matching entries are
// staged in LDS.  expo: packed exponents l | m << 8 | n << 16 of each basis
// index (graded order).  R must hold finite values (zeros) in its padding
// columns L .. LS - 1.
template <typename TIN>
__global__ void __launch_bounds__(256) k_rbf_gemm(const TIN* __restrict__ qx, const TIN* __restrict__ qy,
                                                  const TIN* __restrict__ qz, uint32_t nq,
                                                  const double* __restrict__ R, uint32_t nr, uint32_t LS,
                                                  const uint32_t* __restrict__ expo, int L, int p,
                                                  double* __restrict__ out, uint64_t ostride) {
  __shared__ double pw[RBF_TILE][3][16];
  __shared__ double lq[RBF_TILE][RBF_LD];
  __shared__ double rt[RBF_TILE][RBF_LD];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const uint32_t i0 = blockIdx.x * RBF_TILE, q0 = blockIdx.y * RBF_TILE;
  // scaled powers of the tile's queries: pw[r][axis][k] = t^k / k!
  for (int e = tid; e < RBF_TILE * 3; e += 256) {
    const int r = e / 3, ax = e % 3;
    const uint32_t q = min(q0 + (uint32_t)r, nq - 1);
    const double t = (double)(ax == 0 ? qx[q] : (ax == 1 ? qy[q] : qz[q]));
    double v = 1.0;
    pw[r][ax][0] = 1.0;
    for (int k = 1; k <= p; ++k) {
      v = v * t / (double)k;
      pw[r][ax][k] = v;
    }
  }
  const int qr = w >> 1, qc = w & 1;   // this wave's quadrant (query half, row half)
  rbf_d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = rbf_d4{0.0, 0.0, 0.0, 0.0};
  for (uint32_t k0 = 0; k0 < LS; k0 += RBF_K) {
    __syncthreads();   // the powers are written / the previous round's tiles are read
    for (int e = tid; e < RBF_TILE * RBF_K; e += 256) {
      const int r = e / RBF_K, c = e % RBF_K;
      const uint32_t k = k0 + (uint32_t)c;
      double v = 0.0;
      if (k < (uint32_t)L) {
        const uint32_t x = expo[k];
        v = pw[r][0][x & 255u] * pw[r][1][(x >> 8) & 255u] * pw[r][2][x >> 16];
      }
      lq[r][c] = v;
      const uint32_t i = i0 + (uint32_t)r;
      rt[r][c] = i < nr ? R[(size_t)i * LS + k] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < RBF_K; kk += 4) {
      const int kq = kk + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = lq[32 * qr + 16 * a + (lane & 15)][kq];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = rt[32 * qc + 16 * b + (lane & 15)][kq];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  }
  // accumulator element j of a lane: row 4 j + (lane >> 4), column lane & 15
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t q = q0 + 32 * qr + 16 * a + 4 * j + (lane >> 4);
        const uint32_t i = i0 + 32 * qc + 16 * b + (lane & 15);
        if (q < nq && i < nr) out[(size_t)q * ostride + i] = acc[a][b][j];
      }
}

hipError_t launch_rbf_gemm(int dtype, const void* qx, const void* qy, const void* qz, uint32_t nq, const double* R,
                           uint32_t nr, uint32_t LS, const uint32_t* expo, int L, int p, double* out,
                           uint64_t ostride, hipStream_t s) {
  if (nq == 0 || nr == 0) return hipSuccess;
  dim3 grid((nr + RBF_TILE - 1) / RBF_TILE, (nq + RBF_TILE - 1) / RBF_TILE), block(256);
  if (dtype == FMT_F32)
    hipLaunchKernelGGL(k_rbf_gemm<float>, grid, block, 0, s, (const float*)qx, (const float*)qy, (const float*)qz, nq,
                       R, nr, LS, expo, L, p, out, ostride);
  else
    hipLaunchKernelGGL(k_rbf_gemm<double>, grid, block, 0, s, (const double*)qx, (const double*)qy,
                       (const double*)qz, nq, R, nr, LS, expo, L, p, out, ostride);
  return hipGetLastError();
}

}  // namespace fmt
