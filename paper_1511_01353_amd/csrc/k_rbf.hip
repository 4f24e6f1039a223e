// Gaussian-RBF factorisation (Section 2, eq. fullyfactored).
//
// The Gaussian kernel between query points x_q and points x_i, expanded in
// Taylor series and truncated to the calL monomials of degree <= p on each
// side, is a product of three dense factors:
//   phi'_{q i} = Lambda(x_q) . C . Lambda(x_i)^T,  C = E T E,
// with E = diag(eps^|alpha|) and T the matrix of Hermite numbers.  The basis
// values of both point sets are formed once (k_rbf_basis), then both
// products are dense contractions over the basis on float64 MFMA: first
// B = Lambda(X) C (one row of calL per point), then phi' = Lambda(X_q) B^T,
// an nq x n block written row by row.  One kernel does either product:
// out[q][i] = sum_k A[q][k] R[i][k] for row-major A and R.
#include "k_level.h"

namespace fmt {

typedef double rbf_d4 __attribute__((ext_vector_type(4)));

constexpr int RBF_TM = 128;    // output tile edge (rows of A and of R)
constexpr int RBF_K = 32;      // basis entries per staged round
constexpr int RBF_LD = RBF_K + 1;
constexpr int RBF_LOADS = RBF_TM * RBF_K / 256;   // doubles of each operand a thread stages per round

// Basis values, row-major with stride LS: A[j][k] = Lambda_k(x_j) for k < L,
// 0 for L <= k < LS.  One thread per entry.
template <typename TIN>
__global__ void __launch_bounds__(256) k_rbf_basis(const TIN* __restrict__ x, const TIN* __restrict__ y,
                                                   const TIN* __restrict__ z, uint32_t n,
                                                   const uint32_t* __restrict__ expo, int L, uint32_t LS,
                                                   double* __restrict__ A) {
  const uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (uint64_t)n * LS) return;
  const uint32_t j = (uint32_t)(e / LS), k = (uint32_t)(e % LS);
  double v = 0.0;
  if (k < (uint32_t)L) {
    const uint32_t ex = expo[k];
    const int l = (int)(ex & 255u), m = (int)((ex >> 8) & 255u), nn = (int)(ex >> 16);
    const double t[3] = {(double)x[j], (double)y[j], (double)z[j]};
    const int pw[3] = {l, m, nn};
    v = 1.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
      for (int a = 1; a <= pw[ax]; ++a) v = v * t[ax] / (double)a;   // t^a / a!, as the basis defines it
  }
  A[e] = v;
}

// out[q * ostride + i] = sum_{k < LS} A[q * LS + k] R[i * LS + k] for
// q < nq, i < nr (A and R zero beyond the basis).  Workgroup: a 128 x 128
// tile of (q, i); each of its four waves takes a 64 x 64 quadrant as 4 x 4
// blocks of 16 x 16 on float64 MFMA (k = 4 per step).  Per round 32 entries of
// k of the tile's 128 rows of A and of R are staged in LDS, and the next
// round's are loaded into registers while the current round multiplies.
__global__ void __launch_bounds__(256) k_rbf_gemm(const double* __restrict__ A, uint32_t nq,
                                                  const double* __restrict__ R, uint32_t nr, uint32_t LS,
                                                  double* __restrict__ out, uint64_t ostride) {
  __shared__ double ta[RBF_TM][RBF_LD];
  __shared__ double tr[RBF_TM][RBF_LD];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const uint32_t i0 = blockIdx.x * RBF_TM, q0 = blockIdx.y * RBF_TM;
  const int qr = w >> 1, qc = w & 1;   // this wave's quadrant (rows of A, rows of R)
  rbf_d4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = rbf_d4{0.0, 0.0, 0.0, 0.0};
  // staging map: entry e = tid + 256 u of the 128 x 32 slice -> row e / 32, column e % 32
  double va[RBF_LOADS], vr[RBF_LOADS];
  auto load = [&](uint32_t k0) {
#pragma unroll
    for (int u = 0; u < RBF_LOADS; ++u) {
      const int e = tid + 256 * u, r = e / RBF_K, c = e % RBF_K;
      const uint32_t q = q0 + (uint32_t)r, i = i0 + (uint32_t)r;
      va[u] = q < nq ? A[(size_t)q * LS + k0 + c] : 0.0;
      vr[u] = i < nr ? R[(size_t)i * LS + k0 + c] : 0.0;
    }
  };
  load(0);
  for (uint32_t k0 = 0; k0 < LS; k0 += RBF_K) {
    __syncthreads();   // the previous round's tiles are read
#pragma unroll
    for (int u = 0; u < RBF_LOADS; ++u) {
      const int e = tid + 256 * u, r = e / RBF_K, c = e % RBF_K;
      ta[r][c] = va[u];
      tr[r][c] = vr[u];
    }
    __syncthreads();
    if (k0 + RBF_K < LS) load(k0 + RBF_K);   // in flight during this round's products
#pragma unroll
    for (int kk = 0; kk < RBF_K; kk += 4) {
      const int kq = kk + (lane >> 4);
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = ta[64 * qr + 16 * a + (lane & 15)][kq];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = tr[64 * qc + 16 * b + (lane & 15)][kq];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  }
  // accumulator element j of a lane: row 4 j + (lane >> 4), column lane & 15
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t q = q0 + 64 * qr + 16 * a + 4 * j + (lane >> 4);
        const uint32_t i = i0 + 64 * qc + 16 * b + (lane & 15);
        if (q < nq && i < nr) out[(size_t)q * ostride + i] = acc[a][b][j];
      }
}

hipError_t launch_rbf_basis(int dtype, const void* x, const void* y, const void* z, uint32_t n, const uint32_t* expo,
                            int L, uint32_t LS, double* A, hipStream_t s) {
  const uint64_t total = (uint64_t)n * LS;
  if (total == 0) return hipSuccess;
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
  if (dtype == FMT_F32)
    hipLaunchKernelGGL(k_rbf_basis<float>, grid, block, 0, s, (const float*)x, (const float*)y, (const float*)z, n,
                       expo, L, LS, A);
  else
    hipLaunchKernelGGL(k_rbf_basis<double>, grid, block, 0, s, (const double*)x, (const double*)y, (const double*)z,
                       n, expo, L, LS, A);
  return hipGetLastError();
}

hipError_t launch_rbf_gemm(const double* A, uint32_t nq, const double* R, uint32_t nr, uint32_t LS, double* out,
                           uint64_t ostride, hipStream_t s) {
  if (nq == 0 || nr == 0) return hipSuccess;
  dim3 grid((nr + RBF_TM - 1) / RBF_TM, (nq + RBF_TM - 1) / RBF_TM), block(256);
  hipLaunchKernelGGL(k_rbf_gemm, grid, block, 0, s, A, nq, R, nr, LS, out, ostride);
  return hipGetLastError();
}

}  // namespace fmt
