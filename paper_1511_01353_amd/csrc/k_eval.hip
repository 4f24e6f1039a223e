// K9: evaluation of a fitted tree at query points.
//
// Section 2 evaluates a fit as f'_q = Lambda'_q . F_p (no need to form the
// transform matrix).  The octree fit is a residual decomposition, so the value
// at a query is the sum of the polynomials of every node on its root-to-leaf
// chain: walk down while the child holding the query's cell exists.
#include "k_level.h"

namespace fmt {

template <int P, typename TQ>
__global__ void __launch_bounds__(256) k_eval(EvalTree t, const TQ* __restrict__ qx, const TQ* __restrict__ qy,
                                              const TQ* __restrict__ qz, const uint32_t* __restrict__ perm,
                                              const uint32_t* __restrict__ skeys, uint32_t nq,
                                              double* __restrict__ out) {
  constexpr int L = basis_size(P);
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const double x = (double)qx[i], y = (double)qy[i], z = (double)qz[i];
  uint32_t key;
  if (skeys) {
    key = skeys[i];
  } else {
    bool bad = false;
    const uint32_t cmax = (1u << t.D) - 1u;
    key = (spread3(cell_of(x, t.prm.lo[0], t.prm.qscale[0], cmax, &bad)) << 2) |
          (spread3(cell_of(y, t.prm.lo[1], t.prm.qscale[1], cmax, &bad)) << 1) |
          spread3(cell_of(z, t.prm.lo[2], t.prm.qscale[2], cmax, &bad));
  }
  uint32_t node = t.root;
  double acc = 0.0;
  for (int d = 0;; ++d) {
    const double* geo = t.nt.geo + 6 * (size_t)node;
    acc += poly_eval<P, double>(t.nt.coef + (size_t)node * L, (x - geo[0]) * geo[3], (y - geo[1]) * geo[4],
                                (z - geo[2]) * geo[5]);
    if (d >= t.D) break;
    const uint32_t m = t.nt.child_mask[node];
    const uint32_t o = (key >> (3 * (t.D - d - 1))) & 7u;
    if (!((m >> o) & 1u)) break;
    node = t.nt.first_child[node] + (uint32_t)__popc(m & ((1u << o) - 1u));
  }
  out[perm ? perm[i] : i] = acc;
}

template <int P>
static hipError_t eval_impl(int dtype, const EvalTree& t, const void* qx, const void* qy, const void* qz,
                            const uint32_t* perm, const uint32_t* skeys, uint32_t nq, double* out, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  dim3 grid((nq + 255) / 256), block(256);
  if (dtype == FMT_F32)
    hipLaunchKernelGGL((k_eval<P, float>), grid, block, 0, s, t, (const float*)qx, (const float*)qy,
                       (const float*)qz, perm, skeys, nq, out);
  else
    hipLaunchKernelGGL((k_eval<P, double>), grid, block, 0, s, t, (const double*)qx, (const double*)qy,
                       (const double*)qz, perm, skeys, nq, out);
  return hipGetLastError();
}

hipError_t launch_eval(int p, int dtype, const EvalTree& t, const void* qx, const void* qy, const void* qz,
                       const uint32_t* perm, const uint32_t* skeys, uint32_t nq, double* out, hipStream_t s) {
  FMT_DISPATCH_P(p, eval_impl, dtype, t, qx, qy, qz, perm, skeys, nq, out, s);
}

}  // namespace fmt
