// K9: evaluation of a fitted tree at query points.
//
// Section 2 evaluates a fit as f'_q = Lambda'_q . F_p (no need to form the
// transform matrix).  The octree fit is a residual decomposition (Alg. 1), so
// the value at a query is the sum of the polynomials of every node on its
// root-to-leaf chain.  That sum is itself a polynomial of degree <= p in the
// frame of the deepest node reached, so it is formed once per node
// (k_compose) and a query then evaluates a single polynomial.
#include "k_level.h"

namespace fmt {

// ---------------------------------------------------------------------------
// Composite coefficients.  A child's frame relates to its parent's by
// u_parent = (u_child + sigma) / 2 on each axis (sigma = +1 for the upper
// half of the parent cell, -1 for the lower), so one scaled monomial
// re-expands as
//   u_p^l / l! = sum_{k <= l} (u_c^k / k!) sigma^(l-k) / (2^l (l-k)!),
// applied axis by axis.  Walking from the root along the node's prefix,
// C <- shift(C) + F_child at every level gives the node's composite.
// One wave per node, four nodes per workgroup; roots are stored first, one
// per problem, in problem order.
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_compose(NodeTable nt, uint32_t nodes, double* __restrict__ cc) {
  constexpr int L = basis_size(P);
  constexpr Basis<P> B{};
  __shared__ double buf[4][2][L];
  __shared__ int ex[L][3];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int i = tid; i < L; i += 256) {
    ex[i][0] = B.lx[i];
    ex[i][1] = B.ly[i];
    ex[i][2] = B.lz[i];
  }
  __syncthreads();
  const uint32_t v = blockIdx.x * 4 + (uint32_t)w;
  if (v >= nodes) return;   // the whole wave leaves; no workgroup barrier follows
  const int lv = (int)nt.level[v];
  const uint32_t pre = nt.prefix[v];
  uint32_t node = nt.problem[v];   // the root of v's problem
  double* cur = buf[w][0];
  double* nxt = buf[w][1];
  for (int e = lane; e < L; e += 64) cur[e] = nt.coef[(size_t)node * L + e];
  for (int d = 0; d < lv; ++d) {
    const uint32_t o = (pre >> (3 * (lv - d - 1))) & 7u;
    const uint32_t m = nt.child_mask[node];
    node = nt.first_child[node] + (uint32_t)__popc(m & ((1u << o) - 1u));
#pragma unroll
    for (int axis = 0; axis < 3; ++axis) {
      const double sg = ((o >> (2 - axis)) & 1u) ? 1.0 : -1.0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int e = lane; e < L; e += 64) {
        int xyz[3] = {ex[e][0], ex[e][1], ex[e][2]};
        const int k = xyz[axis];
        const int top = P - (xyz[0] + xyz[1] + xyz[2] - k);
        double sum = 0.0, t = ldexp(1.0, -k);
        for (int l = k; l <= top; ++l) {
          xyz[axis] = l;
          sum = fma(cur[graded(xyz[0], xyz[1], xyz[2])], t, sum);
          t *= sg / (2.0 * (double)(l + 1 - k));
        }
        nxt[e] = sum;
      }
      double* tmp = cur;
      cur = nxt;
      nxt = tmp;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int e = lane; e < L; e += 64) cur[e] += nt.coef[(size_t)node * L + e];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int e = lane; e < L; e += 64) cc[(size_t)v * L + e] = cur[e];
}

// ---------------------------------------------------------------------------
// One query per thread: walk down while the child holding the query's cell
// exists (integer loads only), then evaluate the composite polynomial of the
// node reached.  In sorted mode the coordinates arrive in key order (moved by
// the sort), skeys holds their keys and perm their positions in the caller's
// order, where the result is written.  A wave whose queries all reach one
// node reads that node's coefficients with wave-uniform (scalar) loads.
// ---------------------------------------------------------------------------
template <int P, typename TQ>
__global__ void __launch_bounds__(256) k_eval(EvalTree t, const double* __restrict__ cc,
                                              const double* __restrict__ geo, const TQ* __restrict__ qx,
                                              const TQ* __restrict__ qy, const TQ* __restrict__ qz,
                                              const uint32_t* __restrict__ perm, const uint32_t* __restrict__ skeys,
                                              uint32_t nq, double* __restrict__ out) {
  constexpr int L = basis_size(P);
  const uint32_t i0 = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i0 < nq;
  const uint32_t i = valid ? i0 : nq - 1;   // tail lanes repeat the last query and do not store
  const uint32_t src = perm ? perm[i] : i;   // caller's position of query i
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
  for (int d = 0; d < t.D; ++d) {
    const uint32_t m = t.nt.child_mask[node];
    const uint32_t o = (key >> (3 * (t.D - d - 1))) & 7u;
    if (!((m >> o) & 1u)) break;
    node = t.nt.first_child[node] + (uint32_t)__popc(m & ((1u << o) - 1u));
  }
  const uint32_t n0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)node);
  double val;
  if (__ballot(node != n0) == 0) {
    // read-only constant address space + a wave-uniform address: scalar loads
    typedef const double __attribute__((address_space(4))) cdouble;
    const cdouble* g = (const cdouble*)(geo + 6 * (size_t)n0);
    const cdouble* F = (const cdouble*)(cc + (size_t)n0 * L);
    val = poly_eval<P, double>(F, (x - g[0]) * g[3], (y - g[1]) * g[4], (z - g[2]) * g[5]);
  } else {
    const double* g = geo + 6 * (size_t)node;
    val = poly_eval<P, double>(cc + (size_t)node * L, (x - g[0]) * g[3], (y - g[1]) * g[4], (z - g[2]) * g[5]);
  }
  if (valid) out[src] = val;
}

template <int P>
static hipError_t compose_impl(const NodeTable& nt, uint32_t nodes, double* cc, hipStream_t s) {
  if (nodes == 0) return hipSuccess;
  hipLaunchKernelGGL(k_compose<P>, dim3((nodes + 3) / 4), dim3(256), 0, s, nt, nodes, cc);
  return hipGetLastError();
}

hipError_t launch_compose(int p, const NodeTable& nt, uint32_t nodes, double* cc, hipStream_t s) {
  FMT_DISPATCH_P(p, compose_impl, nt, nodes, cc, s);
}

template <int P>
static hipError_t eval_impl(int dtype, const EvalTree& t, const double* cc, const void* qx, const void* qy,
                            const void* qz, const uint32_t* perm, const uint32_t* skeys, uint32_t nq, double* out,
                            hipStream_t s) {
  if (nq == 0) return hipSuccess;
  dim3 grid((nq + 255) / 256), block(256);
  if (dtype == FMT_F32)
    hipLaunchKernelGGL((k_eval<P, float>), grid, block, 0, s, t, cc, (const double*)t.nt.geo, (const float*)qx,
                       (const float*)qy, (const float*)qz, perm, skeys, nq, out);
  else
    hipLaunchKernelGGL((k_eval<P, double>), grid, block, 0, s, t, cc, (const double*)t.nt.geo, (const double*)qx,
                       (const double*)qy, (const double*)qz, perm, skeys, nq, out);
  return hipGetLastError();
}

hipError_t launch_eval(int p, int dtype, const EvalTree& t, const double* cc, const void* qx, const void* qy,
                       const void* qz, const uint32_t* perm, const uint32_t* skeys, uint32_t nq, double* out,
                       hipStream_t s) {
  FMT_DISPATCH_P(p, eval_impl, dtype, t, cc, qx, qy, qz, perm, skeys, nq, out, s);
}

}  // namespace fmt
