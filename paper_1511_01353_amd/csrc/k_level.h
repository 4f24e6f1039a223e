// Per-level kernels of the octree fit (Alg. 1 / Alg. 2) and the evaluator.
#pragma once

#include "fmt_common.h"

namespace fmt {

// Everything a level kernel needs.  Work items are (node, chunk) pairs: node k
// of the level owns chunks [chunk_off[k], chunk_off[k+1]); chunk j of a node
// covers its sorted points [begin + j*CHUNK, min(begin + count, begin + (j+1)*CHUNK)).
struct LevelArgs {
  NodeTable nt;
  uint32_t node0;            // first node of the level in the table
  uint32_t nnodes;           // nodes in the level
  const uint32_t* chunk_off; // nnodes + 1 entries
  uint32_t nchunks;
  const void* px;            // key-sorted coordinates (input dtype)
  const void* py;
  const void* pz;
  double* r;                 // key-sorted residual
  const uint32_t* skey;      // key-sorted keys
  int level;                 // depth of this level
  int D;                     // maximum depth
  double tol;                // split tolerance
  int refine;                // 0: no refinement; 1: nodes whose conditioning needs it; 2: every node
};

struct EvalTree {
  NodeTable nt;
  uint32_t root;
  int D;               // deepest level holding a node (query keys use this depth)
  int T;               // depth of the cell table (T <= D)
  ProblemParams prm;   // qscale = 2^D / (hi - lo) for that D
  // per level d <= FMT_MAX_DEPTH: cell side h (3) then dilation 2 / h (3),
  // computed as the fit computes node frames (so the values agree bit for bit)
  const double* lvl;
  // cell c of depth T -> deepest node (level <= T) containing it, as
  // node | level << 28
  const uint32_t* cells;
};

// Doubles of the per-level frame table in front of a cell table.
constexpr int LVL_DOUBLES = 6 * (FMT_MAX_DEPTH + 1);

// Doubles of one chunk's partial Gram (upper-triangular 16x16 blocks of the
// augmented (L+1) x (L+1) matrix [Lambda | r]^T [Lambda | r]).
size_t gram_partial_doubles(int p);
// Doubles of one node's stored factor (packed lower Cholesky factor, pivots,
// equilibration scales).
size_t factor_doubles(int p);

// Sum each multi-chunk node's chunk partials (`width` doubles per chunk) into
// its first chunk slot.
hipError_t launch_chunk_reduce(const LevelArgs& a, double* buf, uint32_t width, hipStream_t s);
hipError_t launch_node_geo(const NodeTable& nt, const ProblemParams* prm, uint32_t n, hipStream_t s);
hipError_t launch_roots(const NodeTable& nt, const ProblemParams* prm, int nprob, hipStream_t s);
hipError_t launch_gram(int p, int path, int dtype, const LevelArgs& a, double* partial, hipStream_t s);
// Power moments of every chunk (mode 0: M, B, sum r^2; mode 1: B of r - Lambda F).
size_t moment_partial_doubles(int p);
size_t moment_refine_doubles(int p);
hipError_t launch_moments(int p, int mode, int dtype, const LevelArgs& a, double* part, hipStream_t s);
hipError_t launch_solve(int p, const LevelArgs& a, const double* partial, double* fac, hipStream_t s);
// K6 assembled from power moments (the k_moments mode-0 layout).
hipError_t launch_solve_moments(int p, const LevelArgs& a, const double* part, double* fac, hipStream_t s);
hipError_t launch_refine_solve(int p, const LevelArgs& a, const double* part_b, const double* fac, hipStream_t s);
hipError_t launch_residual(int p, int dtype, const LevelArgs& a, double* part_ss, hipStream_t s);
hipError_t launch_children(int p, const LevelArgs& a, const double* part_ss, uint32_t* cbeg, uint32_t* ccnt,
                           uint32_t* nact, hipStream_t s);
// counters[0..2] = next level's nodes, chunks, points; with hostc (device view
// of host-visible memory) they are also written there, followed by seq at
// hostc[3] (system-scope release).
hipError_t launch_emit(const LevelArgs& a, const ProblemParams* prm, const uint32_t* cbeg, const uint32_t* ccnt,
                       uint32_t* nact, uint32_t next0, uint32_t* next_chunk_off, uint32_t* counters, uint32_t* hostc,
                       uint32_t seq, hipStream_t s);
hipError_t launch_check_coef(int p, const NodeTable& nt, uint32_t nnodes, uint32_t* status, hipStream_t s);
// Composite coefficients of every node (its chain's polynomials in its frame).
hipError_t launch_compose(int p, const NodeTable& nt, uint32_t nodes, double* cc, hipStream_t s);
// Cell table of one tree: 8^T entries, see EvalTree::cells.
// Also writes the frame table lvl (LVL_DOUBLES) of the tree's problem.
hipError_t launch_cell_table(const NodeTable& nt, uint32_t root, int T, const ProblemParams& prm, double* lvl,
                             uint32_t* cells, hipStream_t s);
// perm/skeys: sorted mode (query order and sorted keys), else both null.
hipError_t launch_eval(int p, int dtype, const EvalTree& t, const double* cc, const void* qx, const void* qy,
                       const void* qz, const uint32_t* perm, const uint32_t* skeys, uint32_t nq, double* out,
                       hipStream_t s);

// Device helpers shared by the level kernels ---------------------------------

// Node k of a level owning chunk g: chunk_off[k] <= g < chunk_off[k+1].
__device__ __forceinline__ uint32_t chunk_node(const uint32_t* chunk_off, uint32_t nnodes, uint32_t g) {
  uint32_t lo = 0, hi = nnodes - 1;
  while (lo < hi) {
    uint32_t mid = (lo + hi + 1) >> 1;
    if (chunk_off[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ void load_point(const void* px, const void* py, const void* pz, uint32_t i, double& x,
                                           double& y, double& z) {
  x = (double)((const T*)px)[i];
  y = (double)((const T*)py)[i];
  z = (double)((const T*)pz)[i];
}

}  // namespace fmt

// Instantiate F<P> for the runtime order p (0..FMT_MAX_P).
#define FMT_DISPATCH_P(p, F, ...)                  \
  switch (p) {                                      \
    case 0: return F<0>(__VA_ARGS__);               \
    case 1: return F<1>(__VA_ARGS__);               \
    case 2: return F<2>(__VA_ARGS__);               \
    case 3: return F<3>(__VA_ARGS__);               \
    case 4: return F<4>(__VA_ARGS__);               \
    case 5: return F<5>(__VA_ARGS__);               \
    case 6: return F<6>(__VA_ARGS__);               \
    case 7: return F<7>(__VA_ARGS__);               \
    case 8: return F<8>(__VA_ARGS__);               \
    default: return hipErrorInvalidValue;           \
  }
