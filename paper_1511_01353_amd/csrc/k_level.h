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
  // moment pyramid table (PyrTab::tab: PYR_TAB_WORDS per problem), null
  // when no problem has one.  Nodes at levels d <= kp take M from the
  // pyramid (pyramid_covers)
  const uint32_t* pyr_tab;
  // several right-hand sides in one launch (the fixed-topology refit): grid
  // index y = j selects the residual r + j rstride, the coefficients
  // nt.coef + j cstride and the field's own block of chunk partials (nchunks
  // chunks per field); nfields <= 1 is one field
  uint32_t nfields = 1;
  uint64_t rstride = 0, cstride = 0;
  // factors made ahead of the level loop for the pyramid's upper levels
  // (k_factor_cells) and their flags; the pyramid table's word 3 holds, per
  // problem, the first slot (low 28 bits) and the number of levels covered
  // (high 4 bits).  Null when none were made.
  const double* fac_up = nullptr;
  const uint32_t* up_flags = nullptr;
  // status word: the solves mark nodes whose coefficients are not all finite
  // (FLAG_NONFINITE) and set bit 2 here; null: no check
  uint32_t* status = nullptr;
  // nonzero: the Gram partials are float32 sums (the mixed path); k_solve
  // flags FLAG_REGRAM on nodes whose condition estimate exceeds REGRAM_KAPPA
  // or that deflate a pivot, and leaves their coefficients to the float64
  // re-solve
  uint32_t regram = 0;
  // nonzero: k_moments (mode 0), k_chunk_reduce, the moment solves and k_residual
  // take only the nodes whose flags hold one of these bits (the float64
  // re-solve; the refinement's correction pass)
  uint32_t only_flag = 0;
  // refinement after the residual update: the sweep (mode 1) takes the
  // residual as it stands (r already holds r - Lambda F) instead of
  // subtracting Lambda F itself, and the refinement solve also writes its
  // correction delta (calL per level node, at delta + k calL) so that a
  // residual pass can subtract Lambda delta
  uint32_t sweep_current = 0;
  double* delta = nullptr;
  // level-local indices of the nodes that span more than one chunk (the
  // topology kernel lists them for the next level), nmulti of them; null:
  // not listed, the chunk reduction looks at every node
  const uint32_t* multi = nullptr;
  uint32_t nmulti = 0;
  // non-null: the launch covers only the listed nodes of the level (the
  // late refinement's passes over the nodes flagged for it, as the topology
  // kernel lists them): level-local indices sel[0 .. nsel), ascending, and
  // sel_off[j] the first work item of node sel[j] (its chunks in order;
  // sel_off[nsel] = nsel_chunks).  Chunk-wide launches then have
  // nsel_chunks workgroups, node-wide ones nsel.
  const uint32_t* sel = nullptr;
  const uint32_t* sel_off = nullptr;
  uint32_t nsel = 0, nsel_chunks = 0;
  // the level's nodes with fewer than SMALL_NODE points (UINT32_MAX: not
  // counted); the moment launches skip a size class the level lacks
  uint32_t nsmall = UINT32_MAX;
};

// Nodes with fewer points than this take the r-weighted moments in mode 4
// (unstaged, two waves per chunk), the others in mode 2; the choice depends
// on the node alone, so a problem gets the same bits in any batch.
constexpr uint32_t SMALL_NODE = 1024;

// Grid rows of a launch over the fields of a LevelArgs.
inline unsigned field_rows(const LevelArgs& a) { return a.nfields > 1 ? a.nfields : 1u; }

// Moment pyramid tables (k_pyramid.hip).  The per-problem words: first
// pyramid entry, depth kp (0: none), first flat finest cell, and the factors
// made ahead of the level loop (first slot | levels << 28; 0: none).
constexpr int PYR_TAB_WORDS = 4;
struct PyrTab {
  const uint32_t* tab;      // PYR_TAB_WORDS per problem
  const uint32_t* cstart;   // nbase + 1: first flat finest cell of each pyramid
  const uint32_t* bq;       // nbase: problem of each pyramid
  uint32_t nbase;           // problems with a pyramid
};

// Entries of levels 0 .. d-1 of one pyramid: (8^d - 1) / 7.
__host__ __device__ __forceinline__ uint32_t level_first(int d) { return ((1u << (3 * d)) - 1u) / 7u; }

// Whether level `level` of a problem with pyramid depth kp reads M from it.
__host__ __device__ __forceinline__ bool pyramid_covers(uint32_t kp, int level) {
  return kp > 0 && (uint32_t)level <= kp;
}

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
// its first chunk slot (per field: a.nchunks * width doubles each).
hipError_t launch_chunk_reduce(const LevelArgs& a, double* buf, uint32_t width, hipStream_t s);
hipError_t launch_node_geo(const NodeTable& nt, const ProblemParams* prm, uint32_t n, hipStream_t s);
hipError_t launch_roots(const NodeTable& nt, const ProblemParams* prm, int nprob, hipStream_t s);
hipError_t launch_gram(int p, int path, int dtype, const LevelArgs& a, double* partial, hipStream_t s);
// Power moments of every chunk (mode 0: M, B, sum r^2 (for p <= 4 in two
// launches by node size); mode 1: B of r - Lambda F; mode 2: B of the nodes
// with at least SMALL_NODE points; mode 3: M; mode 4: B as mode 2, unstaged,
// of the smaller nodes).  The grid is a.nchunks workgroups,
// which may exceed chunk_off[nnodes] (the extra ones exit).  With
// a.pyr_tab, mode 2 skips the nodes the pyramid does not cover and mode 0
// those it covers.
size_t moment_partial_doubles(int p);   // mode 0
size_t moment_refine_doubles(int p);    // modes 1 and 2
size_t moment_base_doubles(int p);      // mode 3
hipError_t launch_moments(int p, int mode, int dtype, const LevelArgs& a, double* part, hipStream_t s);
hipError_t launch_solve(int p, const LevelArgs& a, const double* partial, double* fac, hipStream_t s);
// K6 assembled from power moments: M and B from the mode-0 partials part_m,
// or, for nodes the pyramid covers (a.pyr_tab), M from the pyramid and B from
// the mode-2 partials part_b.
hipError_t launch_solve_moments(int p, const LevelArgs& a, const double* part_m, const double* part_b,
                                const double* pyr, double* fac, hipStream_t s);
// The same solve with the matrix in one wave's registers (k_solve_reg.hip),
// for the orders solve_reg_order accepts (p <= 6); launch_solve_moments
// takes it for those orders.
bool solve_reg_order(int p);
hipError_t launch_solve_reg(int p, const LevelArgs& a, const double* part_m, const double* part_b, const double* pyr,
                            double* fac, hipStream_t s);
// Moment pyramid (k_pyramid.hip): moment_base_doubles(p) doubles per entry.
// The finest cells of all pyramids (flat numbering): point range, frame (6
// doubles), chunk count and pyramid entry.  begin and count must hold zeros
// on entry (empty cells are never written by the boundary pass).
hipError_t launch_pyr_cells(const uint32_t* skey, uint32_t n, int D, int nprob, const ProblemParams* prm,
                            const PyrTab& pt, uint32_t ncell, uint32_t* begin, uint32_t* count, double* geo,
                            uint32_t* nchk, uint32_t* dst, hipStream_t s);
// off[0..ncell] = exclusive scan of nchk (one workgroup).
hipError_t launch_pyr_scan(const uint32_t* nchk, uint32_t ncell, uint32_t* off, hipStream_t s);
// Sum each flat cell's chunk partials (width doubles each) into pyramid
// entry dst[cell] (zeros if it has none).
hipError_t launch_pyr_base(const uint32_t* off, uint32_t ncell, const double* part, uint32_t width,
                           const uint32_t* dst, double* pyr, hipStream_t s);
// Level d of the nlist pyramids list[0..nlist) (problems with kp > d) from
// level d+1.
hipError_t launch_pyr_up(int p, double* pyr, const uint32_t* tab, const uint32_t* list, uint32_t nlist, int d,
                         hipStream_t s);
hipError_t launch_refine_solve(int p, const LevelArgs& a, const double* part_b, const double* fac, hipStream_t s);
// Factor only: the equilibrated normal equations of every node from the
// mode-3 partials (chunks summed beforehand), factored into fac
// (factor_doubles(p) per node of the level), with the condition estimate
// (a.refine == 1) and the rank flags.  No coefficients are written.
hipError_t launch_factor_moments(int p, const LevelArgs& a, const double* part_m, double* fac, hipStream_t s);
// The solve of the nodes whose factor was made ahead (a.fac_up; other nodes
// are left to launch_solve_moments, which skips these).
hipError_t launch_solve_ahead(int p, const LevelArgs& a, const double* part_b, double* fac, hipStream_t s);
// Factors of n pyramid entries list[0..n) (M from the pyramid), made before
// the level loop: slot g gets the factor of entry list[g] (factor_doubles(p)
// doubles) and the flags of its condition estimate and deflation (up_flags
// must hold zeros on entry).  refine as LevelArgs::refine.
hipError_t launch_factor_cells(int p, const double* pyr, const uint32_t* list, uint32_t n, int refine,
                               double* fac_up, uint32_t* up_flags, hipStream_t s);
// F = G^-1 Lambda^T r on every node from the mode-2 partials (chunks summed
// beforehand) and the factors of launch_factor_moments.
hipError_t launch_factor_solve(int p, const LevelArgs& a, const double* part_b, const double* fac, hipStream_t s);
hipError_t launch_residual(int p, int dtype, const LevelArgs& a, double* part_ss, hipStream_t s);
// r <- r - Lambda F for every field of a multi-field LevelArgs (one launch,
// the points read once per group of fields), without octant statistics.
hipError_t launch_residual_fields(int p, int dtype, const LevelArgs& a, hipStream_t s);
hipError_t launch_children(int p, const LevelArgs& a, const double* part_ss, uint32_t* cbeg, uint32_t* ccnt,
                           uint32_t* nact, hipStream_t s);
// counters[0..2] = next level's nodes, chunks, points, counters[4] = its
// nodes with fewer than SMALL_NODE points, counters[5] = this level's nodes
// flagged for refinement (FLAG_REFINE), counters[6] = next level's nodes
// that span more than one chunk, whose level-local indices go to next_multi
// (room for 8 nnodes entries; in no fixed order), counters[7] = the chunks
// of this level's flagged nodes; those nodes go to sel (level-local
// indices, ascending) and their first chunk numbers among them to
// sel + nnodes + 1 (LevelArgs::sel, sel_off; room for 2 nnodes + 2
// entries).  With hostc (device view of host-visible memory) the counters
// are also written there (same positions), and the sequence number at
// hostc[3] last (system-scope release), once the launch has written
// everything else.  Large levels take the tiled launches, whose scratch is
// tiles (emit_tile_words(a.nnodes) words; may be null when that is 0) and
// counters[8].
hipError_t launch_emit(const LevelArgs& a, const ProblemParams* prm, const uint32_t* cbeg, const uint32_t* ccnt,
                       uint32_t* nact, uint32_t next0, uint32_t* next_chunk_off, uint32_t* counters, uint32_t* hostc,
                       uint32_t seq, uint32_t* next_multi, uint32_t* sel, uint32_t* tiles, hipStream_t s);
size_t emit_tile_words(uint32_t nnodes);
hipError_t launch_check_coef(int p, const NodeTable& nt, uint32_t nnodes, uint32_t* status, hipStream_t s);
// Row stride (doubles) of the composite coefficient table: calL rounded up to
// even, so that every row starts on a 16-byte boundary.
// Composite coefficient rows start on 128-byte boundaries (one L2 line), so
// a row of calL = 84 doubles occupies exactly six lines.
__host__ __device__ constexpr int ccoef_stride(int L) { return (L + 15) / 16 * 16; }
// Composite coefficients (a node's chain of polynomials in its frame),
// ccoef_stride(calL) doubles per node (the tail of a row is zero), of the
// nodes first .. first+count-1 of any levels (each wave walks its node's
// chain; no row depends on another).
hipError_t launch_compose(int p, const NodeTable& nt, uint32_t first, uint32_t count, double* cc, hipStream_t s);
// Cell table of one tree: 8^T entries, see EvalTree::cells.
// Also writes the frame table lvl (LVL_DOUBLES) of the tree's problem.
hipError_t launch_cell_table(const NodeTable& nt, uint32_t root, int T, const ProblemParams& prm, double* lvl,
                             uint32_t* cells, hipStream_t s);
// perm/skeys: sorted mode (query order and sorted keys), else both null.
hipError_t launch_eval(int p, int dtype, const EvalTree& t, const double* cc, const void* qx, const void* qy,
                       const void* qz, const uint32_t* perm, const uint32_t* skeys, uint32_t nq, double* out,
                       hipStream_t s);

// Large bases (k_wide.hip): orders p = 10, 12, 14 (calL = 286, 455, 680),
// whose normal equations do not fit a workgroup's LDS.  Per node of the level
// a factor of wide_factor_doubles(p) doubles in device memory (fac + k *
// that for level node k): the equilibrated matrix assembled from the node's
// mode-0 partial (chunks summed beforehand) and factored by a blocked
// Cholesky; then the solve writes F (with the condition estimate when
// a.refine == 1, and the rank flags), and the refinement solve adds the
// correction from the node's mode-1 partial (chunks summed beforehand).
bool wide_order(int p);
size_t wide_factor_doubles(int p);
hipError_t launch_wide_factor(int p, const LevelArgs& a, const double* part_m, double* fac, hipStream_t s);
hipError_t launch_wide_solve(int p, const LevelArgs& a, const double* part_m, const double* fac, hipStream_t s);
hipError_t launch_wide_refine_solve(int p, const LevelArgs& a, const double* part_b, const double* fac,
                                    hipStream_t s);
// Gaussian-RBF factorisation (k_rbf.hip).  Basis values of n points of
// dtype, row-major with stride LS (a multiple of 32): A[j LS + k] =
// Lambda_k(x_j) for k < L, zero beyond; expo holds the packed exponents
// (l | m << 8 | n << 16) of the L basis indices.
hipError_t launch_rbf_basis(int dtype, const void* x, const void* y, const void* z, uint32_t n, const uint32_t* expo,
                            int L, uint32_t LS, double* A, hipStream_t s);
// out[q * ostride + i] = sum_{k < LS} A[q LS + k] R[i LS + k] for q < nq
// (< 2^23), i < nr, on float64 MFMA.
hipError_t launch_rbf_gemm(const double* A, uint32_t nq, const double* R, uint32_t nr, uint32_t LS, double* out,
                           uint64_t ostride, hipStream_t s);
// The moment kernels (modes 0 and 1 only) of the large orders, each compiled
// in a translation unit of its own (k_moments.hip built with
// FMT_MOMENTS_WIDE_P defined); launch_moments dispatches to them.
hipError_t launch_moments_p10(int mode, int dtype, const LevelArgs& a, double* part, hipStream_t s);
hipError_t launch_moments_p12(int mode, int dtype, const LevelArgs& a, double* part, hipStream_t s);
hipError_t launch_moments_p14(int mode, int dtype, const LevelArgs& a, double* part, hipStream_t s);

// Device helpers shared by the level kernels ---------------------------------

// Node k of a level owning chunk g: the last k with chunk_off[k] <= g, so
// chunk_off[k] <= g < chunk_off[k+1] (nodes without chunks are skipped).
// The whole wave searches together (g must be wave-uniform and every lane
// active): each round its 64 lanes probe evenly spaced offsets of the
// remaining range and a ballot narrows the range 64-fold, so 4096 nodes take
// two rounds of loads instead of twelve.
__device__ __forceinline__ uint32_t chunk_node(const uint32_t* chunk_off, uint32_t nnodes, uint32_t g) {
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t lo = 0, hi = nnodes;   // the answer lies in [lo, hi); chunk_off[lo] <= g
  while (hi - lo > 1) {
    const uint32_t step = (hi - lo + 63) / 64;
    const uint32_t idx = lo + lane * step;
    // probes at or below g form a prefix of the lanes (offsets ascend)
    const uint32_t c = (uint32_t)__popcll(__ballot(idx < hi && chunk_off[idx] <= g));
    lo += (c - 1) * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

// Work item w of a launch over the listed nodes' chunks (LevelArgs::sel):
// the node k (level-local) and its chunk g among the level's chunks.
// False past the last listed chunk.
__device__ __forceinline__ bool listed_chunk(const LevelArgs& a, uint32_t w, uint32_t& k, uint32_t& g) {
  if (w >= a.nsel_chunks) return false;
  const uint32_t j = chunk_node(a.sel_off, a.nsel, w);
  k = a.sel[j];
  g = a.chunk_off[k] + (w - a.sel_off[j]);
  return true;
}

// Cell coordinates (i, j, k) of a Morton prefix with `level` triples.
__device__ __forceinline__ void decode_cell(uint32_t prefix, int level, uint32_t& ci, uint32_t& cj, uint32_t& ck) {
  ci = cj = ck = 0;
  for (int b = level - 1; b >= 0; --b) {
    const uint32_t t = (prefix >> (3 * b)) & 7u;
    ci = (ci << 1) | ((t >> 2) & 1u);
    cj = (cj << 1) | ((t >> 1) & 1u);
    ck = (ck << 1) | (t & 1u);
  }
}

// Centre and dilation of a node: h = (hi - lo) / 2^level, c = lo + (i + 1/2) h,
// u = (x - c) * (2 / h).  Separate roundings, no fused multiply-add.
__device__ __forceinline__ void node_geo(const ProblemParams& P, int level, uint32_t prefix, double* geo) {
  uint32_t c[3];
  decode_cell(prefix, level, c[0], c[1], c[2]);
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const double h = ldexp(__dsub_rn(P.hi[ax], P.lo[ax]), -level);
    geo[ax] = __dadd_rn(P.lo[ax], __dmul_rn((double)c[ax] + 0.5, h));
    geo[3 + ax] = __ddiv_rn(2.0, h);
  }
}

// Copy N doubles (N a compile-time count) from global memory to LDS with
// NT threads: every thread issues all of its loads before its first store,
// so the copy costs one memory latency rather than one per round.
template <int NT, int N>
__device__ __forceinline__ void copy_to_lds(double* __restrict__ dst, const double* __restrict__ src, int tid) {
  constexpr int R = (N + NT - 1) / NT;
  double v[R > 0 ? R : 1];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int e = tid + q * NT;
    v[q] = e < N ? src[e] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int e = tid + q * NT;
    if (e < N) dst[e] = v[q];
  }
}

template <typename T>
__device__ __forceinline__ void load_point(const void* px, const void* py, const void* pz, uint32_t i, double& x,
                                           double& y, double& z) {
  x = (double)((const T*)px)[i];
  y = (double)((const T*)py)[i];
  z = (double)((const T*)pz)[i];
}

}  // namespace fmt

// Instantiate F<P> for the runtime order p of the small bases (0..8).
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

// Instantiate F<P> for every supported order: the small bases 0..8 and the
// large ones 10, 12, 14 (kernels whose work per point or node is a loop over
// the basis, not a factorisation held in LDS).
#define FMT_DISPATCH_P_ALL(p, F, ...)              \
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
    case 10: return F<10>(__VA_ARGS__);             \
    case 12: return F<12>(__VA_ARGS__);             \
    case 14: return F<14>(__VA_ARGS__);             \
    default: return hipErrorInvalidValue;           \
  }
