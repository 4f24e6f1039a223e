/*
 * fmt.h -- C ABI of the free-mesh transform (FMT) library for MI355X (gfx950).
 *
 * The library fits a scattered-data interpolant by top-down octree scoping of
 * the residual and evaluates it at new points (Challacombe, "A N-Body Solver
 * for Free Mesh Interpolation", arXiv:1511.01353):
 *
 *   fit  : Alg. 1 (recursive octree decomposition of the residual) with
 *          Alg. 2 (least-squares moments of one node) at every node;
 *   eval : the practical transform f'_q = Lambda'_q . F_p of Section 2, summed
 *          over the root-to-leaf chain of nodes that hold the query.
 *
 * Conventions shared by every call:
 *   - Points live in a box [box_lo, box_hi] (default the unit cube).  The
 *     root node is the box; a node of depth d has side h = (hi - lo) / 2^d per
 *     axis.  Cells at the finest depth D are
 *       q = clamp(floor((x - lo) * (2^D / (hi - lo))), 0, 2^D - 1)
 *     evaluated in float64; a point on a split plane belongs to the upper
 *     child, a point at x = hi to the last cell.  Keys interleave the cell bits
 *     from the top level down, x highest in each triple.
 *   - Basis: all monomials of total degree <= p in graded order (degree 0;
 *     then x, y, z; then the six of degree 2 with the x exponent descending,
 *     then y descending; ...), Lambda_{lmn}(u) = u^l v^m w^n / (l! m! n!) in
 *     the node frame u = (x - c) * (2 / h) (Section 2, geometric moments;
 *     calL = (p+1)(p+2)(p+3)/6 basis functions).
 *   - A child octant is fitted iff its depth is <= max_depth, it holds at
 *     least calL points, and its RMS residual after the parent's fit exceeds
 *     tol (strict), as Alg. 1 tests it.  The root is always fitted.
 *   - Device pointers are HIP device addresses; host pointers are ordinary
 *     host memory.  Every call says which it takes.  `stream` is a
 *     hipStream_t passed as void* (NULL = the null stream).
 *   - Calls return fmt_status; on failure fmt_last_error() (thread-local)
 *     holds a message.  No C++ exception crosses this boundary.
 *   - The library never keeps a caller's pointer after a call returns; the
 *     caller keeps inputs valid until the stream has passed the call's work.
 */
#ifndef FMT_H
#define FMT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMT_MAX_P 14         /* largest supported total degree (calL = 680); the
                                supported orders are 0..8, 10, 12 and 14 */
#define FMT_MAX_DEPTH 10     /* deepest supported level; keys use 3*D bits */
#define FMT_MAX_LEVELS (FMT_MAX_DEPTH + 1)
#define FMT_REFIT_MAX_FIELDS 4096   /* value fields one fmt_refit call takes */

typedef enum {
  FMT_OK = 0,
  FMT_E_INVALID_ARG = 1,     /* bad option, size, dtype or NULL pointer */
  FMT_E_DOMAIN = 2,          /* a point is NaN/inf or outside [box_lo, box_hi] */
  FMT_E_UNDERDETERMINED = 3, /* the root holds fewer than calL points */
  FMT_E_OOM = 4,             /* device allocation failed; nothing leaked */
  FMT_E_NUMERIC = 5,         /* a non-finite coefficient was produced */
  FMT_E_DEVICE = 6,          /* a HIP runtime call failed */
  FMT_E_BUSY = 7             /* reserved for callers that admit work by budget */
} fmt_status;

typedef enum { FMT_F32 = 0, FMT_F64 = 1 } fmt_dtype;

typedef enum {
  /* every step in float64: normal equations (power moments on the vector
     ALUs, or the Gram on float64 MFMA), Cholesky, refinement */
  FMT_PATH_FP64 = 0,
  /* Gram of the monomials on float32 MFMA (float32 accumulation within a
     chunk of points, chunks summed in float64); float64 Cholesky; float64
     refinement sweeps (residual, Lambda^T r) recover float64 accuracy.
     Nodes whose float32 Gram is too ill-conditioned for that (estimated
     condition number above 1e6, or a deflated pivot) are solved again from
     float64 power moments */
  FMT_PATH_MIXED = 1
} fmt_path;

typedef enum {
  /* power moments M_gamma = sum u^gamma (|gamma| <= 2p) accumulated on the
     float64 vector ALUs; Gram entries are M_{alpha+beta} / (alpha! beta!).
     M does not depend on the residual: for the top levels of the tree it is
     accumulated once over the cells of one level (the deepest whose cells
     hold calL points on average, at most 5) and carried to the coarser
     levels by an exact change of frame (the moment pyramid); each of those
     levels then accumulates only the r-weighted moments B_alpha */
  FMT_GRAM_MOMENTS = 0,
  /* the Gram [Lambda|r]^T [Lambda|r] formed on float64 MFMA */
  FMT_GRAM_MFMA = 1,
  /* power moments as FMT_GRAM_MOMENTS, but M and B accumulated from the
     points at every level (no pyramid) */
  FMT_GRAM_MOMENTS_LEVEL = 2
} fmt_gram;

typedef struct {
  int p;               /* maximum total degree: 0..8, 10, 12 or 14.  The
                          large orders (calL = 286, 455, 680) take the float64
                          path with per-level power moments and a tiled
                          solve in device memory; they have no mixed path,
                          MFMA Gram or fixed-topology refit */
  double tol;          /* tau: split tolerance on the octant RMS residual, >= 0 */
  int max_depth;       /* D, 0..FMT_MAX_DEPTH; the root is depth 0 */
  int path;            /* fmt_path */
  int refine_steps;    /* iterative-refinement sweeps, 0..8: a sweep
                          recomputes the residual from the points and
                          corrects the coefficients with the kept factor.
                          The mixed path applies them to every node; the
                          float64 path only to nodes whose equilibrated
                          normal equations have an estimated condition
                          number above 1e6 or a deflated pivot (elsewhere
                          the float64 solve is already accurate). */
  double box_lo[3];    /* root box; default 0 */
  double box_hi[3];    /* default 1; box_hi > box_lo on every axis */
  int gram;            /* fmt_gram: how the float64 path forms the normal
                          equations (the mixed path always uses MFMA) */
} fmt_fit_opts;

typedef struct fmt_tree fmt_tree;   /* opaque; its storage lives in device memory */

typedef struct {
  int64_t nodes;                          /* nodes in this tree */
  int64_t n_points;                       /* points it was fitted on (0 if imported) */
  int32_t depth;                          /* deepest level present */
  int32_t p;                              /* total degree */
  int32_t L;                              /* calL */
  int32_t max_depth;                      /* D */
  int32_t path;                           /* fmt_path */
  int32_t rank_deficient_nodes;           /* nodes where a Cholesky pivot was deflated */
  int64_t per_level[FMT_MAX_LEVELS];      /* nodes at each depth */
  int64_t device_bytes;                   /* device memory held by the tree's forest */
} fmt_tree_info;

/* Fill `opts` with the defaults: p = 4, tol = 1e-8, max_depth = 6,
   path = FMT_PATH_FP64, refine_steps = 1, box = [0,1]^3,
   gram = FMT_GRAM_MOMENTS. */
void fmt_default_opts(fmt_fit_opts* opts);

/*
 * Fit one problem (Alg. 1 at the root, Alg. 2 at every node).
 *   x, y, z, f : device arrays of n values of `dtype` (SoA coordinates and the
 *                sampled function).  f is not modified.
 *   n          : number of points, calL <= n < 2^31.
 *   out        : receives a new tree; release it with fmt_tree_destroy.
 * The call validates options synchronously, then runs the fit on `stream`;
 * it returns after the tree is complete (the host reads small per-level
 * counts).  Errors: INVALID_ARG, UNDERDETERMINED (n < calL), DOMAIN, OOM,
 * NUMERIC, DEVICE.  On error *out is NULL.
 */
fmt_status fmt_fit(const fmt_fit_opts* opts, const void* x, const void* y, const void* z,
                   const void* f, int64_t n, int dtype, void* stream, fmt_tree** out);

/*
 * Fit `count` independent problems in one pass: one sort of composite keys
 * (problem id above the Morton bits) and one launch per level and kernel that
 * covers every problem's nodes at that level.
 *   opts       : host array of `count` options.  Problems may differ in p,
 *                path and box; they are grouped by (p, path, max_depth,
 *                refine_steps) and each group runs as one batched pass.
 *   x,y,z,f    : host arrays of `count` device pointers.
 *   n          : host array of `count` sizes (each >= its calL).
 *   out        : host array of `count` tree handles, filled on success.
 * Trees of one group share device storage; each handle keeps it alive.
 * Errors as fmt_fit; on error no handle is returned.
 */
fmt_status fmt_fit_batch(const fmt_fit_opts* opts, const void* const* x, const void* const* y,
                         const void* const* z, const void* const* f, const int64_t* n,
                         int count, int dtype, void* stream, fmt_tree** out);

/*
 * Evaluate a tree at nq query points (Section 2, f'_q = Lambda'_q F_p, summed
 * over the existing root-to-leaf chain).
 *   qx,qy,qz   : device arrays of nq values of `dtype`.
 *   out        : device array of nq float64 results.
 *   sort_queries: 0 = evaluate in input order; 1 = sort queries by key first
 *                (coherent coefficient reads; results still in input order);
 *                -1 = let the library choose.
 * Queries outside the box follow the clamped cell path; their polynomials
 * are evaluated at the true coordinates.  Asynchronous on `stream`.
 * Errors: INVALID_ARG, OOM, DEVICE.
 */
fmt_status fmt_eval(const fmt_tree* tree, const void* qx, const void* qy, const void* qz,
                    int64_t nq, int dtype, double* out, int sort_queries, void* stream);

/*
 * fmt_eval for callers that cannot allocate device memory: code recorded
 * under HIP graph capture, tight serving loops, and harnesses that forbid
 * allocation.  Arguments, results and errors are those of fmt_eval; the
 * differences:
 *   - The sorted mode takes its scratch (query keys, positions, sorted
 *     coordinates, sort histograms) from one static device array of
 *     FMT_EVAL_NOALLOC_SCRATCH_BYTES per GPU, held from the first call on that
 *     GPU until the process ends; no call allocates or frees memory.  The
 *     sorted mode of nq queries needs 6 * round256(nq * sizeof(coordinate))
 *     + 16 nq + about 4 nq / 16 bytes: every nq <= 2^20 fits for either
 *     dtype; a larger nq in sorted mode fails with INVALID_ARG (evaluate in
 *     pieces, or unsorted, which needs no scratch).
 *   - The tree's evaluation tables (composite coefficients, cell table) are
 *     built by the first fmt_eval of the tree; before that this call fails
 *     with INVALID_ARG.
 *   - Calls that overlap in time on one GPU share the array and race: the
 *     caller serialises them (one stream, or events).  Nothing in the array
 *     needs to start at zero; every call writes what it reads.
 *   - The call enqueues kernels only (no allocation, copy or memset), so it
 *     can be recorded into a HIP graph and replayed; a replay evaluates the
 *     query arrays captured, at their current contents.
 */
#define FMT_EVAL_NOALLOC_SCRATCH_BYTES (72u << 20)
fmt_status fmt_eval_noalloc(const fmt_tree* tree, const void* qx, const void* qy, const void* qz,
                            int64_t nq, int dtype, double* out, int sort_queries, void* stream);

/*
 * Gaussian-RBF factorisation (Section 2, eq. fullyfactored): the Gaussian
 * kernel exp(-eps^2 |x_q - x_i|^2) expanded in Taylor series and truncated
 * to the calL monomials of degree <= p on each side,
 *   out[q n + i] = sum_{a,b} Lambda_a(x_q) eps^|a| T_ab eps^|b| Lambda_b(x_i),
 *   T_ab = (-1)^|a| H_{a1+b1}(0) H_{a2+b2}(0) H_{a3+b3}(0),
 * with Lambda_a(x) = x^a / a! in the points' own coordinates (no frame) and
 * H_m(0) the physicists' Hermite numbers, the values at zero of the Hermite
 * functions exp(-t^2) H_m(t) the section defines.  A check of the theory
 * behind the method, off the fit / eval path.
 *   p          : 0..14 (every order).
 *   eps        : shape parameter, finite, >= 0.
 *   x, y, z    : device arrays of n points (dtype); 0 <= n < 2^31.
 *   xq, yq, zq : device arrays of nq query points (dtype); 0 <= nq < 2^22.
 *   out        : device array of nq * n float64, row q for query q.
 * Asynchronous on `stream` (scratch from the stream-ordered allocator).
 * Errors: INVALID_ARG, OOM, DEVICE.
 */
fmt_status fmt_rbf_factored(int p, double eps, const void* x, const void* y, const void* z, int64_t n,
                            const void* xq, const void* yq, const void* zq, int64_t nq, int dtype, double* out,
                            void* stream);

/* Wait for all work of the tree's forest and report device-side status
   (DOMAIN for points outside the box, NUMERIC for non-finite coefficients).
   The tree is the octree record P that Alg. 1 builds (per node its centre
   P_C, scale P_Scale and coefficients P_F, created by FMT_New_Octant). */
fmt_status fmt_tree_wait(const fmt_tree* tree);

/* Host-side summary of a tree (Alg. 1's node records P, counted per level). */
fmt_status fmt_tree_get_info(const fmt_tree* tree, fmt_tree_info* info);

/*
 * Copy the tree's nodes to host buffers (any pointer may be NULL): Alg. 1's
 * node records P, with the coefficients P_F that Alg. 2 writes.  Nodes are
 * in (level, prefix) order; each buffer holds info.nodes entries (coeffs:
 * info.nodes * info.L float64 in graded order, the Lambda basis).
 *   prefix : the node's key prefix (Morton bits of its cell, 3*level bits)
 *   begin  : first position of its points in the key-sorted point order
 *   count  : its point count
 *   flags  : bit 0 set if a Cholesky pivot was deflated (the node's points
 *            do not determine every basis coefficient: the fitted values at
 *            the points are unique, the polynomial away from them is not);
 *            bit 1 set if a coefficient was not finite;
 *            bit 2 set if the node's coefficients went through the
 *            refinement sweep (always on the mixed path; on the float64 path
 *            only for nodes whose normal equations are ill-conditioned or
 *            deflated, see fmt_fit_opts.refine_steps);
 *            bit 3 set (mixed path) if the node's float32 Gram was too
 *            ill-conditioned (estimated condition number above 1e6, or a
 *            deflated pivot) and its normal equations were formed again
 *            from float64 power moments
 */
fmt_status fmt_tree_export_nodes(const fmt_tree* tree, uint8_t* level, uint32_t* prefix,
                                 uint32_t* begin, uint32_t* count, uint32_t* flags, double* coeffs);

/*
 * Copy per-point results to host buffers of info.n_points entries, indexed by
 * the caller's input index (any pointer may be NULL); the residual is the f
 * that Alg. 2 leaves after the deepest node's fit (f - Lambda P_F, summed
 * down the tree):
 *   keys     : Morton key of the point's cell at depth D
 *   order    : order[i] = input index of the i-th point in key order (stable)
 *   leaf     : index (in export order) of the deepest node holding the point
 *   residual : final residual f - fitted value (float64)
 */
fmt_status fmt_tree_export_points(const fmt_tree* tree, uint32_t* keys, uint32_t* order,
                                  uint32_t* leaf, double* residual);

/*
 * Rebuild an evaluable tree from exported nodes (checkpoint / resume of
 * Alg. 1's node records P; the evaluation is Section 2's f'_q = Lambda'_q F_p
 * summed down the tree):
 * `opts` supplies p, max_depth and the box; level, prefix and coeffs are host
 * arrays of `nodes` entries as fmt_tree_export_nodes writes them.  Every
 * non-root node's parent must be present.  Errors: INVALID_ARG, OOM, DEVICE.
 */
fmt_status fmt_tree_import(const fmt_fit_opts* opts, int64_t nodes, const uint8_t* level,
                           const uint32_t* prefix, const double* coeffs, void* stream,
                           fmt_tree** out);

/*
 * Fixed-topology transform: refit `m` new value fields on the points of a
 * fitted tree, keeping its node set.  The map from values to coefficients is
 * then linear (the operator I' of Section 2, eq. identityprime, applied
 * through the tree's nodes): every node of the tree is fitted (Alg. 2) to the
 * residual its ancestors leave of the new field, parents before children,
 * and no octant test is taken.  The power moments and the factor of each
 * node are formed once and shared by the m fields; each field then costs the
 * r-weighted moments, one solve with the kept factor and the residual update
 * per level.  Normal equations in float64 power moments, whatever path the
 * tree was fitted with; the tree's refine_steps apply where the conditioning
 * estimate asks for them (see fmt_fit_opts.refine_steps).
 *   tree       : a tree from fmt_fit or fmt_fit_batch (not an imported one).
 *   x, y, z    : device arrays of n values of `dtype`: the points the tree was
 *                fitted on, in the same order (each point is checked against
 *                the cell the tree recorded for it).
 *   f          : device array of m * n values of `dtype`, field j at f + j n,
 *                in the points' order.  Not modified.
 *   n          : the tree's point count.
 *   m          : 1 .. FMT_REFIT_MAX_FIELDS.
 *   out        : host array of m handles, each a new single-problem tree with
 *                the source tree's nodes (export order and prefixes equal),
 *                its field's coefficients and final residual; release each
 *                with fmt_tree_destroy.  The source tree is unchanged.
 * Runs on `stream` and returns once the trees are complete.  Errors:
 * INVALID_ARG (bad argument, an imported tree, n differs, a point differs
 * from the tree's), OOM, NUMERIC, DEVICE.  On error every out[j] is NULL.
 */
fmt_status fmt_refit(const fmt_tree* tree, const void* x, const void* y, const void* z, const void* f,
                     int64_t n, int m, int dtype, void* stream, fmt_tree** out);

/*
 * Kernel timing (a profiling aid, not part of the method).  While enabled,
 * every kernel launch of fit and eval is bracketed by HIP events recorded on
 * the launch's own stream; fmt_profile_read waits for those events and
 * accumulates, per kernel class, the launch count, the summed duration in
 * milliseconds and the summed work units (points for point sweeps, nodes for
 * per-node kernels, queries for eval).
 */
typedef struct {
  char name[32];
  int64_t launches;
  double ms;
  double units;
} fmt_kernel_stat;

/* Turn timing on (nonzero) or off; returns the previous setting. */
int fmt_profile_enable(int on);
/* Clear the accumulated table. */
void fmt_profile_reset(void);
/* Copy up to max_entries rows (one per kernel class) into `out`; returns the
   number written, or the number of classes if out is NULL. */
int fmt_profile_read(fmt_kernel_stat* out, int max_entries);

/* Release a tree (NULL is ignored).  Waits for the forest's pending work. */
void fmt_tree_destroy(fmt_tree* tree);

/* Message for the last failed call on this thread ("" if none). */
const char* fmt_last_error(void);

/* Library version string. */
const char* fmt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FMT_H */
