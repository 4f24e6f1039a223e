// Host runtime of the FMT library: the level loop that drives the kernels,
// forests (the device storage of one fit or one batch of fits), and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "fmt_common.h"
#include "k_level.h"
#include "k_sort.h"

using namespace fmt;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace {

thread_local std::string g_last_error;

struct FmtError : std::runtime_error {
  fmt_status code;
  FmtError(fmt_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(fmt_status c, const std::string& m) { throw FmtError(c, m); }

void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    fail(FMT_E_OOM, std::string(what) + ": out of device memory");
  }
  fail(FMT_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(x) hip_check((x), #x)

// ---------------------------------------------------------------------------
// kernel timing: events around each launch on its own stream, resolved when
// the caller reads the table
// ---------------------------------------------------------------------------
struct ProfRecord {
  int kernel;
  hipEvent_t a, b;
  double units;   // points (or queries) the launch covered
};
const char* kKernelNames[] = {"keygen", "sort", "gather", "gram", "gram_reduce", "solve", "refine_sweep",
                              "refine_solve", "residual", "children", "emit", "eval_keys", "eval_sort", "eval", "compose",
                              "bmoments", "base_moments", "pyramid", "refit_gather", "refit_moments",
                              "refit_factor", "refit_bmoments", "refit_solve", "refit_residual", "factor_ahead",
                              "solve_ahead", "regram", "rbf_rows", "rbf_pairs"};
enum { KN_KEYGEN, KN_SORT, KN_GATHER, KN_GRAM, KN_REDUCE, KN_SOLVE, KN_RSWEEP, KN_RSOLVE, KN_RESID, KN_CHILD,
       KN_EMIT, KN_EKEYS, KN_ESORT, KN_EVAL, KN_COMPOSE, KN_BMOM, KN_BASEM, KN_PYR, KN_XGATHER, KN_XMOM, KN_XFACTOR,
       KN_XBMOM, KN_XSOLVE, KN_XRESID, KN_UPFAC, KN_FSOLVE, KN_REGRAM, KN_RBF_ROWS, KN_RBF_PAIRS, KN_COUNT };
static_assert(sizeof(kKernelNames) / sizeof(kKernelNames[0]) == KN_COUNT, "one name per kernel class");
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof_pending;
struct ProfAcc {
  int64_t launches = 0;
  double ms = 0, units = 0;
};
ProfAcc g_prof_acc[KN_COUNT];

// Events are recycled: creating them per launch would put host work
// between the launches being timed.
std::vector<hipEvent_t> g_event_pool;

hipEvent_t pooled_event() {
  {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (!g_event_pool.empty()) {
      hipEvent_t e = g_event_pool.back();
      g_event_pool.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  HIPCHK(hipEventCreate(&e));
  return e;
}

struct ProfScope {
  bool on;
  int kernel;
  double units;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(int k, double u, hipStream_t st) : kernel(k), units(u), s(st) {
    {
      std::lock_guard<std::mutex> g(g_prof_mu);
      on = g_prof_on;
    }
    if (on) {
      a = pooled_event();
      b = pooled_event();
      HIPCHK(hipEventRecord(a, s));
    }
  }
  ~ProfScope() {
    if (!on) return;
    if (hipEventRecord(b, s) != hipSuccess) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_pending.push_back(ProfRecord{kernel, a, b, units});
  }
};

void prof_resolve() {
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (auto& r : g_prof_pending) {
    (void)hipEventSynchronize(r.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      g_prof_acc[r.kernel].launches += 1;
      g_prof_acc[r.kernel].ms += ms;
      g_prof_acc[r.kernel].units += r.units;
    }
    g_event_pool.push_back(r.a);
    g_event_pool.push_back(r.b);
  }
  g_prof_pending.clear();
}

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------
// Owning device allocation, or a non-owning view of part of one (view()).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = true;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), owned(o.owned) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      owned = o.owned;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  static DevBuf view(void* base, size_t offset, size_t n) {
    DevBuf b;
    b.p = (char*)base + offset;
    b.bytes = n;
    b.owned = false;
    return b;
  }
  void alloc(size_t n) {
    release();
    if (n == 0) n = 256;
    hip_check(hipMalloc(&p, n), "hipMalloc");
    bytes = n;
    owned = true;
  }
  // grow-only reallocation (contents are not kept)
  void reserve(size_t n) {
    if (n > bytes) alloc(std::max(n, bytes + bytes / 2));
  }
  void release() {
    if (p && owned) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T> T* as() const { return (T*)p; }
};

// Reusable scratch of the level loop, one set per stream (fits on one stream
// are serialised by the stream itself; different streams never share).
struct Workspace {
  // px, py, pz, pf: key-ordered inputs (payload set A); px2 .. pf2: set B
  DevBuf keys_alt, vals_alt, sort_scratch, px, py, pz, pf, px2, py2, pz2, pf2;
  DevBuf partial, fac, part_b, part_ss, cbeg, ccnt, nact, chunk_a, chunk_b, counters, status;
  // the level's nodes flagged for the late refinement and their chunk offsets
  // among them, as the topology kernel lists them; the tiled topology
  // launches' per-tile sums
  DevBuf fsel, emit_tiles;
  // the levels' lists of nodes that span several chunks (one written while
  // the other is read)
  DevBuf multi_a, multi_b;
  // refinement corrections of a level's nodes (late refinement)
  DevBuf delta;
  // float64 moment partials of the mixed path's re-solved nodes
  DevBuf part_rg;
  // a fit's small tables (parameters, pointers, pyramid table, level-0 chunk
  // offsets, status word, flags of the factors made ahead), filled by one copy
  DevBuf small;
  // moment pyramid: entries, the finest cells' point ranges (begin, then
  // count), frames, chunk counts, entries, chunk offsets and chunk partials;
  // the B-only partials of the levels it covers
  DevBuf pyr, pyr_begin, pyr_geo, pyr_nchk, pyr_dst, pyr_off, pyr_part, part_m2;
  // factors of the pyramid's upper levels made ahead of the level loop
  DevBuf fac_up;
  uint32_t* host_counters = nullptr;
  // host-visible, fine-grained words the topology kernel writes the next
  // level's counters and a sequence number into (host view and device view)
  uint32_t* level_flag = nullptr;
  uint32_t* level_flag_dev = nullptr;
  uint32_t level_seq = 0;
  char* stage = nullptr;        // pinned staging for small host-to-device copies
  size_t stage_bytes = 0;
  std::mutex mu;
  Workspace() {
    hip_check(hipHostMalloc((void**)&host_counters, 64, hipHostMallocDefault), "hipHostMalloc");
    hip_check(hipHostMalloc((void**)&level_flag, 64, hipHostMallocMapped | hipHostMallocCoherent), "hipHostMalloc");
    std::memset(level_flag, 0, 64);
    hip_check(hipHostGetDevicePointer((void**)&level_flag_dev, level_flag, 0), "hipHostGetDevicePointer");
  }
  ~Workspace() {
    if (host_counters) (void)hipHostFree(host_counters);
    if (level_flag) (void)hipHostFree(level_flag);
    if (stage) (void)hipHostFree(stage);
  }
  // Wait for the topology kernel's counters of sequence number seq: spin on
  // the host-visible word; every few thousand spins ask whether the stream
  // has drained (then the word must be there, else read the device copy).
  // out: next level's nodes, chunks, points, small nodes; this level's
  // nodes flagged for refinement; next level's multi-chunk nodes; the
  // flagged nodes' chunks
  void wait_level(uint32_t seq, hipStream_t s, uint32_t out[7]) {
    for (uint64_t it = 1;; ++it) {
      if (__atomic_load_n(level_flag + 3, __ATOMIC_ACQUIRE) == seq) {
        out[0] = __atomic_load_n(level_flag + 0, __ATOMIC_RELAXED);
        out[1] = __atomic_load_n(level_flag + 1, __ATOMIC_RELAXED);
        out[2] = __atomic_load_n(level_flag + 2, __ATOMIC_RELAXED);
        out[3] = __atomic_load_n(level_flag + 4, __ATOMIC_RELAXED);
        out[4] = __atomic_load_n(level_flag + 5, __ATOMIC_RELAXED);
        out[5] = __atomic_load_n(level_flag + 6, __ATOMIC_RELAXED);
        out[6] = __atomic_load_n(level_flag + 7, __ATOMIC_RELAXED);
        return;
      }
      if ((it & 4095) == 0) {
        const hipError_t e = hipStreamQuery(s);
        if (e == hipSuccess) {
          if (__atomic_load_n(level_flag + 3, __ATOMIC_ACQUIRE) == seq) continue;
          HIPCHK(hipMemcpy(host_counters, counters_dev, 32, hipMemcpyDeviceToHost));
          out[0] = host_counters[0];
          out[1] = host_counters[1];
          out[2] = host_counters[2];
          out[3] = host_counters[4];
          out[4] = host_counters[5];
          out[5] = host_counters[6];
          out[6] = host_counters[7];
          return;
        }
        if (e != hipErrorNotReady) hip_check(e, "level wait");
      }
      __builtin_ia32_pause();
    }
  }
  const void* counters_dev = nullptr;
  // Pinned buffer of at least n bytes; callers reuse it only after the
  // stream has passed the copies that read it.
  char* staging(size_t n) {
    if (n > stage_bytes) {
      if (stage) (void)hipHostFree(stage);
      stage = nullptr;
      stage_bytes = 0;
      hip_check(hipHostMalloc((void**)&stage, std::max<size_t>(n, 4096), hipHostMallocDefault), "hipHostMalloc");
      stage_bytes = std::max<size_t>(n, 4096);
    }
    return stage;
  }
};

std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> g_ws;

Workspace& workspace_for(hipStream_t s) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_ws_mu);
  auto& w = g_ws[{dev, s}];
  if (!w) w.reset(new Workspace());
  return *w;
}

// ---------------------------------------------------------------------------
// forests and trees
// ---------------------------------------------------------------------------
struct ProblemInfo {
  ProblemParams prm;
  uint32_t root;    // node index of the root
  int64_t n;
};

struct Forest {
  int p = 0, L = 0, D = 0, path = 0, dtype = 0, refine = 0, gram = 0;
  int nprob = 0;
  int pbits = 0;                         // problem-id bits above the Morton bits
  uint32_t nodes = 0;
  std::vector<uint32_t> level_start, level_count, level_points;
  std::vector<ProblemInfo> probs;
  // node table (exact size)
  DevBuf nb_begin, nb_count, nb_prefix, nb_level, nb_problem, nb_parent, nb_first_child, nb_child_mask, nb_flags,
      nb_geo, nb_coef;
  // per point, key order
  DevBuf skey, order, resid;
  uint32_t ntot = 0;
  hipStream_t stream = nullptr;
  uint32_t device_status = 0;
  int device = 0;
  // host copies made on first export
  std::mutex host_mu;
  bool host_ready = false;
  std::vector<uint32_t> h_begin, h_count, h_prefix, h_level, h_problem, h_flags;
  std::vector<double> h_coef;
  // deepest level holding a node
  int depth_present = 0;
  // composite coefficients (each node's chain of polynomials in its own
  // frame), built on the first evaluation; `composed` marks their completion
  std::mutex compose_mu;
  // a single tree's composite coefficients and cell table in one allocation
  // (nb_ccoef and cell_tab[0] are views of it)
  DevBuf eval_mem;
  DevBuf nb_ccoef;
  hipEvent_t composed = nullptr;
  // per problem: cell table (cell of depth T -> deepest node), its depth and
  // the event marking its completion; built on the problem's first evaluation
  std::vector<DevBuf> cell_tab;
  std::vector<int> cell_T;
  std::vector<hipEvent_t> cell_ev;
  ~Forest() {
    if (composed) (void)hipEventDestroy(composed);
    for (hipEvent_t e : cell_ev)
      if (e) (void)hipEventDestroy(e);
  }

  NodeTable table() const {
    NodeTable t;
    t.begin = nb_begin.as<uint32_t>();
    t.count = nb_count.as<uint32_t>();
    t.prefix = nb_prefix.as<uint32_t>();
    t.level = nb_level.as<uint32_t>();
    t.problem = nb_problem.as<uint32_t>();
    t.parent = nb_parent.as<uint32_t>();
    t.first_child = nb_first_child.as<uint32_t>();
    t.child_mask = nb_child_mask.as<uint32_t>();
    t.flags = nb_flags.as<uint32_t>();
    t.geo = nb_geo.as<double>();
    t.coef = nb_coef.as<double>();
    return t;
  }
  size_t device_bytes() const {
    return nb_begin.bytes + nb_count.bytes + nb_prefix.bytes + nb_level.bytes + nb_problem.bytes + nb_parent.bytes +
           nb_first_child.bytes + nb_child_mask.bytes + nb_flags.bytes + nb_geo.bytes + nb_coef.bytes + skey.bytes +
           order.bytes + resid.bytes + nb_ccoef.bytes + cell_bytes();
  }
  size_t cell_bytes() const {
    size_t b = 0;
    for (const DevBuf& t : cell_tab) b += t.bytes;
    return b;
  }
  // The node table lives in one allocation: the node set's arrays (begin ..
  // child_mask, geo) first, topo_bytes of them, then flags and coefficients.
  DevBuf node_block;
  size_t topo_bytes = 0;
  static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
  static size_t node_bytes(uint32_t cap, int L) {
    const size_t u = sizeof(uint32_t) * (size_t)cap;
    return 8 * al256(u) + al256(48ull * cap) + al256(u) + al256(sizeof(double) * (size_t)L * cap);
  }
  // Node arrays for `cap` nodes as views into base (node_bytes(cap, L) bytes).
  void place_nodes(void* base, uint32_t cap) {
    const size_t u = sizeof(uint32_t) * (size_t)cap, g = sizeof(double) * 6 * (size_t)cap;
    topo_bytes = 8 * al256(u) + al256(g);
    DevBuf* u32[8] = {&nb_begin, &nb_count, &nb_prefix, &nb_level, &nb_problem, &nb_parent, &nb_first_child,
                      &nb_child_mask};
    for (int q = 0; q < 8; ++q) *u32[q] = DevBuf::view(base, q * al256(u), u);
    nb_geo = DevBuf::view(base, 8 * al256(u), g);
    nb_flags = DevBuf::view(base, topo_bytes, u);
    nb_coef = DevBuf::view(base, topo_bytes + al256(u), sizeof(double) * (size_t)L * cap);
  }
  void alloc_nodes(uint32_t cap) {
    node_block.alloc(node_bytes(cap, L));
    place_nodes(node_block.p, cap);
  }
  // Take over another forest's node table (block and views).
  void adopt_nodes(Forest& o) {
    nb_begin = std::move(o.nb_begin); nb_count = std::move(o.nb_count); nb_prefix = std::move(o.nb_prefix);
    nb_level = std::move(o.nb_level); nb_problem = std::move(o.nb_problem); nb_parent = std::move(o.nb_parent);
    nb_first_child = std::move(o.nb_first_child); nb_child_mask = std::move(o.nb_child_mask);
    nb_flags = std::move(o.nb_flags); nb_geo = std::move(o.nb_geo); nb_coef = std::move(o.nb_coef);
    node_block = std::move(o.node_block);
    topo_bytes = o.topo_bytes;
  }
  // Per-point arrays (keys, permutation, residual) in one allocation.
  DevBuf point_block;
  static size_t point_bytes(uint32_t n) { return 2 * al256(4ull * n) + 8ull * n; }
  void place_points(void* base, uint32_t n) {
    skey = DevBuf::view(base, 0, 4ull * n);
    order = DevBuf::view(base, al256(4ull * n), 4ull * n);
    resid = DevBuf::view(base, 2 * al256(4ull * n), 8ull * n);
  }
  void alloc_points(uint32_t n) {
    point_block.alloc(point_bytes(n));
    place_points(point_block.p, n);
  }
  // storage shared with other forests (the trees of one refit call), kept
  // alive while any of them lives
  std::shared_ptr<DevBuf> shared;
  void fetch_host() {
    std::lock_guard<std::mutex> g(host_mu);
    if (host_ready) return;
    HIPCHK(hipStreamSynchronize(stream));
    auto get = [&](std::vector<uint32_t>& v, const DevBuf& b) {
      v.resize(nodes);
      if (nodes) HIPCHK(hipMemcpy(v.data(), b.p, sizeof(uint32_t) * nodes, hipMemcpyDeviceToHost));
    };
    get(h_begin, nb_begin); get(h_count, nb_count); get(h_prefix, nb_prefix); get(h_level, nb_level);
    get(h_problem, nb_problem); get(h_flags, nb_flags);
    h_coef.resize((size_t)nodes * L);
    if (nodes) HIPCHK(hipMemcpy(h_coef.data(), nb_coef.p, sizeof(double) * nodes * L, hipMemcpyDeviceToHost));
    host_ready = true;
  }
};

}  // namespace

struct fmt_tree {
  std::shared_ptr<Forest> forest;
  int problem = 0;
  std::vector<uint32_t> nodes;   // this tree's node indices in (level, prefix) order (filled lazily)
  bool nodes_ready = false;
  std::mutex mu;
};

namespace {

const int kRefineMax = 8;

// Streams on which the groups of one batched fit run concurrently: created
// once per device (default priority, blocking like the caller's) and kept
// until the process ends, with their workspaces.
constexpr int kGroupStreams = 4;
std::mutex g_group_mu;
std::map<std::pair<int, int>, hipStream_t> g_group_streams;

hipStream_t group_stream(int idx) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_group_mu);
  hipStream_t& s = g_group_streams[{dev, idx}];
  if (!s) HIPCHK(hipStreamCreate(&s));
  return s;
}

int ceil_log2(int k) {
  int b = 0;
  while ((1 << b) < k) ++b;
  return b;
}

void validate_opts(const fmt_fit_opts& o) {
  if (o.p < 0 || o.p > FMT_MAX_P || (o.p > 8 && !wide_order(o.p)))
    fail(FMT_E_INVALID_ARG, "p must be 0..8, 10, 12 or 14");
  if (o.p > 8 && o.path != FMT_PATH_FP64) fail(FMT_E_INVALID_ARG, "the mixed path supports p <= 8");
  if (o.p > 8 && o.gram == FMT_GRAM_MFMA) fail(FMT_E_INVALID_ARG, "the MFMA Gram supports p <= 8");
  if (o.max_depth < 0 || o.max_depth > FMT_MAX_DEPTH) fail(FMT_E_INVALID_ARG, "max_depth out of range 0..10");
  if (!(o.tol >= 0.0) || std::isinf(o.tol)) fail(FMT_E_INVALID_ARG, "tol must be finite and >= 0");
  if (o.path != FMT_PATH_FP64 && o.path != FMT_PATH_MIXED) fail(FMT_E_INVALID_ARG, "unknown path");
  if (o.refine_steps < 0 || o.refine_steps > kRefineMax) fail(FMT_E_INVALID_ARG, "refine_steps out of range 0..8");
  if (o.gram != FMT_GRAM_MOMENTS && o.gram != FMT_GRAM_MFMA && o.gram != FMT_GRAM_MOMENTS_LEVEL)
    fail(FMT_E_INVALID_ARG, "unknown gram method");
  for (int a = 0; a < 3; ++a)
    if (!(o.box_hi[a] > o.box_lo[a]) || !std::isfinite(o.box_lo[a]) || !std::isfinite(o.box_hi[a]))
      fail(FMT_E_INVALID_ARG, "box_hi must exceed box_lo on every axis");
}

ProblemParams make_params(const fmt_fit_opts& o, uint32_t n, uint32_t offset) {
  ProblemParams P;
  for (int a = 0; a < 3; ++a) {
    P.lo[a] = o.box_lo[a];
    P.hi[a] = o.box_hi[a];
    P.qscale[a] = std::ldexp(1.0, o.max_depth) / (o.box_hi[a] - o.box_lo[a]);
  }
  P.n = n;
  P.offset = offset;
  return P;
}

struct FitInput {
  const void *x, *y, *z, *f;
  int64_t n;
};

// Moment pyramid of a set of problems (the float64 power-moment path): the
// finest cells' ranges, frames and chunks from the sorted keys, their power
// moments M (mode 3, one pass over the points), and each pyramid's coarser
// levels from the finer ones by exact frame shifts.  `tab` is the device
// table (PYR_TAB_WORDS per problem | first finest cell of each pyramid, and
// the total | its problem | at list_off[d] the list_n[d] problems with
// kp > d).  W.pyr_begin (begin, then count, of the finest cells) must hold
// zeros; the pyramid's buffers must be reserved.
struct PyramidShape {
  int K = 0, npyr = 0, kp_max = 0;
  uint64_t base_cells = 0, pyr_cells = 0, chunk_bound = 0;
  std::vector<uint32_t> list_off, list_n;
};
void build_pyramid(Workspace& W, int p, int D, int dtype, const PyramidShape& ps_, const uint32_t* tab,
                   const ProblemParams* d_prm, const uint32_t* skey, uint32_t N, double* resid, hipStream_t s) {
  const uint32_t nbc = (uint32_t)ps_.base_cells;
  const uint32_t NMB = (uint32_t)moment_base_doubles(p);
  const uint32_t* cst = tab + (size_t)PYR_TAB_WORDS * ps_.K;
  PyrTab pt{tab, cst, cst + ps_.npyr + 1, (uint32_t)ps_.npyr};
  {
    ProfScope ps(KN_PYR, nbc, s);
    HIPCHK(launch_pyr_cells(skey, N, D, ps_.K, d_prm, pt, nbc, W.pyr_begin.as<uint32_t>(),
                            W.pyr_begin.as<uint32_t>() + nbc, W.pyr_geo.as<double>(), W.pyr_nchk.as<uint32_t>(),
                            W.pyr_dst.as<uint32_t>(), s));
    HIPCHK(launch_pyr_scan(W.pyr_nchk.as<uint32_t>(), nbc, W.pyr_off.as<uint32_t>(), s));
  }
  {
    // the finest cells as a level of nodes (range, frame, chunks)
    ProfScope ps(KN_BASEM, N, s);
    LevelArgs c{};
    c.nt.begin = W.pyr_begin.as<uint32_t>();
    c.nt.count = W.pyr_begin.as<uint32_t>() + nbc;
    c.nt.geo = W.pyr_geo.as<double>();
    c.node0 = 0;
    c.nnodes = nbc;
    c.chunk_off = W.pyr_off.as<uint32_t>();
    c.nchunks = (uint32_t)ps_.chunk_bound;
    c.px = W.px.p;
    c.py = W.py.p;
    c.pz = W.pz.p;
    c.r = resid;
    c.skey = skey;
    c.D = D;
    HIPCHK(launch_moments(p, 3, dtype, c, W.pyr_part.as<double>(), s));
  }
  {
    ProfScope ps(KN_PYR, (double)ps_.pyr_cells, s);
    HIPCHK(launch_pyr_base(W.pyr_off.as<uint32_t>(), nbc, W.pyr_part.as<double>(), NMB, W.pyr_dst.as<uint32_t>(),
                           W.pyr.as<double>(), s));
    for (int d = ps_.kp_max - 1; d >= 0; --d)
      HIPCHK(launch_pyr_up(p, W.pyr.as<double>(), tab, tab + ps_.list_off[d], ps_.list_n[d], d, s));
  }
}
void reserve_pyramid(Workspace& W, int p, const PyramidShape& ps_) {
  const uint64_t NMB = moment_base_doubles(p), nbc = ps_.base_cells;
  W.pyr.reserve(8ull * NMB * ps_.pyr_cells);
  W.pyr_begin.reserve(8ull * nbc);   // begin, then count
  W.pyr_geo.reserve(48ull * nbc);
  W.pyr_nchk.reserve(4ull * nbc);
  W.pyr_dst.reserve(4ull * nbc);
  W.pyr_off.reserve(4ull * (nbc + 1));
  W.pyr_part.reserve(8ull * NMB * ps_.chunk_bound);
}

// The r-weighted moments of a level (same output layout either way): the
// nodes with at least SMALL_NODE points in staged chunks of eight waves
// (mode 2), the smaller ones with two waves per chunk reading the points in
// place (mode 4); a launch only for a kind the level holds.
void launch_bmoments(int p, int dtype, const LevelArgs& a, uint32_t small, double* part, hipStream_t s) {
  if (small < a.nnodes) HIPCHK(launch_moments(p, 2, dtype, a, part, s));
  if (small > 0) HIPCHK(launch_moments(p, 4, dtype, a, part, s));
}

// One batched pass of Alg. 1 over `in.size()` problems sharing p, D, path
// and refinement count.
std::shared_ptr<Forest> fit_group(const fmt_fit_opts& o, const std::vector<fmt_fit_opts>& per,
                                  const std::vector<FitInput>& in, int dtype, hipStream_t s) {
  auto F = std::make_shared<Forest>();
  F->p = o.p;
  F->L = basis_size(o.p);
  F->D = o.max_depth;
  F->path = o.path;
  F->dtype = dtype;
  F->refine = o.refine_steps;
  F->gram = o.path == FMT_PATH_MIXED ? FMT_GRAM_MFMA : o.gram;
  // large bases: per-level moments (no pyramid: its frame shifts of moments
  // up to degree 2p = 28 would cancel too many digits) and the tiled solve
  const bool wide = wide_order(o.p);
  if (wide) F->gram = FMT_GRAM_MOMENTS_LEVEL;
  F->nprob = (int)in.size();
  F->stream = s;
  HIPCHK(hipGetDevice(&F->device));
  const int K = F->nprob;
  F->pbits = K > 1 ? ceil_log2(K) : 0;
  if (3 * F->D + F->pbits > 32) fail(FMT_E_INVALID_ARG, "too many problems for the key width at this depth");
  const uint32_t L = (uint32_t)F->L;
  uint64_t ntot = 0;
  std::vector<ProblemParams> prm(K);
  std::vector<PtrSet> ptrs(K);
  std::vector<double> tols(K);
  for (int k = 0; k < K; ++k) {
    if (in[k].n < (int64_t)L) fail(FMT_E_UNDERDETERMINED, "the root holds fewer than calL points");
    if (!in[k].x || !in[k].y || !in[k].z || !in[k].f) fail(FMT_E_INVALID_ARG, "NULL input pointer");
    prm[k] = make_params(per[k], (uint32_t)in[k].n, (uint32_t)ntot);
    ptrs[k] = PtrSet{in[k].x, in[k].y, in[k].z, in[k].f};
    tols[k] = per[k].tol;
    ntot += (uint64_t)in[k].n;
    if (ntot >= (1ull << 31)) fail(FMT_E_INVALID_ARG, "total point count must stay below 2^31");
  }
  for (int k = 1; k < K; ++k)
    if (tols[k] != tols[0]) fail(FMT_E_INVALID_ARG, "one batched pass needs one tolerance");
  const uint32_t N = (uint32_t)ntot;
  F->ntot = N;
  const size_t esz = dtype == FMT_F32 ? 4 : 8;

  Workspace& W = workspace_for(s);
  std::lock_guard<std::mutex> wlock(W.mu);

  // per-point storage kept by the forest
  F->alloc_points(N);
  W.keys_alt.reserve(4ull * N);
  W.vals_alt.reserve(4ull * N);
  W.sort_scratch.reserve(4 * radix_sort_scratch_words(N));
  for (DevBuf* b : {&W.px, &W.py, &W.pz, &W.pf, &W.px2, &W.py2, &W.pz2, &W.pf2}) b->reserve(esz * N);
  W.counters.reserve(64);

  // Moment pyramid of each problem (float64 power-moment path): its depth
  // kp is the deepest level (at most 5, at most D) whose cells hold calL
  // points on average, 0 (none) if that is the root.  It depends on the
  // problem alone, so a problem fitted in a batch gets the bits it gets
  // fitted alone.  Batches beyond the table limits fit without pyramids.
  const bool use_moments = F->gram == FMT_GRAM_MOMENTS || F->gram == FMT_GRAM_MOMENTS_LEVEL;
  const uint32_t NMB = (uint32_t)moment_base_doubles(F->p);
  std::vector<uint32_t> kp(K, 0);
  if (F->gram == FMT_GRAM_MOMENTS)
    for (int k = 0; k < K; ++k) {
      int d = 0;
      while (d < std::min(F->D, 5) && (uint64_t)in[k].n >= ((uint64_t)L << (3 * (d + 1)))) ++d;
      kp[k] = (uint32_t)d;
    }
  // device table: (first entry, kp, first flat finest cell, 0) per problem |
  // first flat finest cell of each pyramid (+ total) | its problem | per
  // level d, the problems with kp > d
  std::vector<uint32_t> ptab;
  uint64_t pyr_cells = 0, base_cells = 0, pyr_chunk_bound = 0;
  int npyr = 0, kp_max = 0;
  std::vector<uint32_t> list_off, list_n;
  for (int pass = 0; pass < 2; ++pass) {
    ptab.assign((size_t)PYR_TAB_WORDS * K, 0);
    std::vector<uint32_t> cstart, bq;
    pyr_cells = base_cells = 0;
    kp_max = 0;
    for (int k = 0; k < K; ++k) {
      ptab[PYR_TAB_WORDS * k] = (uint32_t)pyr_cells;
      ptab[PYR_TAB_WORDS * k + 1] = kp[k];
      ptab[PYR_TAB_WORDS * k + 2] = (uint32_t)base_cells;
      if (kp[k] == 0) continue;
      cstart.push_back((uint32_t)base_cells);
      bq.push_back((uint32_t)k);
      pyr_cells += level_first((int)kp[k] + 1);
      base_cells += 1ull << (3 * kp[k]);
      kp_max = std::max(kp_max, (int)kp[k]);
    }
    npyr = (int)bq.size();
    pyr_chunk_bound = N / CHUNK + base_cells;   // >= the finest cells' chunk count
    if (pass == 0 && npyr > 0 &&
        (base_cells > (1ull << 18) || 8ull * NMB * (pyr_cells + pyr_chunk_bound) > (2ull << 30))) {
      std::fill(kp.begin(), kp.end(), 0u);
      continue;
    }
    cstart.push_back((uint32_t)base_cells);
    ptab.insert(ptab.end(), cstart.begin(), cstart.end());
    ptab.insert(ptab.end(), bq.begin(), bq.end());
    list_off.assign(kp_max, 0);
    list_n.assign(kp_max, 0);
    for (int d = 0; d < kp_max; ++d) {
      list_off[d] = (uint32_t)ptab.size();
      for (int k = 0; k < K; ++k)
        if ((int)kp[k] > d) ptab.push_back((uint32_t)k);
      list_n[d] = (uint32_t)ptab.size() - list_off[d];
    }
    break;
  }
  if (npyr == 0) ptab.clear();
  // Factors of the pyramid's upper levels (above each problem's finest), made
  // in one launch before the level loop: per problem the levels 0 .. ku-1,
  // ku <= kp, as many as fit a bound on their storage.  Their pyramid
  // entries are listed after the table; word 3 of a problem's entry gives its
  // first slot and ku.
  uint32_t up_cells = 0, up_off = 0;
  const size_t fd_bytes = 8 * factor_doubles(F->p);
  if (npyr > 0) {
    int ku_max = kp_max;
    auto cells_for = [&](int ku) {
      uint64_t c = 0;
      for (int k = 0; k < K; ++k) c += level_first(std::min((int)kp[k], ku));
      return c;
    };
    while (ku_max > 0 && cells_for(ku_max) * fd_bytes > (256ull << 20)) --ku_max;
    up_off = (uint32_t)ptab.size();
    for (int k = 0; k < K && ku_max > 0; ++k) {
      const uint32_t ku = (uint32_t)std::min((int)kp[k], ku_max);
      if (ku == 0) continue;
      ptab[PYR_TAB_WORDS * k + 3] = up_cells | (ku << 28);
      for (uint32_t e = 0; e < level_first((int)ku); ++e) ptab.push_back(ptab[PYR_TAB_WORDS * k] + e);
      up_cells += level_first((int)ku);
    }
  }
  PyramidShape pshape;
  pshape.K = K;
  pshape.npyr = npyr;
  pshape.kp_max = kp_max;
  pshape.base_cells = base_cells;
  pshape.pyr_cells = pyr_cells;
  pshape.chunk_bound = pyr_chunk_bound;
  pshape.list_off = list_off;
  pshape.list_n = list_n;
  if (npyr > 0) {
    reserve_pyramid(W, F->p, pshape);
    if (up_cells) W.fac_up.reserve(fd_bytes * up_cells);
  }

  // The small per-fit tables go to the device in one copy from pinned
  // staging: parameters, pointers, the pyramid table, the level-0 chunk
  // offsets, and zeros for the status word and the ahead factors' flags.
  std::vector<uint32_t> off0(K + 1, 0);
  for (int k = 0; k < K; ++k) off0[k + 1] = off0[k] + (uint32_t)((in[k].n + CHUNK - 1) / CHUNK);
  auto al256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t prm_b = sizeof(ProblemParams) * K, ptr_b = sizeof(PtrSet) * K, off_b = 4ull * (K + 1);
  const size_t tab_b = 4ull * ptab.size();
  const size_t o_ptr = al256(prm_b), o_tab = o_ptr + al256(ptr_b), o_off = o_tab + al256(tab_b);
  const size_t o_st = o_off + al256(off_b), o_up = o_st + 256, n_small = o_up + al256(4ull * up_cells);
  W.small.reserve(n_small);
  char* stg = W.staging(n_small);
  std::memcpy(stg, prm.data(), prm_b);
  std::memcpy(stg + o_ptr, ptrs.data(), ptr_b);
  if (tab_b) std::memcpy(stg + o_tab, ptab.data(), tab_b);
  std::memcpy(stg + o_off, off0.data(), off_b);
  std::memset(stg + o_st, 0, n_small - o_st);
  HIPCHK(hipMemcpyAsync(W.small.p, stg, n_small, hipMemcpyHostToDevice, s));
  char* sm = W.small.as<char>();
  const ProblemParams* d_prm = reinterpret_cast<const ProblemParams*>(sm);
  const PtrSet* d_ptrs = reinterpret_cast<const PtrSet*>(sm + o_ptr);
  const uint32_t* pyr_dev = npyr > 0 ? reinterpret_cast<const uint32_t*>(sm + o_tab) : nullptr;
  uint32_t* d_status = reinterpret_cast<uint32_t*>(sm + o_st);
  uint32_t* d_upflags = reinterpret_cast<uint32_t*>(sm + o_up);

  // K1 keys, K2 sort with the inputs as payload (K3: the sort itself leaves
  // them in key order).  With an odd number of sort passes the keys start in
  // the alternate buffer so that the sorted result lands in the forest's
  // arrays.  A batch's inputs are first concatenated (by the key kernel) so
  // that the first pass reads one array per coordinate.
  const int key_bits = 3 * F->D + F->pbits;
  const bool odd = (radix_sort_passes(key_bits) & 1) != 0;
  uint32_t* k_in = odd ? W.keys_alt.as<uint32_t>() : F->skey.as<uint32_t>();
  uint32_t* v_in = odd ? W.vals_alt.as<uint32_t>() : F->order.as<uint32_t>();
  uint32_t* k_out = odd ? F->skey.as<uint32_t>() : W.keys_alt.as<uint32_t>();
  uint32_t* v_out = odd ? F->order.as<uint32_t>() : W.vals_alt.as<uint32_t>();
  PtrSet cat{nullptr, nullptr, nullptr, nullptr};
  if (K > 1) cat = PtrSet{W.px.p, W.py.p, W.pz.p, W.pf.p};
  {
    ProfScope ps(KN_KEYGEN, N, s);
    HIPCHK(launch_keygen(dtype, d_ptrs, d_prm, K, F->D, N, k_in, d_status, cat, s));
  }
  bool in_alt = false;
  {
    ProfScope ps(KN_SORT, N, s);
    const void* pin[4];
    if (K > 1) {
      pin[0] = W.px.p; pin[1] = W.py.p; pin[2] = W.pz.p; pin[3] = W.pf.p;
    } else {
      pin[0] = in[0].x; pin[1] = in[0].y; pin[2] = in[0].z; pin[3] = in[0].f;
    }
    void* pay[4] = {W.px.p, W.py.p, W.pz.p, W.pf.p};
    void* pay_alt[4] = {W.px2.p, W.py2.p, W.pz2.p, W.pf2.p};
    HIPCHK(radix_sort_payload(dtype, 4, k_in, v_in, k_out, v_out, pin, pay, pay_alt, N, key_bits,
                              W.sort_scratch.as<uint32_t>(), s, &in_alt));
  }
  if (in_alt != odd) fail(FMT_E_DEVICE, "internal: sort result in an unexpected buffer");
  if (in_alt) {
    std::swap(W.px, W.px2);
    std::swap(W.py, W.py2);
    std::swap(W.pz, W.pz2);
    std::swap(W.pf, W.pf2);
  }
  {
    ProfScope ps(KN_GATHER, N, s);
    // the pyramid's finest-cell ranges (begin, then count) are cleared here too
    HIPCHK(launch_widen(dtype, W.pf.p, N, F->resid.as<double>(), npyr > 0 ? W.pyr_begin.as<uint32_t>() : nullptr,
                        npyr > 0 ? 2 * (uint32_t)base_cells : 0u, s));
  }

  if (npyr > 0) {
    // finest cells of every pyramid: ranges, frames, chunks; their power
    // moments M; then each pyramid's coarser levels from the finer ones
    build_pyramid(W, F->p, F->D, dtype, pshape, pyr_dev, d_prm, F->skey.as<uint32_t>(), N, F->resid.as<double>(), s);
    if (up_cells) {
      ProfScope ps(KN_UPFAC, up_cells, s);
      HIPCHK(launch_factor_cells(F->p, W.pyr.as<double>(), pyr_dev + up_off, up_cells, F->refine > 0 ? 1 : 0,
                                 W.fac_up.as<double>(), d_upflags, s));
    }
  }

  // node capacity: at depth d at most min(K 8^d, N / L) nodes
  uint64_t cap = 0;
  for (int d = 0; d <= F->D; ++d) {
    uint64_t a = (uint64_t)K << std::min(3 * d, 40);
    cap += std::min<uint64_t>(a, d == 0 ? (uint64_t)K : std::max<uint64_t>(N / L, 1));
  }
  if (cap >= (1ull << 31)) fail(FMT_E_INVALID_ARG, "node capacity overflow");
  Forest tmp;   // workspace node table with the capacity bound
  tmp.L = F->L;
  tmp.alloc_nodes((uint32_t)cap);
  NodeTable nt = tmp.table();
  HIPCHK(launch_roots(nt, d_prm, K, s));


  uint32_t nnodes = (uint32_t)K, nchunks = off0[K], node0 = 0;
  uint32_t level_points = N;
  uint32_t nsmall = 0;   // nodes of the level with fewer than SMALL_NODE points
  for (int k = 0; k < K; ++k) nsmall += in[k].n < (int64_t)SMALL_NODE ? 1u : 0u;
  F->level_start.clear();
  F->level_count.clear();
  // chunk offsets: level 0's from the staged tables, then chunk_a and
  // chunk_b in turn
  const uint32_t* cur_off = reinterpret_cast<const uint32_t*>(sm + o_off);
  DevBuf* next_off = &W.chunk_a;
  // the level's multi-chunk nodes as the previous topology pass listed them
  // (level 0: not listed)
  const uint32_t* cur_multi = nullptr;
  uint32_t cur_nmulti = 0;
  DevBuf* next_multi = &W.multi_a;
  const size_t gpd = use_moments ? moment_partial_doubles(F->p) : gram_partial_doubles(F->p);
  const size_t fd = wide ? wide_factor_doubles(F->p) : factor_doubles(F->p);
  const size_t rbd = moment_refine_doubles(F->p);
  for (int d = 0; d <= F->D && nnodes > 0; ++d) {
    F->level_start.push_back(node0);
    F->level_count.push_back(nnodes);
    // nodes of this level whose M the pyramid holds (mode 2) and the others (mode 0)
    bool lvl_pyr = false, lvl_pts = !use_moments;
    for (int k = 0; k < K; ++k) {
      if (pyramid_covers(kp[k], d)) lvl_pyr = true;
      else lvl_pts = true;
    }
    if (lvl_pts) W.partial.reserve(8ull * gpd * nchunks);
    if (lvl_pyr) W.part_m2.reserve(8ull * rbd * nchunks);
    if (wide) {
      // every node's factor stays in device memory for the level
      if (8ull * fd * nnodes > (32ull << 30))
        fail(FMT_E_OOM, "a level of the large-basis fit needs more than 32 GiB of factors");
      W.fac.reserve(8ull * fd * nnodes);
    }
    if (F->refine > 0) {
      W.fac.reserve(8ull * fd * nnodes);
      W.part_b.reserve(8ull * rbd * nchunks);
    }
    W.part_ss.reserve(8ull * 16 * nchunks);
    W.cbeg.reserve(4ull * 8 * nnodes);
    W.ccnt.reserve(4ull * 8 * nnodes);
    W.nact.reserve(4ull * nnodes);
    next_off->reserve(4ull * (8ull * nnodes + 1));
    next_multi->reserve(4ull * 8ull * nnodes);
    W.fsel.reserve(4ull * (2ull * nnodes + 2));
    W.emit_tiles.reserve(4ull * emit_tile_words(nnodes));

    LevelArgs a;
    a.nt = nt;
    a.node0 = node0;
    a.nnodes = nnodes;
    a.chunk_off = cur_off;
    a.multi = cur_multi;
    a.nmulti = cur_nmulti;
    a.nchunks = nchunks;
    a.px = W.px.p;
    a.py = W.py.p;
    a.pz = W.pz.p;
    a.r = F->resid.as<double>();
    a.skey = F->skey.as<uint32_t>();
    a.level = d;
    a.D = F->D;
    a.tol = tols[0];
    // the mixed path's float32 Gram always needs the sweeps; the float64
    // path applies them where the conditioning estimate asks for them
    a.refine = F->refine == 0 ? 0 : (F->path == FMT_PATH_MIXED ? 2 : 1);
    a.pyr_tab = npyr > 0 ? pyr_dev : nullptr;
    a.fac_up = up_cells ? W.fac_up.as<double>() : nullptr;
    a.up_flags = up_cells ? d_upflags : nullptr;
    a.status = d_status;
    a.nsmall = nsmall;
    // the mixed path's float32 Gram: too ill-conditioned nodes go to a
    // float64 re-solve
    a.regram = F->path == FMT_PATH_MIXED ? 1u : 0u;

    const bool multi = nchunks > nnodes;   // some node spans several chunks
    if (lvl_pyr) {
      ProfScope ps(KN_BMOM, level_points, s);
      launch_bmoments(F->p, dtype, a, nsmall, W.part_m2.as<double>(), s);
    }
    if (lvl_pts) {
      ProfScope ps(KN_GRAM, level_points, s);
      if (use_moments) HIPCHK(launch_moments(F->p, 0, dtype, a, W.partial.as<double>(), s));
      else HIPCHK(launch_gram(F->p, F->path, dtype, a, W.partial.as<double>(), s));
    }
    if (multi) {
      ProfScope ps(KN_REDUCE, (double)nchunks * (double)((lvl_pts ? gpd : 0) + (lvl_pyr ? rbd : 0)), s);
      if (lvl_pts) HIPCHK(launch_chunk_reduce(a, W.partial.as<double>(), (uint32_t)gpd, s));
      if (lvl_pyr) HIPCHK(launch_chunk_reduce(a, W.part_m2.as<double>(), (uint32_t)rbd, s));
    }
    // nodes whose factor was made ahead (problems with ku > d) and the others
    uint32_t n_ahead_probs = 0;
    for (int k = 0; k < K && up_cells; ++k)
      if ((ptab[PYR_TAB_WORDS * k + 3] >> 28) > (uint32_t)d) ++n_ahead_probs;
    {
      double* fac = F->refine > 0 ? W.fac.as<double>() : nullptr;
      if (n_ahead_probs > 0) {
        ProfScope ps(KN_FSOLVE, nnodes, s);
        HIPCHK(launch_solve_ahead(F->p, a, W.part_m2.as<double>(), fac, s));
      }
      if (wide) {
        ProfScope ps(KN_SOLVE, nnodes, s);
        HIPCHK(launch_wide_factor(F->p, a, W.partial.as<double>(), W.fac.as<double>(), s));
        HIPCHK(launch_wide_solve(F->p, a, W.partial.as<double>(), W.fac.as<double>(), s));
      } else if (n_ahead_probs < (uint32_t)K) {
        ProfScope ps(KN_SOLVE, nnodes, s);
        if (use_moments)
          HIPCHK(launch_solve_moments(F->p, a, W.partial.as<double>(), W.part_m2.as<double>(), W.pyr.as<double>(),
                                      fac, s));
        else HIPCHK(launch_solve(F->p, a, W.partial.as<double>(), fac, s));
      }
      if (a.regram) {
        // nodes whose float32 Gram the solve refused (FLAG_REGRAM): float64
        // power moments of their chunks, then the float64 solve; the other
        // nodes' workgroups exit at once
        ProfScope ps(KN_REGRAM, level_points, s);
        const size_t mpd = moment_partial_doubles(F->p);
        W.part_rg.reserve(8ull * mpd * nchunks);
        LevelArgs r = a;
        r.regram = 0;
        r.only_flag = FLAG_REGRAM;
        HIPCHK(launch_moments(F->p, 0, dtype, r, W.part_rg.as<double>(), s));
        if (multi) HIPCHK(launch_chunk_reduce(r, W.part_rg.as<double>(), (uint32_t)mpd, s));
        HIPCHK(launch_solve_moments(F->p, r, W.part_rg.as<double>(), nullptr, nullptr, fac, s));
      }
    }
    // The float64 small-basis path refines only the nodes its condition
    // estimate flags, usually none: the refinement then runs after the
    // residual update and the level's topology pass, which reports how many
    // nodes are flagged, and only if there are any (late refinement: sweep
    // of the updated residual, correction delta, r -= Lambda delta on the
    // flagged nodes, topology again).  The mixed path (every node) and the
    // large bases refine before the residual update.
    const bool late_refine = a.refine == 1 && !wide;
    // the topology pass's counters (see wait_level)
    uint32_t cnt[7];
    // listed: the topology pass has listed the flagged nodes (cnt holds their
    // numbers), and the passes launch over those alone
    auto refine_late = [&](bool listed) {
      W.delta.reserve(8ull * L * nnodes);
      LevelArgs r = a;
      r.sweep_current = 1;
      r.delta = W.delta.as<double>();
      if (listed) {
        r.sel = W.fsel.as<uint32_t>();
        r.sel_off = r.sel + nnodes + 1;
        r.nsel = cnt[4];
        r.nsel_chunks = cnt[6];
      }
      for (int it = 0; it < F->refine; ++it) {
        {
          ProfScope ps(KN_RSWEEP, level_points, s);
          HIPCHK(launch_moments(F->p, 1, dtype, r, W.part_b.as<double>(), s));
        }
        {
          ProfScope ps(KN_RSOLVE, nnodes, s);
          HIPCHK(launch_refine_solve(F->p, r, W.part_b.as<double>(), W.fac.as<double>(), s));
        }
        ProfScope ps(KN_RESID, level_points, s);
        LevelArgs c = r;
        c.only_flag = FLAG_REFINE;
        HIPCHK(launch_residual(F->p, dtype, c, W.part_ss.as<double>(), s));
        if (listed) {
          // the listed nodes that span several chunks
          c.multi = r.sel;
          c.nmulti = r.nsel;
        }
        if (multi && d < F->D) HIPCHK(launch_chunk_reduce(c, W.part_ss.as<double>(), 16, s));
      }
    };
    for (int it = 0; it < (late_refine ? 0 : F->refine); ++it) {
      {
        ProfScope ps(KN_RSWEEP, level_points, s);
        HIPCHK(launch_moments(F->p, 1, dtype, a, W.part_b.as<double>(), s));
        // every node refined, or the tiled solve (which reads the summed
        // partial): sum the chunks in parallel first (the refinement solve
        // otherwise sums its node's chunks itself)
        if (multi && (a.refine == 2 || wide))
          HIPCHK(launch_chunk_reduce(a, W.part_b.as<double>(), (uint32_t)rbd, s));
      }
      ProfScope ps(KN_RSOLVE, nnodes, s);
      if (wide) HIPCHK(launch_wide_refine_solve(F->p, a, W.part_b.as<double>(), W.fac.as<double>(), s));
      else HIPCHK(launch_refine_solve(F->p, a, W.part_b.as<double>(), W.fac.as<double>(), s));
    }
    {
      ProfScope ps(KN_RESID, level_points, s);
      HIPCHK(launch_residual(F->p, dtype, a, W.part_ss.as<double>(), s));
      if (multi && d < F->D) HIPCHK(launch_chunk_reduce(a, W.part_ss.as<double>(), 16, s));
    }
    F->level_points.push_back(level_points);
    if (d == F->D) {
      if (late_refine && F->refine > 0) refine_late(false);   // no topology pass to list the flagged nodes
      node0 += nnodes;
      break;
    }
    const uint32_t next0 = node0 + nnodes;
    auto topology = [&](void) {
      {
        ProfScope ps(KN_CHILD, nnodes, s);
        HIPCHK(launch_children(F->p, a, W.part_ss.as<double>(), W.cbeg.as<uint32_t>(), W.ccnt.as<uint32_t>(),
                               W.nact.as<uint32_t>(), s));
      }
      const uint32_t seq = ++W.level_seq;
      {
        ProfScope ps(KN_EMIT, nnodes, s);
        HIPCHK(launch_emit(a, d_prm, W.cbeg.as<uint32_t>(), W.ccnt.as<uint32_t>(), W.nact.as<uint32_t>(), next0,
                           next_off->as<uint32_t>(), W.counters.as<uint32_t>(), W.level_flag_dev, seq,
                           next_multi->as<uint32_t>(), W.fsel.as<uint32_t>(), W.emit_tiles.as<uint32_t>(), s));
      }
      W.counters_dev = W.counters.p;
      W.wait_level(seq, s, cnt);
    };
    topology();
    if (late_refine && F->refine > 0 && cnt[4] > 0) {
      // flagged nodes: refine them and take the topology of the corrected
      // residual
      refine_late(true);
      topology();
    }
    node0 = next0;
    nnodes = cnt[0];
    nchunks = cnt[1];
    level_points = cnt[2];
    nsmall = cnt[3];
    cur_off = next_off->as<uint32_t>();
    next_off = next_off == &W.chunk_a ? &W.chunk_b : &W.chunk_a;
    cur_multi = next_multi->as<uint32_t>();
    cur_nmulti = cnt[5];
    next_multi = next_multi == &W.multi_a ? &W.multi_b : &W.multi_a;
  }
  F->nodes = node0;
  F->depth_present = (int)F->level_start.size() - 1;

  // hand the node table to the forest; copy it down to its exact size only
  // when the capacity bound would hold much more memory than the nodes need
  const size_t per_node = 4ull * 9 + 48ull + 8ull * L;
  if ((uint64_t)cap * per_node <= (64ull << 20) || (uint64_t)cap <= 2ull * F->nodes) {
    F->adopt_nodes(tmp);
  } else {
    F->alloc_nodes(std::max<uint32_t>(F->nodes, 1));
    auto cp = [&](DevBuf& dst, const DevBuf& src, size_t bytes) {
      if (bytes) HIPCHK(hipMemcpyAsync(dst.p, src.p, bytes, hipMemcpyDeviceToDevice, s));
    };
    const size_t un = 4ull * F->nodes;
    cp(F->nb_begin, tmp.nb_begin, un); cp(F->nb_count, tmp.nb_count, un); cp(F->nb_prefix, tmp.nb_prefix, un);
    cp(F->nb_level, tmp.nb_level, un); cp(F->nb_problem, tmp.nb_problem, un); cp(F->nb_parent, tmp.nb_parent, un);
    cp(F->nb_first_child, tmp.nb_first_child, un); cp(F->nb_child_mask, tmp.nb_child_mask, un);
    cp(F->nb_flags, tmp.nb_flags, un);
    cp(F->nb_geo, tmp.nb_geo, 48ull * F->nodes);
    cp(F->nb_coef, tmp.nb_coef, 8ull * L * F->nodes);
  }
  HIPCHK(hipMemcpyAsync(W.host_counters + 4, d_status, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  F->device_status = W.host_counters[4];

  F->probs.resize(K);
  for (int k = 0; k < K; ++k) {
    F->probs[k].prm = prm[k];
    F->probs[k].root = (uint32_t)k;
    F->probs[k].n = in[k].n;
  }
  if (F->device_status & STATUS_DOMAIN) fail(FMT_E_DOMAIN, "a point is NaN or outside the box");
  if (F->device_status & STATUS_NONFINITE) fail(FMT_E_NUMERIC, "a non-finite coefficient was produced");
  return F;
}

// Node table of a single-problem forest from its nodes in (level, prefix)
// order (level, prefix, first sorted point, count): parents, first children
// and child masks from the (level, prefix) pairs, frames from the box, flags
// cleared, level ranges and depth.  Coefficients are uploaded when hcoef is
// given.  Fails on a duplicate node or a missing parent.  The uploads are
// asynchronous on s from host vectors: the caller synchronises s before they
// go out of scope.
void build_single_nodes(Forest& F, const std::vector<uint32_t>& hl, const std::vector<uint32_t>& hp,
                        const std::vector<uint32_t>& hb, const std::vector<uint32_t>& hc, const double* hcoef,
                        const ProblemParams& prm, hipStream_t s) {
  const uint32_t M = (uint32_t)hl.size();
  // level ranges (nodes are in (level, prefix) order)
  F.level_start.clear();
  F.level_count.clear();
  for (uint32_t j = 0; j < M; ++j) {
    if (j == 0 || hl[j] != hl[j - 1]) {
      F.level_start.push_back(j);
      F.level_count.push_back(0);
    } else if (hp[j] == hp[j - 1]) {
      fail(FMT_E_INVALID_ARG, "duplicate node");
    }
    ++F.level_count.back();
  }
  if (!F.nb_begin.p) F.alloc_nodes(std::max<uint32_t>(M, 1));
  F.nodes = M;
  // host image of the node set's arrays, laid out as on the device
  const size_t u = 4ull * std::max<uint32_t>(M, 1), ua = (u + 255) & ~(size_t)255;
  std::vector<uint32_t> img(F.topo_bytes / 4 + ua / 4, 0u);   // + flags (zero)
  uint32_t* hbeg = img.data();
  uint32_t* hcnt = hbeg + ua / 4;
  uint32_t* hpre = hbeg + 2 * ua / 4;
  uint32_t* hlev = hbeg + 3 * ua / 4;
  uint32_t* hpar = hbeg + 5 * ua / 4;
  uint32_t* hfc = hbeg + 6 * ua / 4;
  uint32_t* hcm = hbeg + 7 * ua / 4;
  size_t d = 0;   // level index of node j
  for (uint32_t j = 0; j < M; ++j) {
    while (d + 1 < F.level_start.size() && F.level_start[d + 1] <= j) ++d;
    hbeg[j] = hb[j];
    hcnt[j] = hc[j];
    hpre[j] = hp[j];
    hlev[j] = hl[j];
    if (hl[j] == 0) {
      hpar[j] = j;
      continue;
    }
    // the parent: prefix >> 3 in the previous level present, which must be level hl[j] - 1
    if (d == 0 || hl[F.level_start[d - 1]] != hl[j] - 1) fail(FMT_E_INVALID_ARG, "a node's parent is missing");
    const uint32_t* lo = hp.data() + F.level_start[d - 1];
    const uint32_t* hi = lo + F.level_count[d - 1];
    const uint32_t* it = std::lower_bound(lo, hi, hp[j] >> 3);
    if (it == hi || *it != (hp[j] >> 3)) fail(FMT_E_INVALID_ARG, "a node's parent is missing");
    const uint32_t par = (uint32_t)(it - hp.data());
    hpar[j] = par;
    if (hcm[par] == 0) hfc[par] = j;
    hcm[par] |= 1u << (hp[j] & 7u);
  }
  // one upload of the whole image (geo is computed on the device below; the
  // flags after it start at zero)
  HIPCHK(hipMemcpyAsync(F.nb_begin.p, img.data(), 8 * ua, hipMemcpyHostToDevice, s));   // start of the node arrays
  HIPCHK(hipMemcpyAsync(F.nb_flags.p, img.data() + F.topo_bytes / 4, u, hipMemcpyHostToDevice, s));
  if (hcoef && M) HIPCHK(hipMemcpyAsync(F.nb_coef.p, hcoef, 8ull * M * F.L, hipMemcpyHostToDevice, s));
  DevBuf dprm(sizeof(ProblemParams));
  HIPCHK(hipMemcpyAsync(dprm.p, &prm, sizeof(ProblemParams), hipMemcpyHostToDevice, s));
  HIPCHK(launch_node_geo(F.table(), dprm.as<ProblemParams>(), M, s));
  HIPCHK(hipStreamSynchronize(s));   // dprm and the host image die here
  F.depth_present = M ? (int)hl[M - 1] : 0;
}

fmt_status guard(const std::function<void()>& body) {
  try {
    body();
    g_last_error.clear();
    return FMT_OK;
  } catch (const FmtError& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host out of memory";
    return FMT_E_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return FMT_E_DEVICE;
  } catch (...) {
    g_last_error = "unknown error";
    return FMT_E_DEVICE;
  }
}

void ensure_tree_nodes(fmt_tree* t) {
  std::lock_guard<std::mutex> g(t->mu);
  if (t->nodes_ready) return;
  Forest& F = *t->forest;
  F.fetch_host();
  t->nodes.clear();
  for (uint32_t i = 0; i < F.nodes; ++i)
    if ((int)F.h_problem[i] == t->problem) t->nodes.push_back(i);
  t->nodes_ready = true;
}

// Fixed-topology refit of m value fields on the points of tree t (see
// fmt_refit).  Per level: the power moments M of every node once (mode 3),
// its factor once, then per field the r-weighted moments B (mode 2), the
// solve with the kept factor, the refinement sweeps where the conditioning
// estimate asks for them, and the residual update.  Returns m single-problem
// forests holding the tree's node set.
std::vector<std::shared_ptr<Forest>> refit_forests(fmt_tree& t, const void* x, const void* y, const void* z,
                                                   const void* f, int m, int dtype, hipStream_t s) {
  Forest& S = *t.forest;
  const ProblemInfo& P = S.probs[t.problem];
  const uint32_t N = (uint32_t)P.n, off = P.prm.offset;
  const int p = S.p;
  const uint32_t L = (uint32_t)S.L;
  const uint32_t M = (uint32_t)t.nodes.size();
  std::vector<uint32_t> hl(M), hp(M), hb(M), hc(M);
  for (uint32_t j = 0; j < M; ++j) {
    const uint32_t i = t.nodes[j];
    hl[j] = S.h_level[i];
    hp[j] = S.h_prefix[i];
    hb[j] = S.h_begin[i] - off;
    hc[j] = S.h_count[i];
  }
  ProblemParams prm = P.prm;
  prm.offset = 0;

  // one allocation for every field's tree: m node tables, then m point
  // arrays, at fixed strides (the kernels address field j by them)
  const uint32_t cap = std::max<uint32_t>(M, 1);
  const size_t NB = Forest::node_bytes(cap, (int)L), PB = Forest::al256(Forest::point_bytes(N));
  auto blk = std::make_shared<DevBuf>((NB + PB) * (size_t)m);
  char* base = blk->as<char>();
  std::vector<std::shared_ptr<Forest>> outs(m);
  for (int j = 0; j < m; ++j) {
    auto F = std::make_shared<Forest>();
    F->p = p;
    F->L = (int)L;
    F->D = S.D;
    F->path = FMT_PATH_FP64;
    F->dtype = dtype;
    F->refine = S.refine;
    F->gram = FMT_GRAM_MOMENTS_LEVEL;
    F->nprob = 1;
    F->stream = s;
    F->device = S.device;
    F->ntot = N;
    F->probs.resize(1);
    F->probs[0].prm = prm;
    F->probs[0].root = 0;
    F->probs[0].n = P.n;
    F->shared = blk;
    F->place_nodes(base + NB * j, cap);
    F->place_points(base + NB * m + PB * j, N);
    outs[j] = F;
  }
  Forest& F0 = *outs[0];
  build_single_nodes(F0, hl, hp, hb, hc, nullptr, prm, s);
  const uint32_t kmask = 3 * S.D >= 32 ? 0xffffffffu : ((1u << (3 * S.D)) - 1u);
  HIPCHK(launch_slice_points(S.skey.as<uint32_t>(), S.order.as<uint32_t>(), off, N, kmask, F0.skey.as<uint32_t>(),
                             F0.order.as<uint32_t>(), s));
  // the other trees: the node set's arrays, keys and permutation replicated
  HIPCHK(launch_replicate(base, F0.topo_bytes, base + NB, NB, m - 1, s));
  HIPCHK(launch_replicate(F0.skey.p, (size_t)((char*)F0.resid.p - (char*)F0.skey.p), (char*)F0.skey.p + PB, PB,
                          m - 1, s));
  for (int j = 1; j < m; ++j) {
    Forest& F = *outs[j];
    F.nodes = M;
    F.level_start = F0.level_start;
    F.level_count = F0.level_count;
    F.depth_present = F0.depth_present;
    F.topo_bytes = F0.topo_bytes;
  }

  // per level: first node, nodes, points and chunk offsets (concatenated)
  const size_t nlev = F0.level_start.size();
  std::vector<uint32_t> choff, cbase(nlev), nchk(nlev), lpts(nlev), lsmall(nlev, 0);
  uint32_t max_chunks = 1, max_nodes = 1;
  for (size_t d = 0; d < nlev; ++d) {
    cbase[d] = (uint32_t)choff.size();
    uint32_t run = 0, pts = 0;
    for (uint32_t k = F0.level_start[d]; k < F0.level_start[d] + F0.level_count[d]; ++k) {
      choff.push_back(run);
      run += (hc[k] + CHUNK - 1) / CHUNK;
      pts += hc[k];
      lsmall[d] += hc[k] < SMALL_NODE ? 1u : 0u;
    }
    choff.push_back(run);
    nchk[d] = run;
    lpts[d] = pts;
    max_chunks = std::max(max_chunks, run);
    max_nodes = std::max(max_nodes, F0.level_count[d]);
  }
  F0.level_points = lpts;

  // The power moments of the levels a moment pyramid covers come from one
  // built as the fit builds it (depth kp from the point count), and every
  // node of those levels is factored in one launch before the level loop;
  // deeper levels form M and factor per level.  All factors stay for the
  // loop when they fit a bound (else everything goes per level).
  int kp = 0;
  while (kp < std::min(S.D, 5) && (uint64_t)N >= ((uint64_t)L << (3 * (kp + 1)))) ++kp;
  const size_t fw = factor_doubles(p);
  const uint32_t NMB = (uint32_t)moment_base_doubles(p);
  PyramidShape pshape;
  uint32_t m_pyr = 0;   // nodes at levels <= kp (the first ones: level order)
  for (size_t d = 0; d < nlev && (int)d <= kp; ++d) m_pyr += F0.level_count[d];
  if (kp > 0) {
    pshape.K = 1;
    pshape.npyr = 1;
    pshape.kp_max = kp;
    pshape.base_cells = 1ull << (3 * kp);
    pshape.pyr_cells = level_first(kp + 1);
    pshape.chunk_bound = N / CHUNK + pshape.base_cells;
    for (int d = 0; d < kp; ++d) {
      pshape.list_off.push_back((uint32_t)(PYR_TAB_WORDS + 3 + d));
      pshape.list_n.push_back(1u);
    }
  }
  const bool whole = kp > 0 && 8ull * fw * M <= (1ull << 30) &&
                     8ull * NMB * (pshape.pyr_cells + pshape.chunk_bound) <= (2ull << 30);
  // device tables in one staged copy: chunk offsets | pyramid table |
  // pyramid entries of the nodes factored ahead | problem parameters
  std::vector<uint32_t> tab;
  if (whole) {
    tab = {0u, (uint32_t)kp, 0u, 0u, 0u, (uint32_t)pshape.base_cells, 0u};
    for (int d = 0; d < kp; ++d) tab.push_back(0u);
  }
  auto al256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t o_tab = al256(4ull * choff.size()), o_list = o_tab + al256(4ull * tab.size());
  const size_t o_prm = o_list + al256(4ull * (whole ? m_pyr : 0)), n_small = o_prm + sizeof(ProblemParams);

  Workspace& W = workspace_for(s);
  std::lock_guard<std::mutex> wlock(W.mu);
  const size_t esz = dtype == FMT_F32 ? 4 : 8;
  for (DevBuf* b : {&W.px, &W.py, &W.pz}) b->reserve(esz * N);
  W.partial.reserve(8ull * NMB * max_chunks);
  W.part_b.reserve(8ull * L * max_chunks * (size_t)m);
  W.fac.reserve(8ull * fw * (whole ? M : max_nodes));
  W.small.reserve(n_small);
  W.status.reserve(64);
  if (whole) reserve_pyramid(W, p, pshape);
  char* stg = W.staging(n_small);
  std::memcpy(stg, choff.data(), 4ull * choff.size());
  if (whole) {
    std::memcpy(stg + o_tab, tab.data(), 4ull * tab.size());
    uint32_t* lst = reinterpret_cast<uint32_t*>(stg + o_list);
    for (uint32_t j = 0; j < m_pyr; ++j) lst[j] = level_first((int)hl[j]) + hp[j];
  }
  std::memcpy(stg + o_prm, &prm, sizeof(ProblemParams));
  HIPCHK(hipMemcpyAsync(W.small.p, stg, n_small, hipMemcpyHostToDevice, s));
  const uint32_t* d_choff = W.small.as<uint32_t>();
  HIPCHK(hipMemsetAsync(W.status.p, 0, 64, s));
  {
    ProfScope ps(KN_XGATHER, (double)N * (1 + m), s);
    HIPCHK(launch_refit_gather(dtype, S.order.as<uint32_t>(), S.skey.as<uint32_t>(), off, N, x, y, z, P.prm, S.D,
                               W.px.p, W.py.p, W.pz.p, W.status.as<uint32_t>(), s));
    HIPCHK(launch_gather_fields(dtype, S.order.as<uint32_t>(), off, N, f, m, N, F0.resid.as<double>(), PB / 8, s));
  }
  if (whole) {
    HIPCHK(hipMemsetAsync(W.pyr_begin.p, 0, 8ull * pshape.base_cells, s));   // begin and count
    build_pyramid(W, p, S.D, dtype, pshape, reinterpret_cast<const uint32_t*>(W.small.as<char>() + o_tab),
                  reinterpret_cast<const ProblemParams*>(W.small.as<char>() + o_prm), F0.skey.as<uint32_t>(), N,
                  F0.resid.as<double>(), s);
    ProfScope ps(KN_XFACTOR, m_pyr, s);
    HIPCHK(launch_factor_cells(p, W.pyr.as<double>(), reinterpret_cast<const uint32_t*>(W.small.as<char>() + o_list),
                               m_pyr, S.refine > 0 ? 1 : 0, W.fac.as<double>(), F0.nb_flags.as<uint32_t>(), s));
  }

  for (size_t d = 0; d < nlev; ++d) {
    LevelArgs a{};
    a.nt = F0.table();
    a.node0 = F0.level_start[d];
    a.nnodes = F0.level_count[d];
    a.chunk_off = d_choff + cbase[d];
    a.nchunks = nchk[d];
    a.px = W.px.p;
    a.py = W.py.p;
    a.pz = W.pz.p;
    a.r = F0.resid.as<double>();
    a.skey = F0.skey.as<uint32_t>();
    a.level = (int)d;
    // no octant statistics: the node set is fixed
    a.D = (int)d;
    a.tol = 0.0;
    // float64 moments: refinement where the conditioning estimate asks for it
    a.refine = S.refine > 0 ? 1 : 0;
    a.pyr_tab = nullptr;
    const bool multi = a.nchunks > a.nnodes;
    // this level's factors (level-local node k at fac + k * fw)
    double* fac = W.fac.as<double>() + (whole ? (size_t)a.node0 * fw : 0);
    if (!whole || (int)d > kp) {
      {
        ProfScope ps(KN_XMOM, lpts[d], s);
        HIPCHK(launch_moments(p, 3, dtype, a, W.partial.as<double>(), s));
        if (multi) HIPCHK(launch_chunk_reduce(a, W.partial.as<double>(), NMB, s));
      }
      ProfScope ps(KN_XFACTOR, a.nnodes, s);
      HIPCHK(launch_factor_moments(p, a, W.partial.as<double>(), fac, s));
    }
    // all fields in each launch (grid rows)
    a.nfields = (uint32_t)m;
    a.rstride = PB / 8;
    a.cstride = NB / 8;
    {
      ProfScope ps(KN_XBMOM, (double)lpts[d] * m, s);
      launch_bmoments(p, dtype, a, lsmall[d], W.part_b.as<double>(), s);
      if (multi) HIPCHK(launch_chunk_reduce(a, W.part_b.as<double>(), L, s));
    }
    {
      ProfScope ps(KN_XSOLVE, (double)a.nnodes * m, s);
      HIPCHK(launch_factor_solve(p, a, W.part_b.as<double>(), fac, s));
    }
    for (int it = 0; it < S.refine; ++it) {
      {
        ProfScope ps(KN_RSWEEP, (double)lpts[d] * m, s);
        HIPCHK(launch_moments(p, 1, dtype, a, W.part_b.as<double>(), s));
      }
      ProfScope ps(KN_RSOLVE, (double)a.nnodes * m, s);
      HIPCHK(launch_refine_solve(p, a, W.part_b.as<double>(), fac, s));
    }
    {
      ProfScope ps(KN_XRESID, (double)lpts[d] * m, s);
      HIPCHK(launch_residual_fields(p, dtype, a, s));
    }
  }
  // the rank and refinement flags belong to the node set: every field's tree
  // gets the same ones, then its own non-finite marks
  for (int j = 1; j < m; ++j) outs[j]->level_points = lpts;
  HIPCHK(launch_replicate(F0.nb_flags.p, 4ull * M, (char*)F0.nb_flags.p + NB, NB, m - 1, s));
  for (int j = 0; j < m; ++j) HIPCHK(launch_check_coef(p, outs[j]->table(), M, W.status.as<uint32_t>(), s));
  HIPCHK(hipMemcpyAsync(W.host_counters + 4, W.status.p, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const uint32_t st = W.host_counters[4];
  if (st & STATUS_MISMATCH) fail(FMT_E_INVALID_ARG, "the points differ from the points the tree was fitted on");
  if (st & STATUS_NONFINITE) fail(FMT_E_NUMERIC, "a non-finite coefficient was produced");
  return outs;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void fmt_default_opts(fmt_fit_opts* o) {
  if (!o) return;
  o->p = 4;
  o->tol = 1e-8;
  o->max_depth = 6;
  o->path = FMT_PATH_FP64;
  o->refine_steps = 1;
  for (int a = 0; a < 3; ++a) {
    o->box_lo[a] = 0.0;
    o->box_hi[a] = 1.0;
  }
  o->gram = FMT_GRAM_MOMENTS;
}

const char* fmt_last_error(void) { return g_last_error.c_str(); }

const char* fmt_version(void) { return "fmt-mi355x 0.1 (gfx950)"; }

fmt_status fmt_fit(const fmt_fit_opts* opts, const void* x, const void* y, const void* z, const void* f, int64_t n,
                   int dtype, void* stream, fmt_tree** out) {
  if (out) *out = nullptr;
  return guard([&] {
    if (!opts || !out) fail(FMT_E_INVALID_ARG, "NULL opts or out");
    if (dtype != FMT_F32 && dtype != FMT_F64) fail(FMT_E_INVALID_ARG, "dtype must be FMT_F32 or FMT_F64");
    validate_opts(*opts);
    if (n < 0) fail(FMT_E_INVALID_ARG, "negative n");
    std::vector<fmt_fit_opts> per(1, *opts);
    std::vector<FitInput> in(1, FitInput{x, y, z, f, n});
    auto F = fit_group(*opts, per, in, dtype, (hipStream_t)stream);
    fmt_tree* t = new fmt_tree();
    t->forest = F;
    t->problem = 0;
    *out = t;
  });
}

fmt_status fmt_fit_batch(const fmt_fit_opts* opts, const void* const* x, const void* const* y, const void* const* z,
                         const void* const* f, const int64_t* n, int count, int dtype, void* stream,
                         fmt_tree** out) {
  return guard([&] {
    if (!opts || !x || !y || !z || !f || !n || !out) fail(FMT_E_INVALID_ARG, "NULL argument");
    if (count <= 0) fail(FMT_E_INVALID_ARG, "count must be positive");
    if (dtype != FMT_F32 && dtype != FMT_F64) fail(FMT_E_INVALID_ARG, "dtype must be FMT_F32 or FMT_F64");
    for (int k = 0; k < count; ++k) {
      out[k] = nullptr;
      validate_opts(opts[k]);
      if (n[k] < 0) fail(FMT_E_INVALID_ARG, "negative n");
    }
    // group by (p, path, max_depth, refine_steps, tol)
    std::map<std::tuple<int, int, int, int, double, int>, std::vector<int>> groups;
    for (int k = 0; k < count; ++k)
      groups[std::make_tuple(opts[k].p, opts[k].path, opts[k].max_depth, opts[k].refine_steps, opts[k].tol,
                             opts[k].gram)]
          .push_back(k);
    std::vector<std::vector<int>> glist;
    for (auto& kv : groups) glist.push_back(std::move(kv.second));
    std::vector<std::shared_ptr<Forest>> forests(glist.size());
    auto run_group = [&](size_t g, hipStream_t s) {
      const std::vector<int>& ids = glist[g];
      std::vector<fmt_fit_opts> per;
      std::vector<FitInput> in;
      for (int k : ids) {
        per.push_back(opts[k]);
        in.push_back(FitInput{x[k], y[k], z[k], f[k], n[k]});
      }
      forests[g] = fit_group(per[0], per, in, dtype, s);
    };
    if (glist.size() == 1) {
      run_group(0, (hipStream_t)stream);
    } else {
      // Groups (problems of different order, path, depth or tolerance) run
      // concurrently: up to kGroupStreams host threads, each driving its
      // groups' level loops on a stream of its own, so that their launches
      // and level boundaries overlap on the device.  Those streams first
      // wait for the caller's stream (the inputs); every group's fit ends
      // with its stream drained, so the trees are complete on return.
      const int nw = (int)std::min<size_t>(glist.size(), (size_t)kGroupStreams);
      hipEvent_t ready = nullptr;
      HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
      hipError_t er = hipEventRecord(ready, (hipStream_t)stream);
      std::vector<hipStream_t> ws(nw);
      for (int w = 0; w < nw && er == hipSuccess; ++w) {
        ws[w] = group_stream(w);
        er = hipStreamWaitEvent(ws[w], ready, 0);
      }
      (void)hipEventDestroy(ready);
      hip_check(er, "batch group streams");
      int dev = 0;
      HIPCHK(hipGetDevice(&dev));
      std::vector<std::exception_ptr> errs(nw);
      std::vector<std::thread> th;
      for (int w = 0; w < nw; ++w)
        th.emplace_back([&, w] {
          try {
            hip_check(hipSetDevice(dev), "hipSetDevice");   // a new thread starts on device 0
            for (size_t g = (size_t)w; g < glist.size(); g += (size_t)nw) run_group(g, ws[w]);
          } catch (...) {
            errs[w] = std::current_exception();
          }
        });
      for (auto& t : th) t.join();
      for (auto& e : errs)
        if (e) std::rethrow_exception(e);
    }
    std::vector<fmt_tree*> made(count, nullptr);
    try {
      for (size_t g = 0; g < glist.size(); ++g) {
        const std::vector<int>& ids = glist[g];
        for (size_t j = 0; j < ids.size(); ++j) {
          fmt_tree* t = new fmt_tree();
          t->forest = forests[g];
          t->problem = (int)j;
          made[ids[j]] = t;
        }
      }
    } catch (...) {
      for (auto* t : made) delete t;
      throw;
    }
    for (int k = 0; k < count; ++k) out[k] = made[k];
  });
}

// Composite coefficients of a forest, built once on the first evaluation;
// every evaluating stream waits for their completion.
static void ensure_composed(Forest& F, int problem, hipStream_t s) {
  std::lock_guard<std::mutex> g(F.compose_mu);
  if (F.nodes >= (1u << 28)) fail(FMT_E_INVALID_ARG, "too many nodes for evaluation (2^28 at most)");
  if (F.cell_tab.size() != F.probs.size()) {
    F.cell_tab.resize(F.probs.size());
    F.cell_T.assign(F.probs.size(), -1);
    F.cell_ev.assign(F.probs.size(), nullptr);
  }
  if (!F.cell_ev[problem]) {
    // 8^T entries: T <= 6 for one tree (1 MiB), <= 4 per tree of a batch
    const int T = std::min(F.depth_present, F.probs.size() == 1 ? 6 : 4);
    // [frame table | cells]; the frames use the problem's box, the same
    // scale as the fit's node frames
    DevBuf& b = F.cell_tab[problem];
    const size_t cell_bytes = 1024 + (sizeof(uint32_t) << (3 * T));
    if (F.probs.size() == 1 && !F.composed && !F.nb_ccoef.p) {
      // one allocation for the tree's cell table and composite coefficients
      const size_t cb = (cell_bytes + 255) & ~(size_t)255;
      const size_t ccb = sizeof(double) * (size_t)ccoef_stride(F.L) * std::max<uint32_t>(F.nodes, 1);
      F.eval_mem.alloc(cb + ccb);
      b = DevBuf::view(F.eval_mem.p, 0, cell_bytes);
      F.nb_ccoef = DevBuf::view(F.eval_mem.p, cb, ccb);
    } else {
      b.alloc(cell_bytes);
    }
    HIPCHK(launch_cell_table(F.table(), F.probs[problem].root, T, F.probs[problem].prm, b.as<double>(),
                             (uint32_t*)(b.as<char>() + 1024), s));
    hipEvent_t ev = nullptr;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev, s));
    F.cell_T[problem] = T;
    F.cell_ev[problem] = ev;
  }
  HIPCHK(hipStreamWaitEvent(s, F.cell_ev[problem], 0));
  if (!F.composed) {
    if (!F.nb_ccoef.p) F.nb_ccoef.alloc(sizeof(double) * (size_t)ccoef_stride(F.L) * std::max<uint32_t>(F.nodes, 1));
    {
      ProfScope ps(KN_COMPOSE, F.nodes, s);
      HIPCHK(launch_compose(F.p, F.table(), 0, F.nodes, F.nb_ccoef.as<double>(), s));
    }
    hipEvent_t ev = nullptr;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev, s));
    F.composed = ev;
  }
  HIPCHK(hipStreamWaitEvent(s, F.composed, 0));
}

}  // extern "C"

// Scratch of fmt_eval_noalloc: one array per device, held until the process
// ends.  Host code never uses this name as an address: the device address
// comes from hipGetSymbolAddress (noalloc_scratch) once per device.
static __device__ __align__(256) unsigned char scratch[FMT_EVAL_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the
// device's first call, with that device current).
void* noalloc_scratch() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(FMT_E_INVALID_ARG, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(FMT_E_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_dev[dev] = ptr;
  }
  return g_scratch_dev[dev];
}

// Bytes of device scratch the sorted evaluation of n queries uses: the
// coordinates twice (sort passes alternate), keys and positions twice, the
// sort's histograms.
size_t sorted_eval_bytes(uint32_t n, size_t esz) {
  const size_t pbytes = (esz * n + 255) & ~(size_t)255;
  return 6 * pbytes + 16ull * n + 4 * radix_sort_scratch_words(n) + 256;
}

// fmt_eval and fmt_eval_noalloc.  With `fixed` null the sorted mode takes
// its scratch from hipMallocAsync and the tree's evaluation tables are built
// on first use; with `fixed` (the no-alloc entry point) the scratch is that
// array and the tables must exist already.
void eval_tree(const fmt_tree* tree, const void* qx, const void* qy, const void* qz, int64_t nq, int dtype,
               double* out, int sort_queries, hipStream_t s, void* fixed) {
  if (!tree) fail(FMT_E_INVALID_ARG, "NULL tree");
  if (dtype != FMT_F32 && dtype != FMT_F64) fail(FMT_E_INVALID_ARG, "dtype must be FMT_F32 or FMT_F64");
  if (nq < 0 || nq >= (1ll << 31)) fail(FMT_E_INVALID_ARG, "nq out of range");
  if (nq == 0) return;
  if (!qx || !qy || !qz || !out) fail(FMT_E_INVALID_ARG, "NULL query or output pointer");
  Forest& F = *tree->forest;
  if (fixed) {
    // no allocation here: the composite coefficients and the cell table
    // must have been built by an earlier fmt_eval of this tree
    std::lock_guard<std::mutex> g(F.compose_mu);
    if (!F.composed || F.cell_ev.size() != F.probs.size() || !F.cell_ev[tree->problem])
      fail(FMT_E_INVALID_ARG, "the tree's evaluation tables are not built: evaluate it once with fmt_eval first");
    // wait for the tables only while they are still being built (a stream
    // under graph capture may not wait on an event recorded outside it)
    if (hipEventQuery(F.cell_ev[tree->problem]) != hipSuccess)
      HIPCHK(hipStreamWaitEvent(s, F.cell_ev[tree->problem], 0));
    if (hipEventQuery(F.composed) != hipSuccess) HIPCHK(hipStreamWaitEvent(s, F.composed, 0));
  } else {
    ensure_composed(F, tree->problem, s);
  }
  EvalTree t;
  t.nt = F.table();
  t.root = F.probs[tree->problem].root;
  // query cells at the deepest level present: the same top bits as cells at
  // max_depth (the scale differs by an exact power of two)
  t.D = F.depth_present;
  t.T = F.cell_T[tree->problem];
  t.lvl = F.cell_tab[tree->problem].as<double>();
  t.cells = (const uint32_t*)(F.cell_tab[tree->problem].as<char>() + 1024);
  t.prm = F.probs[tree->problem].prm;
  for (int a = 0; a < 3; ++a) t.prm.qscale[a] = std::ldexp(t.prm.qscale[a], t.D - F.D);
  const double* cc = F.nb_ccoef.as<double>();
  const uint32_t n = (uint32_t)nq;
  // Sorting makes the coefficient reads of a wave uniform; without it every
  // lane reads its own node's row.  That is cheaper while the coefficient
  // table stays cache-resident, so sort by default only for large tables.
  const size_t coef_bytes = sizeof(double) * (size_t)F.L * F.nodes;
  const bool sort = t.D > 0 && (sort_queries > 0 || (sort_queries < 0 && n >= (1u << 16) &&
                                                     coef_bytes > (64ull << 20)));
  if (!sort) {
    if (fixed) {
      HIPCHK(launch_eval(F.p, dtype, t, cc, qx, qy, qz, nullptr, nullptr, n, out, s));
      return;
    }
    ProfScope ps(KN_EVAL, n, s);
    HIPCHK(launch_eval(F.p, dtype, t, cc, qx, qy, qz, nullptr, nullptr, n, out, s));
    return;
  }
  const size_t esz = dtype == FMT_F32 ? 4 : 8;
  const size_t pbytes = (esz * n + 255) & ~(size_t)255;
  const size_t bytes = sorted_eval_bytes(n, esz);
  if (fixed && bytes > (size_t)FMT_EVAL_NOALLOC_SCRATCH_BYTES)
    fail(FMT_E_INVALID_ARG, "nq needs more scratch than FMT_EVAL_NOALLOC_SCRATCH_BYTES in sorted mode");
  char* base = nullptr;
  if (fixed) base = (char*)fixed;
  else HIPCHK(hipMallocAsync((void**)&base, bytes, s));
  void* pay[3];
  void* pay_alt[3];
  for (int q = 0; q < 3; ++q) {
    pay[q] = base + q * pbytes;
    pay_alt[q] = base + (3 + q) * pbytes;
  }
  uint32_t* k0 = (uint32_t*)(base + 6 * pbytes);
  uint32_t* v0 = k0 + n;
  uint32_t* k1 = v0 + n;
  uint32_t* v1 = k1 + n;
  uint32_t* scr = v1 + n;
  const void* pin[3] = {qx, qy, qz};
  hipError_t e;
  bool in_alt = false;
  if (fixed) {
    // the same launches without the profiling events
    e = launch_query_keys(dtype, qx, qy, qz, n, t.prm, t.D, k0, s);
    if (e == hipSuccess) e = radix_sort_payload(dtype, 3, k0, v0, k1, v1, pin, pay, pay_alt, n, 3 * t.D, scr, s, &in_alt);
    void* const* sq = in_alt ? pay_alt : pay;
    if (e == hipSuccess)
      e = launch_eval(F.p, dtype, t, cc, sq[0], sq[1], sq[2], in_alt ? v1 : v0, in_alt ? k1 : k0, n, out, s);
    hip_check(e, "eval");
    return;
  }
  {
    ProfScope ps(KN_EKEYS, n, s);
    e = launch_query_keys(dtype, qx, qy, qz, n, t.prm, t.D, k0, s);
  }
  {
    // keys with the query coordinates and positions as payload
    ProfScope ps(KN_ESORT, n, s);
    if (e == hipSuccess)
      e = radix_sort_payload(dtype, 3, k0, v0, k1, v1, pin, pay, pay_alt, n, 3 * t.D, scr, s, &in_alt);
  }
  uint32_t* ks = in_alt ? k1 : k0;
  uint32_t* vs = in_alt ? v1 : v0;
  void* const* sq = in_alt ? pay_alt : pay;
  {
    ProfScope ps(KN_EVAL, n, s);
    if (e == hipSuccess) e = launch_eval(F.p, dtype, t, cc, sq[0], sq[1], sq[2], vs, ks, n, out, s);
  }
  hipError_t e2 = hipFreeAsync(base, s);
  hip_check(e, "eval");
  hip_check(e2, "hipFreeAsync");
}

}  // namespace

extern "C" {

fmt_status fmt_eval(const fmt_tree* tree, const void* qx, const void* qy, const void* qz, int64_t nq, int dtype,
                    double* out, int sort_queries, void* stream) {
  return guard([&] { eval_tree(tree, qx, qy, qz, nq, dtype, out, sort_queries, (hipStream_t)stream, nullptr); });
}

fmt_status fmt_eval_noalloc(const fmt_tree* tree, const void* qx, const void* qy, const void* qz, int64_t nq,
                            int dtype, double* out, int sort_queries, void* stream) {
  return guard([&] {
    void* base = noalloc_scratch();
    eval_tree(tree, qx, qy, qz, nq, dtype, out, sort_queries, (hipStream_t)stream, base);
  });
}

fmt_status fmt_rbf_factored(int p, double eps, const void* x, const void* y, const void* z, int64_t n,
                            const void* xq, const void* yq, const void* zq, int64_t nq, int dtype, double* out,
                            void* stream) {
  return guard([&] {
    if (p < 0 || p > FMT_MAX_P) fail(FMT_E_INVALID_ARG, "p out of range 0..14");
    if (!(eps >= 0.0) || std::isinf(eps)) fail(FMT_E_INVALID_ARG, "eps must be finite and >= 0");
    if (dtype != FMT_F32 && dtype != FMT_F64) fail(FMT_E_INVALID_ARG, "dtype must be FMT_F32 or FMT_F64");
    if (n < 0 || nq < 0 || n >= (1ll << 31) || nq >= (1ll << 22)) fail(FMT_E_INVALID_ARG, "n or nq out of range");
    if (n == 0 || nq == 0) return;
    if (!x || !y || !z || !xq || !yq || !zq || !out) fail(FMT_E_INVALID_ARG, "NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    const int L = basis_size(p);
    const uint32_t LS = (uint32_t)((L + 31) / 32 * 32);
    // Hermite numbers H_m(0) of the physicists' polynomials, from their
    // recurrence at t = 0: H_0 = 1, H_1 = 0, H_{m+1}(0) = -2 m H_{m-1}(0)
    std::vector<double> h(2 * p + 1, 0.0);
    h[0] = 1.0;
    for (int m = 1; m + 1 <= 2 * p; ++m) h[m + 1] = -2.0 * m * h[m - 1];
    // exponents in graded order, then C = E T E with
    // T_ab = (-1)^|a| H_{a1+b1}(0) H_{a2+b2}(0) H_{a3+b3}(0), E = diag(eps^|a|)
    std::vector<uint32_t> expo;
    std::vector<int> ex[3];
    for (int k = 0; k <= p; ++k)
      for (int l = k; l >= 0; --l)
        for (int m = k - l; m >= 0; --m) {
          const int nn = k - l - m;
          expo.push_back((uint32_t)l | ((uint32_t)m << 8) | ((uint32_t)nn << 16));
          ex[0].push_back(l);
          ex[1].push_back(m);
          ex[2].push_back(nn);
        }
    std::vector<double> epow(2 * p + 1, 1.0);
    for (int k = 1; k <= 2 * p; ++k) epow[k] = epow[k - 1] * eps;
    const size_t c_bytes = 8ull * L * LS, e_bytes = 4ull * L;
    const size_t b_bytes = 8ull * (size_t)n * LS, q_bytes = 8ull * (size_t)nq * LS;
    std::vector<char> host(c_bytes + e_bytes, 0);
    double* C = reinterpret_cast<double*>(host.data());
    for (int a = 0; a < L; ++a) {
      const int da = ex[0][a] + ex[1][a] + ex[2][a];
      for (int b = 0; b < L; ++b) {
        const int db = ex[0][b] + ex[1][b] + ex[2][b];
        const double t = h[ex[0][a] + ex[0][b]] * h[ex[1][a] + ex[1][b]] * h[ex[2][a] + ex[2][b]];
        C[(size_t)a * LS + b] = (da & 1 ? -t : t) * epow[da] * epow[db];
      }
    }
    std::memcpy(host.data() + c_bytes, expo.data(), e_bytes);
    // device layout: [C | exponents (padded to 256 bytes) | B | basis of the
    // points | basis of the queries]
    const size_t e_pad = (e_bytes + 255) & ~(size_t)255;
    char* base = nullptr;
    HIPCHK(hipMallocAsync((void**)&base, c_bytes + e_pad + 2 * b_bytes + q_bytes, s));
    double* dC = reinterpret_cast<double*>(base);
    uint32_t* dE = reinterpret_cast<uint32_t*>(base + c_bytes);
    double* dB = reinterpret_cast<double*>(base + c_bytes + e_pad);
    double* dAx = reinterpret_cast<double*>(base + c_bytes + e_pad + b_bytes);
    double* dAq = reinterpret_cast<double*>(base + c_bytes + e_pad + 2 * b_bytes);
    hipError_t e = hipMemcpyAsync(base, host.data(), c_bytes + e_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host image goes out of scope
    // B's padding columns are read (as zeros) by the second product
    if (e == hipSuccess) e = hipMemsetAsync(dB, 0, b_bytes, s);
    if (e == hipSuccess) {
      ProfScope ps(KN_RBF_ROWS, (double)n, s);
      e = launch_rbf_basis(dtype, x, y, z, (uint32_t)n, dE, L, LS, dAx, s);
      if (e == hipSuccess) e = launch_rbf_basis(dtype, xq, yq, zq, (uint32_t)nq, dE, L, LS, dAq, s);
      if (e == hipSuccess) e = launch_rbf_gemm(dAx, (uint32_t)n, dC, (uint32_t)L, LS, dB, LS, s);
    }
    if (e == hipSuccess) {
      ProfScope ps(KN_RBF_PAIRS, (double)n * (double)nq, s);
      e = launch_rbf_gemm(dAq, (uint32_t)nq, dB, (uint32_t)n, LS, out, (uint64_t)n, s);
    }
    hipError_t e2 = hipFreeAsync(base, s);
    hip_check(e, "rbf");
    hip_check(e2, "hipFreeAsync");
  });
}

fmt_status fmt_tree_wait(const fmt_tree* tree) {
  return guard([&] {
    if (!tree) fail(FMT_E_INVALID_ARG, "NULL tree");
    HIPCHK(hipStreamSynchronize(tree->forest->stream));
    HIPCHK(hipDeviceSynchronize());
    const uint32_t st = tree->forest->device_status;
    if (st & STATUS_DOMAIN) fail(FMT_E_DOMAIN, "a point is NaN or outside the box");
    if (st & STATUS_NONFINITE) fail(FMT_E_NUMERIC, "a non-finite coefficient was produced");
  });
}

fmt_status fmt_tree_get_info(const fmt_tree* tree, fmt_tree_info* info) {
  return guard([&] {
    if (!tree || !info) fail(FMT_E_INVALID_ARG, "NULL argument");
    fmt_tree* t = const_cast<fmt_tree*>(tree);
    ensure_tree_nodes(t);
    Forest& F = *t->forest;
    std::memset(info, 0, sizeof(*info));
    info->nodes = (int64_t)t->nodes.size();
    info->n_points = F.probs[t->problem].n;
    info->p = F.p;
    info->L = F.L;
    info->max_depth = F.D;
    info->path = F.path;
    int depth = 0, rd = 0;
    for (uint32_t i : t->nodes) {
      const int lv = (int)F.h_level[i];
      info->per_level[lv] += 1;
      depth = std::max(depth, lv);
      if (F.h_flags[i] & FLAG_DEFLATED) ++rd;
    }
    info->depth = depth;
    info->rank_deficient_nodes = rd;
    info->device_bytes = (int64_t)F.device_bytes();
  });
}

fmt_status fmt_tree_export_nodes(const fmt_tree* tree, uint8_t* level, uint32_t* prefix, uint32_t* begin,
                                 uint32_t* count, uint32_t* flags, double* coeffs) {
  return guard([&] {
    if (!tree) fail(FMT_E_INVALID_ARG, "NULL tree");
    fmt_tree* t = const_cast<fmt_tree*>(tree);
    ensure_tree_nodes(t);
    Forest& F = *t->forest;
    const uint32_t off = F.probs[t->problem].prm.offset;
    for (size_t j = 0; j < t->nodes.size(); ++j) {
      const uint32_t i = t->nodes[j];
      if (level) level[j] = (uint8_t)F.h_level[i];
      if (prefix) prefix[j] = F.h_prefix[i];
      if (begin) begin[j] = F.h_begin[i] - off;
      if (count) count[j] = F.h_count[i];
      if (flags) flags[j] = F.h_flags[i];
      if (coeffs) std::memcpy(coeffs + j * F.L, F.h_coef.data() + (size_t)i * F.L, sizeof(double) * F.L);
    }
  });
}

fmt_status fmt_tree_export_points(const fmt_tree* tree, uint32_t* keys, uint32_t* order, uint32_t* leaf,
                                  double* residual) {
  return guard([&] {
    if (!tree) fail(FMT_E_INVALID_ARG, "NULL tree");
    fmt_tree* t = const_cast<fmt_tree*>(tree);
    ensure_tree_nodes(t);
    Forest& F = *t->forest;
    const ProblemInfo& P = F.probs[t->problem];
    const uint32_t n = (uint32_t)P.n, off = P.prm.offset;
    if (n == 0) return;
    std::vector<uint32_t> sk(n), so(n);
    std::vector<double> sr(n);
    HIPCHK(hipStreamSynchronize(F.stream));
    HIPCHK(hipMemcpy(sk.data(), F.skey.as<uint32_t>() + off, 4ull * n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(so.data(), F.order.as<uint32_t>() + off, 4ull * n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(sr.data(), F.resid.as<double>() + off, 8ull * n, hipMemcpyDeviceToHost));
    const uint32_t kmask = 3 * F.D >= 32 ? 0xffffffffu : ((1u << (3 * F.D)) - 1u);
    std::vector<uint32_t> sleaf(n, 0);
    for (size_t j = 0; j < t->nodes.size(); ++j) {   // deeper nodes come later and overwrite
      const uint32_t i = t->nodes[j];
      const uint32_t b = F.h_begin[i] - off, c = F.h_count[i];
      for (uint32_t q = b; q < b + c; ++q) sleaf[q] = (uint32_t)j;
    }
    for (uint32_t q = 0; q < n; ++q) {
      const uint32_t inp = so[q] - off;
      if (keys) keys[inp] = sk[q] & kmask;
      if (order) order[q] = inp;
      if (leaf) leaf[inp] = sleaf[q];
      if (residual) residual[inp] = sr[q];
    }
  });
}

fmt_status fmt_tree_import(const fmt_fit_opts* opts, int64_t nodes, const uint8_t* level, const uint32_t* prefix,
                           const double* coeffs, void* stream, fmt_tree** out) {
  if (out) *out = nullptr;
  return guard([&] {
    if (!opts || !out || !level || !prefix || !coeffs) fail(FMT_E_INVALID_ARG, "NULL argument");
    validate_opts(*opts);
    if (nodes < 1 || nodes >= (1ll << 31)) fail(FMT_E_INVALID_ARG, "node count out of range");
    hipStream_t s = (hipStream_t)stream;
    auto F = std::make_shared<Forest>();
    F->p = opts->p;
    F->L = basis_size(opts->p);
    F->D = opts->max_depth;
    F->path = opts->path;
    F->nprob = 1;
    F->stream = s;
    HIPCHK(hipGetDevice(&F->device));
    const int L = F->L;
    std::vector<int64_t> idx(nodes);
    for (int64_t i = 0; i < nodes; ++i) {
      idx[i] = i;
      if (level[i] > F->D) fail(FMT_E_INVALID_ARG, "node level above max_depth");
      if (level[i] < 10 && (prefix[i] >> (3 * level[i])) != 0) fail(FMT_E_INVALID_ARG, "prefix wider than its level");
    }
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
      return level[a] != level[b] ? level[a] < level[b] : prefix[a] < prefix[b];
    });
    if (level[idx[0]] != 0 || (nodes > 1 && level[idx[1]] == 0)) fail(FMT_E_INVALID_ARG, "exactly one root needed");
    const uint32_t M = (uint32_t)nodes;
    std::vector<uint32_t> hb(M, 0), hc(M, 0), hp(M), hl(M);
    std::vector<double> hcoef((size_t)M * L);
    for (uint32_t j = 0; j < M; ++j) {
      const int64_t i = idx[j];
      hp[j] = prefix[i];
      hl[j] = level[i];
      std::memcpy(hcoef.data() + (size_t)j * L, coeffs + i * L, sizeof(double) * L);
    }
    ProblemParams prm = make_params(*opts, 0, 0);
    build_single_nodes(*F, hl, hp, hb, hc, hcoef.data(), prm, s);
    HIPCHK(hipStreamSynchronize(s));
    F->probs.resize(1);
    F->probs[0].prm = prm;
    F->probs[0].root = 0;
    F->probs[0].n = 0;
    fmt_tree* t = new fmt_tree();
    t->forest = F;
    t->problem = 0;
    *out = t;
  });
}

fmt_status fmt_refit(const fmt_tree* tree, const void* x, const void* y, const void* z, const void* f, int64_t n,
                     int m, int dtype, void* stream, fmt_tree** out) {
  if (out && m > 0 && m <= FMT_REFIT_MAX_FIELDS)
    for (int j = 0; j < m; ++j) out[j] = nullptr;
  return guard([&] {
    if (!tree || !out) fail(FMT_E_INVALID_ARG, "NULL tree or out");
    if (m < 1 || m > FMT_REFIT_MAX_FIELDS) fail(FMT_E_INVALID_ARG, "m out of range 1..FMT_REFIT_MAX_FIELDS");
    if (dtype != FMT_F32 && dtype != FMT_F64) fail(FMT_E_INVALID_ARG, "dtype must be FMT_F32 or FMT_F64");
    if (!x || !y || !z || !f) fail(FMT_E_INVALID_ARG, "NULL input pointer");
    fmt_tree* t = const_cast<fmt_tree*>(tree);
    ensure_tree_nodes(t);
    const ProblemInfo& P = t->forest->probs[t->problem];
    if (P.n == 0) fail(FMT_E_INVALID_ARG, "the tree holds no points (an imported tree)");
    if (t->forest->p > 8) fail(FMT_E_INVALID_ARG, "the fixed-topology refit supports p <= 8");
    if (n != P.n) fail(FMT_E_INVALID_ARG, "n differs from the tree's point count");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (t->forest->device != dev) fail(FMT_E_INVALID_ARG, "the tree lives on another device");
    auto outs = refit_forests(*t, x, y, z, f, m, dtype, (hipStream_t)stream);
    std::vector<fmt_tree*> made;
    try {
      for (int j = 0; j < m; ++j) {
        fmt_tree* h = new fmt_tree();
        h->forest = outs[j];
        h->problem = 0;
        made.push_back(h);
      }
    } catch (...) {
      for (auto* h : made) delete h;
      throw;
    }
    for (int j = 0; j < m; ++j) out[j] = made[j];
  });
}

int fmt_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  const int prev = g_prof_on ? 1 : 0;
  g_prof_on = on != 0;
  return prev;
}

void fmt_profile_reset(void) {
  prof_resolve();
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (auto& a : g_prof_acc) a = ProfAcc();
}

int fmt_profile_read(fmt_kernel_stat* out, int max_entries) {
  prof_resolve();
  std::lock_guard<std::mutex> g(g_prof_mu);
  int n = 0;
  for (int k = 0; k < KN_COUNT && n < max_entries; ++k) {
    if (!out) break;
    std::memset(&out[n], 0, sizeof(fmt_kernel_stat));
    std::snprintf(out[n].name, sizeof(out[n].name), "%s", kKernelNames[k]);
    out[n].launches = g_prof_acc[k].launches;
    out[n].ms = g_prof_acc[k].ms;
    out[n].units = g_prof_acc[k].units;
    ++n;
  }
  return out ? n : KN_COUNT;
}

void fmt_tree_destroy(fmt_tree* tree) {
  if (!tree) return;
  (void)hipStreamSynchronize(tree->forest->stream);
  delete tree;
}

}  // extern "C"
