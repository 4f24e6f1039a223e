// Launchers of the key, sort and gather kernels.
#pragma once

#include "fmt_common.h"

namespace fmt {

struct PtrSet {
  const void* x;
  const void* y;
  const void* z;
  const void* f;
};

// NP payload arrays moved by a sort pass (passed by value to the kernel).
template <typename PT, int NP>
struct PayloadSet {
  PT* a[NP];
};

constexpr uint32_t STATUS_DOMAIN = 1u;
constexpr uint32_t STATUS_NONFINITE = 2u;
constexpr uint32_t STATUS_MISMATCH = 4u;   // a point is not the one the tree recorded

// cat: if cat.x is set, the inputs are also copied there, concatenated in
// global point order (x, y, z, f).
hipError_t launch_keygen(int dtype, const PtrSet* ptrs, const ProblemParams* prm, int nprob, int depth,
                         uint32_t total, uint32_t* keys, uint32_t* status, const PtrSet& cat, hipStream_t s);
hipError_t launch_query_keys(int dtype, const void* qx, const void* qy, const void* qz, uint32_t nq,
                             const ProblemParams& P, int depth, uint32_t* keys, hipStream_t s);
// number of passes radix_sort makes over `bits` key bits (odd counts leave
// the result in the alternate buffers)
int radix_sort_passes(int bits);
// scratch: radix_sort_scratch_words(n) words of device memory
size_t radix_sort_scratch_words(uint32_t n);
// Sorts (keys, vals) by the low `bits` bits of the keys, stably.  The result
// ends in (keys, vals) or in (keys_alt, vals_alt) as *result_in_alt says.
// With vals_are_iota the input values are not read (value = position).
hipError_t radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, uint32_t n, int bits,
                      bool vals_are_iota, uint32_t* scratch, hipStream_t s, bool* result_in_alt);
// radix_sort that also moves np (3 or 4) payload arrays of the given dtype
// (4 or 8 bytes per element): pass 0 reads pin[] and the passes alternate
// between pay_alt[] and pay[]; the sorted payload ends in pay[] when
// *result_in_alt is false (an even number of passes), else in pay_alt[].
// Values start as source positions (not read).
hipError_t radix_sort_payload(int dtype, int np, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                              uint32_t* vals_alt, const void* const* pin, void* const* pay, void* const* pay_alt,
                              uint32_t n, int bits, uint32_t* scratch, hipStream_t s, bool* result_in_alt);
// r[i] = (double)f[i] for i < n, and zero[j] = 0 for j < nzero (a clear of
// small tables folded into the same launch)
hipError_t launch_widen(int dtype, const void* f, uint32_t n, double* r, uint32_t* zero, uint32_t nzero,
                        hipStream_t s);

// The points of one problem of a fitted forest in its key order, for a
// fixed-topology refit: px[i] = x[order[off + i] - off] (likewise y, z) for
// i < n, with the cell key of each gathered point (problem box P, depth
// `depth`) checked against skey[off + i] (its low 3 depth bits); a point
// outside the box, a differing key or a permutation entry out of range sets
// STATUS_MISMATCH.
hipError_t launch_refit_gather(int dtype, const uint32_t* order, const uint32_t* skey, uint32_t off, uint32_t n,
                               const void* x, const void* y, const void* z, const ProblemParams& P, int depth,
                               void* px, void* py, void* pz, uint32_t* status, hipStream_t s);
// m value fields in key order, widened: r[j rstride + i] =
// f[j fstride + order[off + i] - off] for j < m, i < n (entries whose
// permutation value is out of range are left unwritten).
hipError_t launch_gather_fields(int dtype, const uint32_t* order, uint32_t off, uint32_t n, const void* f, int m,
                                uint64_t fstride, double* r, uint64_t rstride, hipStream_t s);
// One problem's keys and permutation as a single-problem forest holds them:
// okey[i] = skey[off + i] & kmask, oorder[i] = order[off + i] - off.
// rows copies of `bytes` bytes (a multiple of 4) from src: row q to dst + q stride.
hipError_t launch_replicate(const void* src, size_t bytes, void* dst, size_t stride, int rows, hipStream_t s);
hipError_t launch_slice_points(const uint32_t* skey, const uint32_t* order, uint32_t off, uint32_t n, uint32_t kmask,
                               uint32_t* okey, uint32_t* oorder, hipStream_t s);

}  // namespace fmt
