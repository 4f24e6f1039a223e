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

constexpr uint32_t STATUS_DOMAIN = 1u;
constexpr uint32_t STATUS_NONFINITE = 2u;

hipError_t launch_keygen(int dtype, const PtrSet* ptrs, const ProblemParams* prm, int nprob, int depth,
                         uint32_t total, uint32_t* keys, uint32_t* status, hipStream_t s);
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
hipError_t launch_gather(int dtype, const PtrSet* ptrs, const ProblemParams* prm, int nprob, const uint32_t* order,
                         uint32_t total, void* px, void* py, void* pz, double* r, hipStream_t s);
hipError_t launch_permute3(int dtype, const void* x, const void* y, const void* z, const uint32_t* order,
                           uint32_t n, void* ox, void* oy, void* oz, hipStream_t s);

}  // namespace fmt
