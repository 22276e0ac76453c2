// Loads of direct-sum sources from a range whose start is the same in every
// lane (device code only; used by the direct-sum kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmm {

// Loads from a range whose start is the same in every lane: uniform_base moves
// the start to scalar registers and load_source reads it plus a 32-bit
// per-lane byte offset, which the load instruction takes as scalar base and
// vector offset (a loop then needs one 32-bit add and compare per element
// instead of 64-bit pointer arithmetic).  The pointer is marked global:
// through the integer round trip a generic pointer would make the loads flat
// ones.
using gchar = __attribute__((address_space(1))) const char;
typedef double d4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double4 load_source(gchar *q) {
    const d4v v = *(__attribute__((address_space(1))) const d4v *)q;
    return make_double4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ gchar *uniform_base(const double4 *base) {
    const uint64_t bu = reinterpret_cast<uint64_t>(base);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)bu);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(bu >> 32));
    return (gchar *)(((uint64_t)hi << 32) | lo);
}

}  // namespace fmm
