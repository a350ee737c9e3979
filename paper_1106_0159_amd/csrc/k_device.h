// Device helpers shared by the Legendre kernels (FP64 and mixed precision).
#pragma once

#include "sht_internal.h"

namespace sht {

// Workgroups are dispatched to the XCDs in turn (workgroup b runs on XCD
// b mod kXcds).  The launchers round the number of m values up to a multiple
// of kMBlock * kXcds, and the k-th workgroup of XCD x takes part k % parts of
// the m value 64 j + 8 x' + r, with (j, r, part) counted out of k (r fastest
// after the part) and x' = x on even j, 7 - x on odd j.  So the parts (slot
// tiles or groups) of one m share one XCD's L2 for its coefficient column,
// the 8 consecutive m whose entries fill one 128-byte line of a Delta row are
// written (read) through the same L2, m still ascends in launch order, and
// the snake order keeps the XCDs' shares of the work equal.
constexpr int kXcds = 8;
constexpr int kMBlock = 8;  // m values per 128-byte line of a Delta row
struct MPart {
    int m, part;
};
__device__ __forceinline__ MPart xcd_m_part(int parts) {
    const int x = blockIdx.x % kXcds, k = blockIdx.x / kXcds;
    const int per = kMBlock * parts;
    const int j = k / per, rem = k - j * per;
    const int xs = (j & 1) ? kXcds - 1 - x : x;
    return {(j * kXcds + xs) * kMBlock + rem / parts, rem % parts};
}

// number of m values launched: mmax + 1 rounded up to a multiple of kMBlock * kXcds
inline int64_t padded_m(int mmax) {
    constexpr int64_t q = (int64_t)kMBlock * kXcds;
    return ((int64_t)mmax + q) / q * q;
}
inline bool grid_ok(int64_t n) { return n > 0 && n < (int64_t)INT32_MAX; }

// Wave-wide min / max, returned as a wave-uniform (scalar) value so that
// loops bounded by it stay uniform and their coefficient loads scalar.
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off));
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off));
    return __builtin_amdgcn_readfirstlane(v);
}

// Read-only coefficient data (recurrence coefficients, scaled a_lm) seen
// through the constant address space: nothing a kernel stores may alias it,
// so loads at wave-uniform addresses become scalar (SGPR) loads.  (Pointers
// taken from a struct lose the __restrict__ that tells the compiler so.)
template <class T>
using const_ptr = const __attribute__((address_space(4))) T *;
template <class T>
__device__ __forceinline__ const_ptr<T> ro(const T *p) {
    return (const_ptr<T>)p;
}
// complex entries of such an array (re, im interleaved), loaded 16 bytes at a time
typedef double dvec2 __attribute__((ext_vector_type(2)));
struct ConstC {
    const_ptr<dvec2> p;
    __device__ __forceinline__ double2 operator[](int64_t i) const {
        const dvec2 v = p[i];
        return make_double2(v.x, v.y);
    }
};
__device__ __forceinline__ ConstC ro(const double2 *p) { return ConstC{ro(reinterpret_cast<const dvec2 *>(p))}; }

// A wave-uniform 64-bit value restated as such (for addresses that must stay
// on scalar registers).
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

}  // namespace sht
