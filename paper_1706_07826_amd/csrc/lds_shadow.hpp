// LDS race detection for the Metropolis class passes (debug build, SPV_LDS_SHADOW=1).
//
// A class pass updates the sites of one colour class: each task (a site and its
// spin words) reads its own words and its neighbours' and writes its own, and the
// pass ends at a barrier.  It is race-free iff no word is written by two tasks and
// no task reads a word that another task of the same pass writes.  The debug build
// checks both conditions on every pass, independently of timing:
//   1. every task sets its words' bits in a "written this pass" bitmap in LDS (a bit
//      already set is a write-write conflict),
//   2. barrier; every task tests the bits of the neighbour words it will read (a set
//      bit is a read-write conflict: that neighbour changes during the pass),
//   3. the pass itself, barrier, every task clears its bits, barrier.
// Conflicts are counted, never trapped: the kernels run to completion and the host
// reads the counts (write-write, read-write, passes checked, launches whose spin
// area exceeds the bitmap).  In the normal build every hook compiles to nothing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace spv {
namespace shadow {

constexpr bool kOn = kLdsShadow;
// Bitmap capacity: one bit per spin word, S only (a complement word ~S is written by
// the task that writes S).  64 Ki words cover any spin area that fits the LDS.
constexpr int kBits = 65536;
constexpr int kWords = kBits / 32;
static_assert(kShadowLdsBytes == (kOn ? (size_t)kWords * 4 : 0), "LDS the bitmap takes from a workgroup");

enum Stat { kWriteWrite = 0, kReadWrite = 1, kPasses = 2, kUncovered = 3, kStats = 4 };

#if SPV_LDS_SHADOW
// Counts of this translation unit's kernels (each unit keeps its own copy).
static __device__ unsigned long long g_stats[kStats];

__device__ inline uint32_t *bitmap() {
    __shared__ uint32_t bits[kWords];
    return bits;
}
#endif

// A pass's view of the bitmap; `covered` is false when the spin area has more
// words than the bitmap (then nothing is checked and the launch is counted).
struct Pass {
    uint32_t *bits = nullptr;
    bool covered = false;
};

// Clears the bitmap; called once by every thread before the first pass.  Ends with
// a barrier.
__device__ inline Pass begin(uint32_t words) {
    Pass s;
#if SPV_LDS_SHADOW
    s.bits = bitmap();
    s.covered = words <= (uint32_t)kBits;
    for (int k = threadIdx.x; k < kWords; k += blockDim.x) s.bits[k] = 0u;
    if (!s.covered && threadIdx.x == 0) atomicAdd(&g_stats[kUncovered], 1ull);
    __syncthreads();
#else
    (void)words;
#endif
    return s;
}

__device__ inline void mark(const Pass &s, uint32_t w) {
#if SPV_LDS_SHADOW
    if (!s.covered) return;
    const uint32_t bit = 1u << (w & 31u);
    if (atomicOr(&s.bits[w >> 5], bit) & bit) atomicAdd(&g_stats[kWriteWrite], 1ull);
#else
    (void)s;
    (void)w;
#endif
}

__device__ inline void check(const Pass &s, uint32_t w) {
#if SPV_LDS_SHADOW
    if (!s.covered) return;
    if (s.bits[w >> 5] & (1u << (w & 31u))) atomicAdd(&g_stats[kReadWrite], 1ull);
#else
    (void)s;
    (void)w;
#endif
}

__device__ inline void unmark(const Pass &s, uint32_t w) {
#if SPV_LDS_SHADOW
    if (!s.covered) return;
    atomicAnd(&s.bits[w >> 5], ~(1u << (w & 31u)));
#else
    (void)s;
    (void)w;
#endif
}

// One pass counted (thread 0 of the workgroup).
__device__ inline void count_pass(const Pass &s) {
#if SPV_LDS_SHADOW
    if (s.covered && threadIdx.x == 0) atomicAdd(&g_stats[kPasses], 1ull);
#else
    (void)s;
#endif
}

__device__ inline void barrier() {
    if constexpr (kOn) __syncthreads();
}

// Host: adds this unit's counts to out[kStats] and optionally clears them.
#if SPV_LDS_SHADOW
static inline hipError_t read_stats(unsigned long long *out, bool reset) {
    unsigned long long v[kStats] = {};
    hipError_t e = hipMemcpyFromSymbol(v, HIP_SYMBOL(g_stats), sizeof v, 0, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    for (int k = 0; k < kStats; ++k) out[k] += v[k];
    if (reset) {
        const unsigned long long z[kStats] = {};
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_stats), z, sizeof z, 0, hipMemcpyHostToDevice);
    }
    return e;
}
#else
static inline hipError_t read_stats(unsigned long long *, bool) { return hipSuccess; }
#endif

}  // namespace shadow
}  // namespace spv
