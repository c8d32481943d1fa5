// Device helpers shared by the tempering kernels: lane masks, wavefront sums
// and the replica-exchange acceptance test.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"
#include "internal.hpp"

namespace spv {
namespace ptc {

__device__ __forceinline__ unsigned long long lanemask_lt() {
    const int l = dev::lane_id();
    return l == 0 ? 0ull : ((~0ull) >> (64 - l));
}

__device__ __forceinline__ long long wave_sum(long long v) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Replica-exchange decision (digit test of D with the tables of dbeta_k).
__device__ inline bool swap_test(long long D, const uint32_t *__restrict__ T, int nd, uint32_t k, uint32_t t,
                          uint32_t c, uint32_t k0, uint32_t k1) {
    if (D <= 0) return true;
    if (nd < 7 && (D >> (kDigitBits * nd)) != 0) return false;
    dev::Words4 w0 = dev::philox(k, t, c, 3u << 24, k0, k1);
    dev::Words4 w1 = w0;
    if (nd > 4) w1 = dev::philox(k, t, c, (3u << 24) | 1u, k0, k1);
    for (int j = 0; j < nd; ++j) {
        const uint32_t d = (uint32_t)((D >> (kDigitBits * j)) & (kDigitSize - 1));
        if (d == 0) continue;
        const uint32_t w = j < 4 ? w0.w[j] : w1.w[j - 4];
        if (!(w < T[j * kDigitSize + d])) return false;
    }
    return true;
}

}  // namespace ptc
}  // namespace spv
