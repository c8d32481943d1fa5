// Device-side building blocks: counter-based Philox4x32-10 and wavefront/block scans.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spv {
namespace dev {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): ten rounds of the Philox S-box -- two 32x32->64
// multiplications by the published multipliers, the high halves xored with
// the other two counter words and the round key -- with a Weyl key schedule.
// The key and the high counter words are usually wavefront-uniform, so the
// key schedule stays in scalar registers.
struct Words4 {
    uint32_t w[4];
};

__device__ __forceinline__ Words4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        // three-input xor in one gfx950 v_bitop3_b32 (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), c3, k1, 0x96);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    Words4 r;
    r.w[0] = c0;
    r.w[1] = c1;
    r.w[2] = c2;
    r.w[3] = c3;
    return r;
}

// Signed byte b (0..3) of a packed word of four int8 spins.
__device__ __forceinline__ int32_t spin_of(uint32_t w, int b) {
    return ((int32_t)(w << (24 - 8 * b))) >> 24;
}

// Lane index inside the 64-wide wavefront.
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Exclusive prefix count of `flag` over the lanes below this one.
__device__ __forceinline__ int wave_prefix(bool flag, unsigned long long *total) {
    const unsigned long long m = __ballot(flag);
    *total = m;
    const int l = lane_id();
    const unsigned long long below = (l == 0) ? 0ull : (m & ((~0ull) >> (64 - l)));
    return __popcll(below);
}

// Block-wide exclusive scan of small non-negative integers.  `tmp` holds
// blockDim/64 + 1 ints of LDS.  Returns the prefix; *sum receives the total.
__device__ __forceinline__ int block_exclusive_scan(int v, int *tmp, int *sum) {
    const int lane = lane_id();
    const int wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63 || threadIdx.x == blockDim.x - 1) tmp[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < nw; ++w) {
            int t = tmp[w];
            tmp[w] = acc;
            acc += t;
        }
        tmp[nw] = acc;
    }
    __syncthreads();
    int r = tmp[wid] + x - v;
    *sum = tmp[nw];
    __syncthreads();
    return r;
}

}  // namespace dev
}  // namespace spv
