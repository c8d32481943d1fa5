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

// Xor mask (0xFE per accepted byte) of the Metropolis decisions for x[b] = -s f of
// four replicas at their own temperatures (acceptance rows tb[b]): a byte is accepted
// iff every nonzero digit of x passes (x <= 0 has none).  The first digit's block is
// drawn without a branch (some byte of a word almost always has a nonzero first
// digit), so the decisions stay lane masks; a later digit's block is drawn where
// some byte has that digit nonzero (a byte already rejected stays rejected).
template <int ND>
__device__ __forceinline__ uint32_t metropolis_mask4(const int32_t x[4], const uint32_t *const tb[4], uint32_t i,
                                                     uint32_t t, uint32_t quad, uint32_t k0, uint32_t k1) {
    uint32_t d[4], th[4], mask = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        d[b] = x[b] > 0 ? ((uint32_t)x[b] & (kDigitSize - 1)) : 0u;
        th[b] = tb[b][d[b]];  // a zero digit reads a valid entry it ignores
    }
    {
        const dev::Words4 w = dev::philox(i, t, quad, 2u << 24, k0, k1);
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if ((d[b] == 0) | (w.w[b] < th[b])) mask |= 0xFEu << (8 * b);
    }
#pragma unroll
    for (int j = 1; j < ND; ++j) {
        bool need = false;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            d[b] = x[b] > 0 ? (((uint32_t)x[b] >> (kDigitBits * j)) & (kDigitSize - 1)) : 0u;
            need |= d[b] != 0;
            th[b] = tb[b][j * kDigitSize + d[b]];
        }
        if (need) {
            const dev::Words4 w = dev::philox(i, t, quad, (2u << 24) | (uint32_t)j, k0, k1);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if ((d[b] != 0) & (w.w[b] >= th[b])) mask &= ~(0xFEu << (8 * b));
        }
    }
    return mask;
}

// Replica-exchange decision (digit test of D with the tables of dbeta_k).  The
// thresholds of every nonzero digit are fetched together, then compared.
__device__ inline bool swap_test(long long D, const uint32_t *__restrict__ T, int nd, uint32_t k, uint32_t t,
                                 uint32_t c, uint32_t k0, uint32_t k1) {
    if (D <= 0) return true;
    if (nd < 7 && (D >> (kDigitBits * nd)) != 0) return false;
    uint32_t d[7], th[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        d[j] = j < nd ? (uint32_t)((D >> (kDigitBits * j)) & (kDigitSize - 1)) : 0u;
        th[j] = d[j] ? T[j * kDigitSize + d[j]] : 0u;
    }
    dev::Words4 w0 = dev::philox(k, t, c, 3u << 24, k0, k1);
    dev::Words4 w1 = w0;
    if (nd > 4) w1 = dev::philox(k, t, c, (3u << 24) | 1u, k0, k1);
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const uint32_t w = j < 4 ? w0.w[j] : w1.w[j - 4];
        if (d[j]) ok = ok && (w < th[j]);
    }
    return ok;
}

// Neighbour records are fetched this many at a time, so their loads (LDS or
// global) are in flight together instead of one after another.
constexpr int kRecBatch = 8;

// Local fields f[b] = h + sum_k J_k s_k[b] of the 4 replicas in word q of
// position p (spins S[pos][nq], records rec(k, p) = pos << 16 | uint16 J).
// DK > 0: exactly DK records per site (straight-line code); DK = 0: D at run time.
// Positions (16 bits) and word counts fit 24 bits, so the word index takes the
// full-rate 24-bit multiply rather than the quarter-rate 32-bit one.
template <int DK = 0, typename Rec>
__device__ __forceinline__ void quad_fields(Rec rec, int D, int p, const uint32_t *__restrict__ S, int nq, int q,
                                            int32_t h, int32_t f[4]) {
#pragma unroll
    for (int b = 0; b < 4; ++b) f[b] = h;
    if constexpr (DK > 0) {
        uint32_t rr[DK], w[DK];
#pragma unroll
        for (int u = 0; u < DK; ++u) rr[u] = rec(u, p);
#pragma unroll
        for (int u = 0; u < DK; ++u) w[u] = S[__umul24(rr[u] >> 16, (uint32_t)nq) + (uint32_t)q];
#pragma unroll
        for (int u = 0; u < DK; ++u) {
            const int32_t Jv = (int32_t)(int16_t)(rr[u] & 0xffffu);
#pragma unroll
            for (int b = 0; b < 4; ++b) f[b] += Jv * dev::spin_of(w[u], b);
        }
        return;
    }
    for (int k0 = 0; k0 < D; k0 += kRecBatch) {
        uint32_t rr[kRecBatch];
#pragma unroll
        for (int u = 0; u < kRecBatch; ++u) rr[u] = (k0 + u < D) ? rec(k0 + u, p) : 0u;
        uint32_t w[kRecBatch];
#pragma unroll
        for (int u = 0; u < kRecBatch; ++u) w[u] = (k0 + u < D) ? S[__umul24(rr[u] >> 16, (uint32_t)nq) + q] : 0u;
#pragma unroll
        for (int u = 0; u < kRecBatch; ++u) {
            const int32_t Jv = (int32_t)(int16_t)(rr[u] & 0xffffu);
#pragma unroll
            for (int b = 0; b < 4; ++b) f[b] += Jv * dev::spin_of(w[u], b);
        }
    }
}

// Lock-free union-find in LDS over 16-bit parents (parent[x] <= x always: a
// root is only ever hooked under a smaller root, so every find terminates;
// path splitting writes only ancestors, so concurrent finds stay valid).
__device__ __forceinline__ uint32_t uf_find(uint16_t *parent, uint32_t x) {
    uint32_t p = parent[x];
    while (p != x) {
        const uint32_t gp = parent[p];
        if (gp != p) parent[x] = (uint16_t)gp;
        x = p;
        p = gp;
    }
    return x;
}

// Compare-and-swap of one 16-bit half through a 32-bit CAS on its word; fails
// only when the half no longer holds `expect`.
__device__ __forceinline__ bool cas16(uint16_t *addr, uint32_t expect, uint32_t desired) {
    uint32_t *word = reinterpret_cast<uint32_t *>(reinterpret_cast<uintptr_t>(addr) & ~(uintptr_t)3);
    const int sh = (reinterpret_cast<uintptr_t>(addr) & 2) ? 16 : 0;
    uint32_t old = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    for (;;) {
        if (((old >> sh) & 0xffffu) != expect) return false;
        const uint32_t want = (old & ~(0xffffu << sh)) | (desired << sh);
        const uint32_t prev = atomicCAS(word, old, want);
        if (prev == old) return true;
        old = prev;
    }
}

__device__ __forceinline__ void uf_union(uint16_t *parent, uint32_t a, uint32_t b) {
    for (;;) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return;
        if (a > b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        if (cas16(&parent[b], b, a)) return;
    }
}

}  // namespace ptc
}  // namespace spv
