// Byte-parallel simulated-annealing body for instances whose x_bound is at
// most 255 (every sum_j |J_ij| fits a byte).  Results are bit-identical to the
// general body in sa_core.hpp; only the arithmetic layout differs.
//
// A spin byte is a mask, 0xFF for +1 and 0x00 for -1, and LDS holds both the
// spin words S[p][q] and their complements ~S[p][q].  A neighbour record is
// two words: the offset of the neighbour's row in S when J > 0, or in ~S when
// J < 0, and |J| replicated in all four bytes.  Then (row word & |J|rep) holds,
// per replica byte, |J| where the neighbour agrees with the sign of J, so one
// and + one add per neighbour accumulate P = sum of agreeing |J| for four
// replicas at once (no carries), and the local field is f = h - sum|J| + 2P.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device.hpp"
#include "internal.hpp"
#include "lds_shadow.hpp"
#include "sa_core.hpp"

namespace spv {
namespace core {

// Neighbour records of a site are contiguous (read 16 bytes at a time); the
// per-site stride, in records, is even with an odd number of 16-byte units, so
// that consecutive sites' blocks start in distinct LDS banks.
__host__ __device__ constexpr int swar_rec_stride(int D) {
    return (((D + 1) & ~1) / 2) % 2 == 1 ? ((D + 1) & ~1) : ((D + 1) & ~1) + 2;
}

// Acceptance tables sit at the start of the dynamic LDS, two buffers (this
// sweep, next sweep), each indexed by x in [-kSwarTabHalf, kSwarTabHalf) so
// that the row is read at x without clamping (entries below zero are never
// decisive: x <= 0 always flips).  Fixed offsets let the address be 4x plus
// an instruction immediate.
constexpr int kSwarTabHalf = 256;
constexpr int kSwarTabWords = 2 * kSwarTabHalf;

// The spin words follow the tables.  A record holds the neighbour word's LDS
// address itself, so that a lane holding its site's whole row reads it with
// no address arithmetic.
constexpr size_t kSwarSOffset = (size_t)2 * kSwarTabWords * 4;

typedef unsigned int swar_v2u __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) const uint32_t swar_lds_u32;
typedef __attribute__((address_space(3))) const swar_v2u swar_lds_v2u;

// The 32-bit LDS address of a shared-memory object.
__device__ __forceinline__ uint32_t swar_lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void *)p;
}
__device__ __forceinline__ uint32_t swar_ld32(uint32_t a) { return *(swar_lds_u32 *)(uintptr_t)a; }
__device__ __forceinline__ uint2 swar_ld64(uint32_t a) {
    const swar_v2u v = *(swar_lds_v2u *)(uintptr_t)a;
    return make_uint2(v.x, v.y);
}

struct SwarLds {
    uint32_t *tab;   // [2][kSwarTabWords]
    uint32_t *S;     // [2][n][qw]: spins, then their complements
    uint2 *rec;      // [n][stride]: {LDS address of the neighbour row in S or ~S, |J| x 0x01010101}
    uint2 *co;       // [n] {4 (h_p - sum_k |J_pk|) in both 16-bit halves, original index}
    int32_t *hpos;   // [n]
    unsigned long long *E2;  // [4*qw]
};

__host__ __device__ inline size_t swar_layout(int n, int D, int row_len, int qw, SwarLds *L,
                                              unsigned char *base, int e2q = 0) {
    (void)row_len;
    if (e2q < qw) e2q = qw;
    size_t o_tab = 0;
    size_t o_S = kSwarSOffset;
    size_t o_rec = (o_S + (size_t)2 * n * qw * 4 + 15) & ~(size_t)15;
    size_t o_co = o_rec + (size_t)n * swar_rec_stride(D) * 8;
    size_t o_h = o_co + (size_t)n * 8;
    size_t o_E = (o_h + (size_t)n * 4 + 7) & ~(size_t)7;
    size_t end = o_E + (size_t)4 * e2q * 8;
    if (L) {
        L->tab = reinterpret_cast<uint32_t *>(base + o_tab);
        L->S = reinterpret_cast<uint32_t *>(base + o_S);
        L->rec = reinterpret_cast<uint2 *>(base + o_rec);
        L->co = reinterpret_cast<uint2 *>(base + o_co);
        L->hpos = reinterpret_cast<int32_t *>(base + o_h);
        L->E2 = reinterpret_cast<unsigned long long *>(base + o_E);
    }
    return end;
}

__device__ __forceinline__ int32_t swar_cp(uint2 co) { return ((int32_t)(int16_t)(co.x & 0xffffu)) / 4; }

// Global-memory instance of a problem too large for LDS: the same records (with
// addresses relative to the spin words) and site constants, built once per call.
__host__ __device__ inline size_t swar_big_bytes(int n, int D) {
    return (size_t)n * swar_rec_stride(D) * 8 + (size_t)n * 8 + (size_t)n * 4;
}
__device__ inline void swar_bind_big(SwarLds *L, unsigned char *g, int n, int D) {
    L->rec = reinterpret_cast<uint2 *>(g);
    L->co = reinterpret_cast<uint2 *>(g + (size_t)n * swar_rec_stride(D) * 8);
    L->hpos = reinterpret_cast<int32_t *>(g + (size_t)n * swar_rec_stride(D) * 8 + (size_t)n * 8);
}
// LDS of the variant: tables, spins, energy accumulators.
__host__ __device__ inline size_t swar_big_lds_bytes(int n, int qw) {
    const size_t o_E = (kSwarSOffset + (size_t)2 * n * qw * 4 + 7) & ~(size_t)7;
    return o_E + (size_t)4 * qw * 8;
}
__device__ inline void swar_big_layout(int n, int qw, SwarLds *L, unsigned char *base) {
    L->tab = reinterpret_cast<uint32_t *>(base);
    L->S = reinterpret_cast<uint32_t *>(base + kSwarSOffset);
    L->E2 = reinterpret_cast<unsigned long long *>(base + ((kSwarSOffset + (size_t)2 * n * qw * 4 + 7) & ~(size_t)7));
}

// Byte-parallel records and site constants of positions [i0, n) step `step`, record
// addresses based at `sb` (the LDS address of the spin words, or 0 for addresses
// relative to them).
__device__ inline void swar_build(uint2 *rec, uint2 *co, int32_t *hpos, const SaItem &a, uint32_t sb, int i0,
                                  int step) {
    const int n = a.n, D = a.D, Ds = swar_rec_stride(D);
    const int32_t *img = a.image;
    const uint32_t *recs = reinterpret_cast<const uint32_t *>(img + kImgHeader + 3 * n);
    const uint32_t inv = (uint32_t)n * (uint32_t)a.qw;  // offset of ~S
    for (int idx = i0; idx < n * Ds; idx += step) {
        const int p = idx / Ds, k = idx - p * Ds;
        uint2 v = make_uint2(sb, 0u);  // padding: a valid address, weight 0
        if (k < D) {
            const uint32_t r = recs[(size_t)p * D + k];
            const int32_t J = (int32_t)(int16_t)(r & 0xffffu);
            const uint32_t off = (r >> 16) * (uint32_t)a.qw + (J < 0 ? inv : 0u);
            v = make_uint2(sb + 4u * off, (uint32_t)(J < 0 ? -J : J) * 0x01010101u);
        }
        rec[idx] = v;
    }
    for (int p = i0; p < n; p += step) {
        int32_t s = 0;
        for (int k = 0; k < D; ++k) {
            const int32_t J = (int32_t)(int16_t)(recs[(size_t)p * D + k] & 0xffffu);
            s += J < 0 ? -J : J;
        }
        const int32_t h = img[kImgHeader + 2 * n + p];
        const uint32_t c16 = (uint32_t)(4 * (h - s)) & 0xffffu;
        hpos[p] = h;
        co[p] = make_uint2(c16 | (c16 << 16), (uint32_t)img[kImgHeader + p]);
    }
}

// Colour-class bounds only (the instance of the global-memory variant).  Ends with a barrier.
__device__ inline void swar_load_colours(const SaItem &a, int *cs) {
    if ((int)threadIdx.x <= a.C) cs[threadIdx.x] = a.image[3 + threadIdx.x];
    __syncthreads();
}

// Expands the image's 32-bit records into byte-parallel records.  Ends with a barrier.
__device__ inline void swar_load_instance(const SwarLds &L, const SaItem &a, int *cs) {
    const int T = blockDim.x, tid = threadIdx.x;
    if (tid <= a.C) cs[tid] = a.image[3 + tid];
    swar_build(L.rec, L.co, L.hpos, a, swar_lds_addr(L.S), tid, T);
    __syncthreads();
}

// Neighbour records are read this many at a time (loads issued together).
constexpr int kSwarBatch = 8;

// Per byte, the sum of |J_k| over the neighbours agreeing with sign(J_k), for the
// W consecutive quad words of this lane; `rp` is the site's record block and `qb`
// the byte offset of this lane's first column (0 when W = 2).  DK > 0: the record
// count is DK exactly (straight-line code); DK = 0: D at run time.
template <int DK, int W>
__device__ __forceinline__ void swar_agree(const uint2 *__restrict__ rp, uint32_t qb, int D, uint32_t (&P)[W]) {
    auto word = [&](uint32_t addr, uint32_t (&w)[W]) {
        if constexpr (W == 2) {
            const uint2 v = swar_ld64(addr + qb);
            w[0] = v.x;
            w[1] = v.y;
        } else {
            w[0] = swar_ld32(addr + qb);
        }
    };
#pragma unroll
    for (int b = 0; b < W; ++b) P[b] = 0;
    if constexpr (DK > 0) {
        constexpr int U = (DK + 1) / 2;
        uint4 r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = reinterpret_cast<const uint4 *>(rp)[u];
        uint32_t w[DK][W];
#pragma unroll
        for (int k = 0; k < DK; ++k) word((k & 1) ? r[k / 2].z : r[k / 2].x, w[k]);
#pragma unroll
        for (int k = 0; k < DK; ++k)
#pragma unroll
            for (int b = 0; b < W; ++b) P[b] += w[k][b] & ((k & 1) ? r[k / 2].w : r[k / 2].y);
        return;
    }
    for (int k0 = 0; k0 < D; k0 += kSwarBatch) {
        uint2 r[kSwarBatch];
#pragma unroll
        for (int u = 0; u < kSwarBatch; ++u)
            if (k0 + u < D) r[u] = rp[k0 + u];
        uint32_t w[kSwarBatch][W];
#pragma unroll
        for (int u = 0; u < kSwarBatch; ++u)
            if (k0 + u < D) word(r[u].x, w[u]);
#pragma unroll
        for (int u = 0; u < kSwarBatch; ++u)
            if (k0 + u < D)
#pragma unroll
                for (int b = 0; b < W; ++b) P[b] += w[u][b] & r[u].y;
    }
}

__device__ __forceinline__ void swar_store(uint32_t *S, uint32_t idx, uint32_t inv, uint32_t w) {
    S[idx] = w;
    S[idx + inv] = ~w;
}

typedef unsigned short swar_u16x2 __attribute__((ext_vector_type(2)));
typedef short swar_i16x2 __attribute__((ext_vector_type(2)));

// 4x = -4 s f for the four replicas of a word, as two pairs of int16 (replicas 0, 1 and 2, 3):
// 4f = 4 cp + 8 P_b fits 16 bits (|f| <= x_bound <= 255), and the spin byte masks, widened to
// 16 bits, negate it where the spin is +1.  `cp2` holds 4 cp in both halves.
__device__ __forceinline__ void swar_x16(uint32_t P, uint32_t self, uint32_t cp2, swar_i16x2 *lo, swar_i16x2 *hi) {
    const uint32_t Plo = __builtin_amdgcn_perm(P, P, 0x0C010C00u);  // bytes P0, 0, P1, 0
    const uint32_t Phi = __builtin_amdgcn_perm(P, P, 0x0C030C02u);  // bytes P2, 0, P3, 0
    const uint32_t mlo = __builtin_amdgcn_perm(self, self, 0x01010000u);
    const uint32_t mhi = __builtin_amdgcn_perm(self, self, 0x03030202u);
    const swar_u16x2 c = __builtin_bit_cast(swar_u16x2, cp2);
    const swar_u16x2 flo = __builtin_bit_cast(swar_u16x2, Plo) * (unsigned short)8 + c;
    const swar_u16x2 fhi = __builtin_bit_cast(swar_u16x2, Phi) * (unsigned short)8 + c;
    const swar_u16x2 ml = __builtin_bit_cast(swar_u16x2, mlo), mh = __builtin_bit_cast(swar_u16x2, mhi);
    *lo = __builtin_bit_cast(swar_i16x2, (swar_u16x2)((flo ^ ml) - ml));
    *hi = __builtin_bit_cast(swar_i16x2, (swar_u16x2)((fhi ^ mh) - mh));
}

// A contiguous range of sweeps of one workgroup's replicas.  The whole schedule
// is one chunk; a streamed launch splits it, carrying the spin words between
// chunks through global memory.
struct SwarChunk {
    int ls0 = 0;             // first sweep
    int count = -1;          // sweeps (-1: to the end of the schedule)
    bool resume = false;     // the caller has put the spin words (S and ~S) in LDS
    bool keep = false;       // leave the spin words in LDS for the caller (not the last chunk)
    bool poisoned = false;   // last chunk: a wait for an earlier chunk was abandoned
};

// Energy written for every read of a workgroup whose chunks lost their order.
constexpr long long kSwarPoisonEnergy = INT64_MIN;

// W = quad words per lane: 1, or 2 when qw = 2 and a lane holds its site's whole
// row (the neighbour addresses are then the records' addresses as they stand).
// BIG: records and site constants in global memory, record addresses relative to
// the spin words.
template <int DK, int W, bool BIG = false>
__device__ void swar_run(const SwarLds &L, const SaItem &a, const int *cs, const SwarChunk &ch = SwarChunk()) {
    static_assert(W == 1 || W == 2, "one or two words per lane");
    const int n = a.n, D = a.D, qw = W == 2 ? 2 : a.qw, T = blockDim.x, tid = threadIdx.x;
    const int Ds = DK > 0 ? swar_rec_stride(DK) : swar_rec_stride(D);
    const int q0 = a.q0;
    const int lps = qw / W;  // lanes per site
    const int qa = W == 2 ? 0 : tid % lps, slot = tid / lps, nslots = T / lps;
    const bool active = slot < nslots;
    const uint32_t inv = (uint32_t)n * (uint32_t)qw;
    const uint32_t qb = 4u * (uint32_t)qa + (BIG ? swar_lds_addr(L.S) : 0u);
    const int ls0 = ch.ls0, lsend = ch.count < 0 ? a.sweeps : ls0 + ch.count;
    for (int k = tid; k < 2 * kSwarTabWords; k += T) {
        const int i = k % kSwarTabWords - kSwarTabHalf;
        L.tab[k] = (i >= 0 && k < kSwarTabWords && i < a.row_len && ls0 < lsend)
                       ? a.tables[(size_t)ls0 * a.row_len + i]
                       : 0xFFFFFFFFu;
    }
    for (int k = tid; k < 4 * qw; k += T) L.E2[k] = 0ull;
    if (ch.resume) {
        // spin words already in LDS
    } else if (a.init == nullptr) {
        for (int p = slot; active && p < n; p += nslots)
#pragma unroll
            for (int b = 0; b < W; ++b) {
                const dev::Words4 w = dev::philox(L.co[p].y, 0u, (uint32_t)(q0 + qa + b), 1u << 24, a.k0, a.k1);
                uint32_t word = 0;
#pragma unroll
                for (int e = 0; e < 4; ++e) word |= ((w.w[e] >> 31) ? 0xFFu : 0x00u) << (8 * e);
                swar_store(L.S, (uint32_t)p * (uint32_t)qw + (uint32_t)(qa + b), inv, word);
            }
    } else {
        const int32_t *pos_of = a.image + kImgHeader + n;
        unsigned char *Sb = reinterpret_cast<unsigned char *>(L.S);
        for (int idx = tid; idx < 4 * qw * n; idx += T) {
            const int rl = idx / n, i = idx - rl * n;
            const int r = 4 * q0 + rl;
            unsigned char v = 0xFF;
            if (r < a.reads) v = a.init[(size_t)r * n + i] > 0 ? 0xFF : 0x00;
            const size_t at = ((size_t)pos_of[i] * qw + (rl >> 2)) * 4 + (rl & 3);
            Sb[at] = v;
            Sb[at + 4 * inv] = (unsigned char)~v;
        }
    }
    __syncthreads();
    const shadow::Pass sh = shadow::begin(inv);
    const uint32_t s_addr = swar_lds_addr(L.S);
    // Debug build: the class pass's writes, then its neighbour reads, against the bitmap.
    auto shadow_pass = [&](int c, bool before) {
        const int pe = cs[c + 1];
        if (before) {
            for (int p = cs[c] + slot; active && p < pe; p += nslots)
                for (int b = 0; b < W; ++b) shadow::mark(sh, (uint32_t)p * (uint32_t)qw + (uint32_t)(qa + b));
            shadow::barrier();
            for (int p = cs[c] + slot; active && p < pe; p += nslots)
                for (int k = 0; k < (DK > 0 ? DK : D); ++k) {
                    const uint2 r = L.rec[(uint32_t)p * (uint32_t)Ds + (uint32_t)k];
                    if (r.y == 0u) continue;  // padding or J = 0: the value read is unused
                    uint32_t w = (r.x + qb - s_addr) >> 2;
                    if (w >= inv) w -= inv;
                    for (int b = 0; b < W; ++b) shadow::check(sh, w + (uint32_t)b);
                }
            shadow::count_pass(sh);
        } else {
            for (int p = cs[c] + slot; active && p < pe; p += nslots)
                for (int b = 0; b < W; ++b) shadow::unmark(sh, (uint32_t)p * (uint32_t)qw + (uint32_t)(qa + b));
            shadow::barrier();
        }
    };

    // One sweep reading table buffer B (a compile-time constant) and filling the other.
    auto sweep = [&](auto buf, int ls) {
        constexpr int B = decltype(buf)::value;
        const uint32_t t = a.sweep_offset + (uint32_t)ls;
        const char *tz = reinterpret_cast<const char *>(L.tab + B * kSwarTabWords + kSwarTabHalf);
        if (ls + 1 < lsend) {
            uint32_t *tnext = L.tab + (1 - B) * kSwarTabWords + kSwarTabHalf;
            for (int k = tid; k < a.row_len; k += T) tnext[k] = a.tables[(size_t)(ls + 1) * a.row_len + k];
        }
        for (int c = 0; c < a.C; ++c) {
            if constexpr (shadow::kOn) shadow_pass(c, true);
            const int pe = cs[c + 1];
            for (int p = cs[c] + slot; active && p < pe; p += nslots) {
                const uint32_t at = (uint32_t)p * (uint32_t)qw + (uint32_t)qa;
                uint32_t self[W];
                if constexpr (W == 2) {
                    const uint2 v = *reinterpret_cast<const uint2 *>(L.S + at);
                    self[0] = v.x;
                    self[1] = v.y;
                } else {
                    self[0] = L.S[at];
                }
                uint32_t P[W];
                swar_agree<DK, W>(L.rec + (uint32_t)p * (uint32_t)Ds, qb, D, P);
                const uint2 co = L.co[p];
                uint32_t mask[W];
#pragma unroll
                for (int b = 0; b < W; ++b) {
                    swar_i16x2 xlo, xhi;  // 4x
                    swar_x16(P[b], self[b], co.x, &xlo, &xhi);
                    // Random words are drawn for every replica; x <= 0 flips regardless of them.
                    const dev::Words4 r = dev::philox(co.y, t, (uint32_t)(q0 + qa + b), 2u << 24, a.k0, a.k1);
                    // byte offsets 4x into the row (x may be <= 0: the entry is read and ignored)
                    const int32_t o[4] = {xlo.x, xlo.y, xhi.x, xhi.y};
                    uint32_t th[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) th[e] = *reinterpret_cast<const uint32_t *>(tz + o[e]);
                    uint32_t m = 0;
#pragma unroll
                    for (int e = 0; e < 4; ++e) m |= (uint32_t)((o[e] <= 0) | (r.w[e] < th[e])) * (0xFFu << (8 * e));
                    mask[b] = m;
                }
                if constexpr (W == 2) {
                    if (mask[0] | mask[1]) {
                        const uint2 v = make_uint2(self[0] ^ mask[0], self[1] ^ mask[1]);
                        *reinterpret_cast<uint2 *>(L.S + at) = v;
                        *reinterpret_cast<uint2 *>(L.S + at + inv) = make_uint2(~v.x, ~v.y);
                    }
                } else {
                    if (mask[0]) swar_store(L.S, at, inv, self[0] ^ mask[0]);
                }
            }
            __syncthreads();
            if constexpr (shadow::kOn) shadow_pass(c, false);
        }
    };
    for (int ls = ls0; ls < lsend; ls += 2) {
        sweep(std::integral_constant<int, 0>{}, ls);
        if (ls + 1 < lsend) sweep(std::integral_constant<int, 1>{}, ls + 1);
    }
    if (ch.keep) {
        __syncthreads();
        return;
    }

    {
        long long e2[W][4] = {};
        for (int p = slot; active && p < n; p += nslots) {
            uint32_t P[W];
            swar_agree<DK, W>(L.rec + (uint32_t)p * (uint32_t)Ds, qb, D, P);
            const long long cp = swar_cp(L.co[p]), hp = L.hpos[p];
#pragma unroll
            for (int b = 0; b < W; ++b) {
                const uint32_t self = L.S[(uint32_t)p * (uint32_t)qw + (uint32_t)(qa + b)];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const long long f = cp + 2 * (long long)((P[b] >> (8 * e)) & 0xffu);
                    const long long s = ((self >> (8 * e)) & 0xffu) ? 1 : -1;
                    e2[b][e] += s * (hp + f);
                }
            }
        }
        if (active)
#pragma unroll
            for (int b = 0; b < W; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e) atomicAdd(&L.E2[(qa + b) * 4 + e], (unsigned long long)e2[b][e]);
    }
    __syncthreads();
    for (int rl = tid; rl < 4 * qw; rl += T) {
        const int r = 4 * q0 + rl;
        if (r < a.reads) a.energies[r] = ch.poisoned ? kSwarPoisonEnergy : ((long long)L.E2[rl]) / 2;
    }
    const int32_t *pos_of = a.image + kImgHeader + n;
    const unsigned char *Sb = reinterpret_cast<const unsigned char *>(L.S);
    for (int idx = tid; idx < 4 * qw * n; idx += T) {
        const int rl = idx / n, i = idx - rl * n;
        const int r = 4 * q0 + rl;
        if (r < a.reads)
            a.out[(size_t)r * n + i] = Sb[((size_t)pos_of[i] * qw + (rl >> 2)) * 4 + (rl & 3)] ? 1 : -1;
    }
    __syncthreads();
}

// q = x / d and r = x - q d for 0 <= x < 2^20 and 1 <= d < 2^16: the float quotient
// through v_rcp_f32 is within 1 of the true one (relative error below 2^-21), so one
// correction in each direction makes it exact.
__device__ __forceinline__ void swar_divmod(int x, int d, int &q, int &r) {
    q = (int)((float)x * __builtin_amdgcn_rcpf((float)d));
    r = x - q * d;
    if (r < 0) {
        --q;
        r += d;
    }
    if (r >= d) {
        ++q;
        r -= d;
    }
}

// Paired body of the batched launch: `copies` pairs of quad words of one instance.
// Pair k has its own region of the spin area, S_k [n][2] then ~S_k [n][2] (4n words
// at k * 4n), and every pair shares the instance's records, whose neighbour addresses
// are those of region 0 (the lane adds its region's byte offset).  A lane holds one
// site of one pair, both words (8 replicas, as the two-words-per-lane body), and the
// lanes of a class pass take (pair, site) tasks pair-major, so small instances fill
// the workgroup with several pairs.  Pair k's quads are q0 + 2k and q0 + 2k + 1; the
// counters, tables and update order are the one-instance launch's, so the bits are too.
template <int DK>
__device__ void swar_run_pairs(const SwarLds &L, const SaItem &a, const int *cs, int copies) {
    static_assert(DK > 0, "the paired body unrolls a fixed record count");
    constexpr int Ds = swar_rec_stride(DK);
    const int n = a.n, T = blockDim.x, tid = threadIdx.x, q0 = a.q0;
    const uint32_t region = 4u * (uint32_t)n, inv = 2u * (uint32_t)n;
    for (int k = tid; k < 2 * kSwarTabWords; k += T) {
        const int i = k % kSwarTabWords - kSwarTabHalf;
        L.tab[k] = (i >= 0 && k < kSwarTabWords && i < a.row_len && a.sweeps > 0) ? a.tables[i] : 0xFFFFFFFFu;
    }
    for (int k = tid; k < 8 * copies; k += T) L.E2[k] = 0ull;
    for (int v = tid; v < copies * n; v += T) {
        int k, p;
        swar_divmod(v, n, k, p);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const dev::Words4 w = dev::philox(L.co[p].y, 0u, (uint32_t)(q0 + 2 * k + b), 1u << 24, a.k0, a.k1);
            uint32_t word = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) word |= ((w.w[e] >> 31) ? 0xFFu : 0x00u) << (8 * e);
            swar_store(L.S, (uint32_t)k * region + 2u * (uint32_t)p + (uint32_t)b, inv, word);
        }
    }
    __syncthreads();
    // Debug build: bit of S word w of pair k is k * 2n + w.
    const shadow::Pass sh = shadow::begin((uint32_t)copies * inv);
    const uint32_t s_addr = swar_lds_addr(L.S);
    auto shadow_pass = [&](int pb, int cls, bool before) {
        if (before) {
            for (int v = tid; v < copies * cls; v += T)
                for (int b = 0; b < 2; ++b)
                    shadow::mark(sh, (uint32_t)(v / cls) * inv + 2u * (uint32_t)(pb + v % cls) + (uint32_t)b);
            shadow::barrier();
            for (int v = tid; v < copies * cls; v += T) {
                const int k = v / cls, p = pb + v % cls;
                for (int j = 0; j < DK; ++j) {
                    const uint2 r = L.rec[(uint32_t)p * (uint32_t)Ds + (uint32_t)j];
                    if (r.y == 0u) continue;  // padding or J = 0: the value read is unused
                    uint32_t w = (r.x - s_addr) >> 2;  // region 0 address
                    if (w >= inv) w -= inv;
                    for (int b = 0; b < 2; ++b) shadow::check(sh, (uint32_t)k * inv + w + (uint32_t)b);
                }
            }
            shadow::count_pass(sh);
        } else {
            for (int v = tid; v < copies * cls; v += T)
                for (int b = 0; b < 2; ++b)
                    shadow::unmark(sh, (uint32_t)(v / cls) * inv + 2u * (uint32_t)(pb + v % cls) + (uint32_t)b);
            shadow::barrier();
        }
    };

    auto sweep = [&](auto buf, int ls) {
        constexpr int B = decltype(buf)::value;
        const uint32_t t = a.sweep_offset + (uint32_t)ls;
        const char *tz = reinterpret_cast<const char *>(L.tab + B * kSwarTabWords + kSwarTabHalf);
        if (ls + 1 < a.sweeps) {
            uint32_t *tnext = L.tab + (1 - B) * kSwarTabWords + kSwarTabHalf;
            for (int k = tid; k < a.row_len; k += T) tnext[k] = a.tables[(size_t)(ls + 1) * a.row_len + k];
        }
        for (int c = 0; c < a.C; ++c) {
            const int pb = cs[c], cls = cs[c + 1] - pb;
            if constexpr (shadow::kOn) shadow_pass(pb, cls, true);
            if (cls > 0) {
                // this lane's first task and the step between its tasks, as (pair, site)
                int k, loc, dk, dl;
                swar_divmod(tid, cls, k, loc);
                swar_divmod(T, cls, dk, dl);
                while (k < copies) {
                    const int p = pb + loc;
                    const uint32_t at = (uint32_t)k * region + 2u * (uint32_t)p;
                    const uint2 sv = *reinterpret_cast<const uint2 *>(L.S + at);
                    const uint32_t self[2] = {sv.x, sv.y};
                    uint32_t P[2];
                    swar_agree<DK, 2>(L.rec + (uint32_t)p * (uint32_t)Ds, 4u * (uint32_t)k * region, DK, P);
                    const uint2 co = L.co[p];
                    uint32_t mask[2];
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        swar_i16x2 xlo, xhi;  // 4x
                        swar_x16(P[b], self[b], co.x, &xlo, &xhi);
                        const dev::Words4 r =
                            dev::philox(co.y, t, (uint32_t)(q0 + 2 * k + b), 2u << 24, a.k0, a.k1);
                        const int32_t o[4] = {xlo.x, xlo.y, xhi.x, xhi.y};
                        uint32_t th[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) th[e] = *reinterpret_cast<const uint32_t *>(tz + o[e]);
                        uint32_t m = 0;
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            m |= (uint32_t)((o[e] <= 0) | (r.w[e] < th[e])) * (0xFFu << (8 * e));
                        mask[b] = m;
                    }
                    if (mask[0] | mask[1]) {
                        const uint2 v = make_uint2(self[0] ^ mask[0], self[1] ^ mask[1]);
                        *reinterpret_cast<uint2 *>(L.S + at) = v;
                        *reinterpret_cast<uint2 *>(L.S + at + inv) = make_uint2(~v.x, ~v.y);
                    }
                    loc += dl;
                    k += dk;
                    if (loc >= cls) {
                        loc -= cls;
                        ++k;
                    }
                }
            }
            __syncthreads();
            if constexpr (shadow::kOn) shadow_pass(pb, cls, false);
        }
    };
    for (int ls = 0; ls < a.sweeps; ls += 2) {
        sweep(std::integral_constant<int, 0>{}, ls);
        if (ls + 1 < a.sweeps) sweep(std::integral_constant<int, 1>{}, ls + 1);
    }

    // 2E of every replica, sum over sites of s (h + f), one task per (pair, site)
    for (int v = tid; v < copies * n; v += T) {
        int k, p;
        swar_divmod(v, n, k, p);
        uint32_t P[2];
        swar_agree<DK, 2>(L.rec + (uint32_t)p * (uint32_t)Ds, 4u * (uint32_t)k * region, DK, P);
        const long long cp = swar_cp(L.co[p]), hp = L.hpos[p];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const uint32_t self = L.S[(uint32_t)k * region + 2u * (uint32_t)p + (uint32_t)b];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const long long f = cp + 2 * (long long)((P[b] >> (8 * e)) & 0xffu);
                const long long s = ((self >> (8 * e)) & 0xffu) ? 1 : -1;
                atomicAdd(&L.E2[(2 * k + b) * 4 + e], (unsigned long long)(s * (hp + f)));
            }
        }
    }
    __syncthreads();
    for (int rl = tid; rl < 8 * copies; rl += T) {
        const int r = 4 * q0 + rl;
        if (r < a.reads) a.energies[r] = ((long long)L.E2[rl]) / 2;
    }
    const int32_t *pos_of = a.image + kImgHeader + n;
    const unsigned char *Sb = reinterpret_cast<const unsigned char *>(L.S);
    for (int idx = tid; idx < 8 * copies * n; idx += T) {
        int rl, i;
        swar_divmod(idx, n, rl, i);
        const int r = 4 * q0 + rl;
        if (r < a.reads) {
            const int k = rl >> 3, b = (rl >> 2) & 1, e = rl & 3;
            a.out[(size_t)r * n + i] =
                Sb[((size_t)k * region + 2 * (size_t)pos_of[i] + (size_t)b) * 4 + (size_t)e] ? 1 : -1;
        }
    }
    __syncthreads();
}

}  // namespace core
}  // namespace spv
