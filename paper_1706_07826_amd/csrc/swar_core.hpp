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

#include <type_traits>

#include "device.hpp"
#include "internal.hpp"
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

struct SwarLds {
    uint32_t *tab;   // [2][kSwarTabWords]
    uint2 *rec;      // [n][stride]: {offset of the neighbour row in S or ~S, |J| x 0x01010101}
    uint2 *co;       // [n] {(h_p - sum_k |J_pk|) in both 16-bit halves, original index}
    int32_t *hpos;   // [n]
    uint32_t *S;     // [2][n][qw]: spins, then their complements
    unsigned long long *E2;  // [4*qw]
};

__host__ __device__ inline size_t swar_layout(int n, int D, int row_len, int qw, SwarLds *L,
                                              unsigned char *base, int e2q = 0) {
    (void)row_len;
    if (e2q < qw) e2q = qw;
    size_t o_tab = 0;
    size_t o_rec = o_tab + (size_t)2 * kSwarTabWords * 4;
    size_t o_co = o_rec + (size_t)n * swar_rec_stride(D) * 8;
    size_t o_h = o_co + (size_t)n * 8;
    size_t o_S = o_h + (size_t)n * 4;
    size_t o_E = (o_S + (size_t)2 * n * qw * 4 + 7) & ~(size_t)7;
    size_t end = o_E + (size_t)4 * e2q * 8;
    if (L) {
        L->tab = reinterpret_cast<uint32_t *>(base + o_tab);
        L->rec = reinterpret_cast<uint2 *>(base + o_rec);
        L->co = reinterpret_cast<uint2 *>(base + o_co);
        L->hpos = reinterpret_cast<int32_t *>(base + o_h);
        L->S = reinterpret_cast<uint32_t *>(base + o_S);
        L->E2 = reinterpret_cast<unsigned long long *>(base + o_E);
    }
    return end;
}

__device__ __forceinline__ int32_t swar_cp(uint2 co) { return (int32_t)(int16_t)(co.x & 0xffffu); }

// Expands the image's 32-bit records into byte-parallel records.  Ends with a barrier.
__device__ inline void swar_load_instance(const SwarLds &L, const SaItem &a, int *cs) {
    const int n = a.n, D = a.D, T = blockDim.x, tid = threadIdx.x, Ds = swar_rec_stride(D);
    const int32_t *img = a.image;
    if (tid <= a.C) cs[tid] = img[3 + tid];
    const uint32_t *recs = reinterpret_cast<const uint32_t *>(img + kImgHeader + 3 * n);
    const uint32_t inv = (uint32_t)n * (uint32_t)a.qw;  // offset of ~S
    for (int idx = tid; idx < n * Ds; idx += T) {
        const int p = idx / Ds, k = idx - p * Ds;
        uint2 v = make_uint2(0u, 0u);  // padding: offset 0, weight 0
        if (k < D) {
            const uint32_t r = recs[(size_t)p * D + k];
            const int32_t J = (int32_t)(int16_t)(r & 0xffffu);
            const uint32_t off = (r >> 16) * (uint32_t)a.qw + (J < 0 ? inv : 0u);
            v = make_uint2(off, (uint32_t)(J < 0 ? -J : J) * 0x01010101u);
        }
        L.rec[idx] = v;
    }
    for (int p = tid; p < n; p += T) {
        int32_t s = 0;
        for (int k = 0; k < D; ++k) {
            const int32_t J = (int32_t)(int16_t)(recs[(size_t)p * D + k] & 0xffffu);
            s += J < 0 ? -J : J;
        }
        const int32_t h = img[kImgHeader + 2 * n + p];
        const uint32_t c16 = (uint32_t)(h - s) & 0xffffu;
        L.hpos[p] = h;
        L.co[p] = make_uint2(c16 | (c16 << 16), (uint32_t)img[kImgHeader + p]);
    }
    __syncthreads();
}

// Neighbour records are read this many at a time (loads issued together).
constexpr int kSwarBatch = 8;

// Per byte, the sum of |J_k| over the neighbours agreeing with sign(J_k); `rp` is
// the site's record block, `Sq` the spin words shifted to this lane's column.
// DK > 0: the record count is DK exactly (straight-line code); DK = 0: D at run time.
template <int DK>
__device__ __forceinline__ uint32_t swar_agree(const uint2 *__restrict__ rp, const uint32_t *__restrict__ Sq,
                                               int D) {
    if constexpr (DK > 0) {
        constexpr int U = (DK + 1) / 2;
        uint4 r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = reinterpret_cast<const uint4 *>(rp)[u];
        uint32_t w[DK];
#pragma unroll
        for (int k = 0; k < DK; ++k) w[k] = Sq[(k & 1) ? r[k / 2].z : r[k / 2].x];
        uint32_t P = 0;
#pragma unroll
        for (int k = 0; k < DK; ++k) P += w[k] & ((k & 1) ? r[k / 2].w : r[k / 2].y);
        return P;
    }
    uint32_t P = 0;
    for (int k0 = 0; k0 < D; k0 += kSwarBatch) {
        uint2 r[kSwarBatch];
#pragma unroll
        for (int u = 0; u < kSwarBatch; ++u)
            if (k0 + u < D) r[u] = rp[k0 + u];
        uint32_t w[kSwarBatch];
#pragma unroll
        for (int u = 0; u < kSwarBatch; ++u)
            if (k0 + u < D) w[u] = Sq[r[u].x];
#pragma unroll
        for (int u = 0; u < kSwarBatch; ++u)
            if (k0 + u < D) P += w[u] & r[u].y;
    }
    return P;
}

__device__ __forceinline__ void swar_store(uint32_t *S, uint32_t idx, uint32_t inv, uint32_t w) {
    S[idx] = w;
    S[idx + inv] = ~w;
}

typedef unsigned short swar_u16x2 __attribute__((ext_vector_type(2)));
typedef short swar_i16x2 __attribute__((ext_vector_type(2)));

// x = -s * f for the four replicas of a word, as two pairs of int16 (replicas 0, 1 and 2, 3):
// f = cp + 2 P_b fits 16 bits (|f| <= x_bound <= 255), and the spin byte masks, widened to
// 16 bits, negate it where the spin is +1.
__device__ __forceinline__ void swar_x16(uint32_t P, uint32_t self, uint32_t cp2, swar_i16x2 *lo, swar_i16x2 *hi) {
    const uint32_t Plo = __builtin_amdgcn_perm(P, P, 0x0C010C00u);  // bytes P0, 0, P1, 0
    const uint32_t Phi = __builtin_amdgcn_perm(P, P, 0x0C030C02u);  // bytes P2, 0, P3, 0
    const uint32_t mlo = __builtin_amdgcn_perm(self, self, 0x01010000u);
    const uint32_t mhi = __builtin_amdgcn_perm(self, self, 0x03030202u);
    const swar_u16x2 c = __builtin_bit_cast(swar_u16x2, cp2);
    const swar_u16x2 flo = __builtin_bit_cast(swar_u16x2, Plo) * (unsigned short)2 + c;
    const swar_u16x2 fhi = __builtin_bit_cast(swar_u16x2, Phi) * (unsigned short)2 + c;
    const swar_u16x2 ml = __builtin_bit_cast(swar_u16x2, mlo), mh = __builtin_bit_cast(swar_u16x2, mhi);
    *lo = __builtin_bit_cast(swar_i16x2, (swar_u16x2)((flo ^ ml) - ml));
    *hi = __builtin_bit_cast(swar_i16x2, (swar_u16x2)((fhi ^ mh) - mh));
}

template <int DK>
__device__ void swar_run(const SwarLds &L, const SaItem &a, const int *cs) {
    const int n = a.n, D = a.D, qw = a.qw, T = blockDim.x, tid = threadIdx.x;
    const int Ds = DK > 0 ? swar_rec_stride(DK) : swar_rec_stride(D);
    const int q0 = a.q0;
    const int q = tid % qw, slot = tid / qw, nslots = T / qw;
    const bool active = slot < nslots;
    const uint32_t inv = (uint32_t)n * (uint32_t)qw;
    const uint32_t *Sq = L.S + q;
    for (int k = tid; k < 2 * kSwarTabWords; k += T) {
        const int i = k % kSwarTabWords - kSwarTabHalf;
        L.tab[k] = (i >= 0 && k < kSwarTabWords && i < a.row_len) ? a.tables[i] : 0xFFFFFFFFu;
    }
    for (int k = tid; k < 4 * qw; k += T) L.E2[k] = 0ull;
    if (a.init == nullptr) {
        for (int p = slot; active && p < n; p += nslots) {
            const dev::Words4 w =
                dev::philox(L.co[p].y, 0u, (uint32_t)(q0 + q), 1u << 24, a.k0, a.k1);
            uint32_t word = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) word |= ((w.w[b] >> 31) ? 0xFFu : 0x00u) << (8 * b);
            swar_store(L.S, (uint32_t)p * (uint32_t)qw + (uint32_t)q, inv, word);
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

    // One sweep reading table buffer B (a compile-time constant) and filling the other.
    auto sweep = [&](auto buf, int ls) {
        constexpr int B = decltype(buf)::value;
        const uint32_t t = a.sweep_offset + (uint32_t)ls;
        const char *tz = reinterpret_cast<const char *>(L.tab + B * kSwarTabWords + kSwarTabHalf);
        if (ls + 1 < a.sweeps) {
            uint32_t *tnext = L.tab + (1 - B) * kSwarTabWords + kSwarTabHalf;
            for (int k = tid; k < a.row_len; k += T) tnext[k] = a.tables[(size_t)(ls + 1) * a.row_len + k];
        }
        for (int c = 0; c < a.C; ++c) {
            const int pe = cs[c + 1];
            for (int p = cs[c] + slot; active && p < pe; p += nslots) {
                const uint32_t at = (uint32_t)p * (uint32_t)qw + (uint32_t)q;
                const uint32_t self = L.S[at];
                const uint32_t P = swar_agree<DK>(L.rec + (uint32_t)p * (uint32_t)Ds, Sq, D);
                const uint2 co = L.co[p];
                swar_i16x2 xlo, xhi;
                swar_x16(P, self, co.x, &xlo, &xhi);
                const swar_i16x2 xm = __builtin_elementwise_max(xlo, xhi);
                uint32_t mask = 0xFFFFFFFFu;
                if (xm.x > 0 || xm.y > 0) {
                    const dev::Words4 r = dev::philox(co.y, t, (uint32_t)(q0 + q), 2u << 24, a.k0, a.k1);
                    // byte offsets 4x into the row (x may be <= 0: the entry is read and ignored)
                    const swar_i16x2 olo = xlo << (short)2, ohi = xhi << (short)2;
                    const int32_t o[4] = {olo.x, olo.y, ohi.x, ohi.y};
                    uint32_t th[4];
#pragma unroll
                    for (int b = 0; b < 4; ++b) th[b] = *reinterpret_cast<const uint32_t *>(tz + o[b]);
                    mask = 0;
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        mask |= (uint32_t)((o[b] <= 0) | (r.w[b] < th[b])) * (0xFFu << (8 * b));
                }
                if (mask) swar_store(L.S, at, inv, self ^ mask);
            }
            __syncthreads();
        }
    };
    for (int ls = 0; ls < a.sweeps; ls += 2) {
        sweep(std::integral_constant<int, 0>{}, ls);
        if (ls + 1 < a.sweeps) sweep(std::integral_constant<int, 1>{}, ls + 1);
    }

    {
        long long e2[4] = {0, 0, 0, 0};
        for (int p = slot; active && p < n; p += nslots) {
            const uint32_t self = L.S[(size_t)p * qw + q];
            const uint32_t P = swar_agree<DK>(L.rec + (uint32_t)p * (uint32_t)Ds, Sq, D);
            const long long cp = swar_cp(L.co[p]);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const long long f = cp + 2 * (long long)((P >> (8 * b)) & 0xffu);
                const long long s = ((self >> (8 * b)) & 0xffu) ? 1 : -1;
                e2[b] += s * ((long long)L.hpos[p] + f);
            }
        }
        if (active)
#pragma unroll
            for (int b = 0; b < 4; ++b) atomicAdd(&L.E2[q * 4 + b], (unsigned long long)e2[b]);
    }
    __syncthreads();
    for (int rl = tid; rl < 4 * qw; rl += T) {
        const int r = 4 * q0 + rl;
        if (r < a.reads) a.energies[r] = ((long long)L.E2[rl]) / 2;
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

}  // namespace core
}  // namespace spv
