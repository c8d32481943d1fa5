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

#include "device.hpp"
#include "internal.hpp"
#include "sa_core.hpp"

namespace spv {
namespace core {

struct SwarLds {
    uint2 *rec;      // [D][n]: {offset of the neighbour row in S or ~S, |J| x 0x01010101}
    int32_t *cpos;   // [n] h_p - sum_k |J_pk|
    int32_t *hpos;   // [n]
    int32_t *ord;    // [n]
    uint32_t *tab;   // [2][row_len]
    uint32_t *S;     // [2][n][qw]: spins, then their complements
    unsigned long long *E2;  // [4*qw]
};

__host__ __device__ inline size_t swar_layout(int n, int D, int row_len, int qw, SwarLds *L,
                                              unsigned char *base, int e2q = 0) {
    if (e2q < qw) e2q = qw;
    size_t o_rec = 0;
    size_t o_c = o_rec + (size_t)n * D * 8;
    size_t o_h = o_c + (size_t)n * 4;
    size_t o_ord = o_h + (size_t)n * 4;
    size_t o_tab = o_ord + (size_t)n * 4;
    size_t o_S = o_tab + (size_t)2 * row_len * 4;
    size_t o_E = (o_S + (size_t)2 * n * qw * 4 + 7) & ~(size_t)7;
    size_t end = o_E + (size_t)4 * e2q * 8;
    if (L) {
        L->rec = reinterpret_cast<uint2 *>(base + o_rec);
        L->cpos = reinterpret_cast<int32_t *>(base + o_c);
        L->hpos = reinterpret_cast<int32_t *>(base + o_h);
        L->ord = reinterpret_cast<int32_t *>(base + o_ord);
        L->tab = reinterpret_cast<uint32_t *>(base + o_tab);
        L->S = reinterpret_cast<uint32_t *>(base + o_S);
        L->E2 = reinterpret_cast<unsigned long long *>(base + o_E);
    }
    return end;
}

// Expands the image's 32-bit records into byte-parallel records.  Ends with a barrier.
__device__ inline void swar_load_instance(const SwarLds &L, const SaItem &a, int *cs) {
    const int n = a.n, D = a.D, T = blockDim.x, tid = threadIdx.x;
    const int32_t *img = a.image;
    if (tid <= a.C) cs[tid] = img[3 + tid];
    const uint32_t *recs = reinterpret_cast<const uint32_t *>(img + kImgHeader + 3 * n);
    const uint32_t inv = (uint32_t)n * (uint32_t)a.qw;  // offset of ~S
    for (int idx = tid; idx < n * D; idx += T) {
        const int p = idx / D, k = idx - p * D;
        const uint32_t r = recs[idx];
        const int32_t J = (int32_t)(int16_t)(r & 0xffffu);
        const uint32_t off = (r >> 16) * (uint32_t)a.qw + (J < 0 ? inv : 0u);
        L.rec[(size_t)k * n + p] = make_uint2(off, (uint32_t)(J < 0 ? -J : J) * 0x01010101u);
    }
    for (int p = tid; p < n; p += T) {
        int32_t s = 0;
        for (int k = 0; k < D; ++k) {
            const int32_t J = (int32_t)(int16_t)(recs[(size_t)p * D + k] & 0xffffu);
            s += J < 0 ? -J : J;
        }
        const int32_t h = img[kImgHeader + 2 * n + p];
        L.hpos[p] = h;
        L.cpos[p] = h - s;
        L.ord[p] = img[kImgHeader + p];
    }
    __syncthreads();
}

// Neighbour records are read this many at a time (loads issued together).
constexpr int kSwarBatch = 8;

// Per byte, the sum of |J_k| over the neighbours agreeing with sign(J_k).
// DK > 0: the record count is DK exactly (straight-line code); DK = 0: D at run time.
template <int DK>
__device__ __forceinline__ uint32_t swar_agree(const uint2 *__restrict__ rec, const uint32_t *__restrict__ S,
                                               int D, int q, int n) {
    if constexpr (DK > 0) {
        uint2 r[DK];
#pragma unroll
        for (int u = 0; u < DK; ++u) r[u] = rec[(uint32_t)u * (uint32_t)n];
        uint32_t w[DK];
#pragma unroll
        for (int u = 0; u < DK; ++u) w[u] = S[r[u].x + q];
        uint32_t P = 0;
#pragma unroll
        for (int u = 0; u < DK; ++u) P += w[u] & r[u].y;
        return P;
    }
    // 32-bit indices: LDS addresses are 32-bit, wider index arithmetic only costs VALU
    uint32_t P = 0;
    for (int k0 = 0; k0 < D; k0 += kSwarBatch) {
        uint2 r[kSwarBatch];
#pragma unroll
        for (int u = 0; u < kSwarBatch; ++u)
            if (k0 + u < D) r[u] = rec[(uint32_t)(k0 + u) * (uint32_t)n];
        uint32_t w[kSwarBatch];
#pragma unroll
        for (int u = 0; u < kSwarBatch; ++u)
            if (k0 + u < D) w[u] = S[r[u].x + q];
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

template <int DK>
__device__ void swar_run(const SwarLds &L, const SaItem &a, const int *cs) {
    const int n = a.n, D = a.D, qw = a.qw, T = blockDim.x, tid = threadIdx.x;
    const int q0 = a.q0;
    const int q = tid % qw, slot = tid / qw, nslots = T / qw;
    const bool active = slot < nslots;
    const uint32_t inv = (uint32_t)n * (uint32_t)qw;
    for (int k = tid; k < a.row_len; k += T) L.tab[k] = a.tables[k];
    for (int k = tid; k < 4 * qw; k += T) L.E2[k] = 0ull;
    if (a.init == nullptr) {
        for (int p = slot; active && p < n; p += nslots) {
            const dev::Words4 w =
                dev::philox((uint32_t)L.ord[p], 0u, (uint32_t)(q0 + q), 1u << 24, a.k0, a.k1);
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

    for (int ls = 0; ls < a.sweeps; ++ls) {
        const uint32_t t = a.sweep_offset + (uint32_t)ls;
        const uint32_t *tcur = L.tab + (ls & 1) * a.row_len;
        if (ls + 1 < a.sweeps) {
            uint32_t *tnext = L.tab + ((ls + 1) & 1) * a.row_len;
            for (int k = tid; k < a.row_len; k += T) tnext[k] = a.tables[(size_t)(ls + 1) * a.row_len + k];
        }
        for (int c = 0; c < a.C; ++c) {
            const int pe = cs[c + 1];
            for (int p = cs[c] + slot; active && p < pe; p += nslots) {
                const uint32_t at = (uint32_t)p * (uint32_t)qw + (uint32_t)q;
                const uint32_t self = L.S[at];
                const uint32_t P = swar_agree<DK>(L.rec + p, L.S, D, q, n);
                const int32_t cp = L.cpos[p];
                int32_t x[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int32_t f = cp + 2 * (int32_t)((P >> (8 * b)) & 0xffu);
                    const int32_t m = ((int32_t)(self << (24 - 8 * b))) >> 24;  // -1 for +1 spins
                    x[b] = (f ^ m) - m;
                }
                const int32_t xm = max(max(x[0], x[1]), max(x[2], x[3]));
                uint32_t mask = 0xFFFFFFFFu;
                if (xm > 0) {
                    const dev::Words4 r =
                        dev::philox((uint32_t)L.ord[p], t, (uint32_t)(q0 + q), 2u << 24, a.k0, a.k1);
                    // branch-free: the row is read at max(x, 0), a valid index, for every byte
                    uint32_t th[4];
#pragma unroll
                    for (int b = 0; b < 4; ++b) th[b] = tcur[max(x[b], 0)];
                    mask = 0;
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        mask |= (uint32_t)((x[b] <= 0) | (r.w[b] < th[b])) * (0xFFu << (8 * b));
                }
                if (mask) swar_store(L.S, at, inv, self ^ mask);
            }
            __syncthreads();
        }
    }

    {
        long long e2[4] = {0, 0, 0, 0};
        for (int p = slot; active && p < n; p += nslots) {
            const uint32_t self = L.S[(size_t)p * qw + q];
            const uint32_t P = swar_agree<DK>(L.rec + p, L.S, D, q, n);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const long long f = (long long)L.cpos[p] + 2 * (long long)((P >> (8 * b)) & 0xffu);
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
