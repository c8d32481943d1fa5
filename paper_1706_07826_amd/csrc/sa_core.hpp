// Device body of the simulated-annealing sweep, shared by the one-instance
// launch (sa.hip) and the batched persistent launch (batch.hip).
//
// Sampler (Sec. III.A, "SA"): every read starts from its own Philox state (or
// a caller state) and performs one Metropolis sweep per entry of the beta
// schedule; the sample is the final state of every read.  A sweep visits the
// colour classes in order; a class is an independent set, so all of its spins
// are updated in parallel with the same result as any sequential order.
//
// LDS holds the position-ordered instance (ELL records: neighbour position <<
// 16 | int16 coupling), two threshold rows (current sweep and next sweep) and
// the spins as S[p][q]: one 32-bit word per (position, quad of 4 replicas), a
// signed byte per replica.  A thread keeps one quad q for the whole schedule;
// for each position it forms the four local fields, draws one Philox block
// that serves the four replicas and applies the integer threshold test.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"
#include "lds_shadow.hpp"
#include "internal.hpp"

namespace spv {
namespace core {

struct SaLds {
    uint32_t *nbr;
    int32_t *hpos;
    int32_t *ord;
    uint32_t *tab;  // [2][row_len]
    uint32_t *S;    // [n][qw]
    unsigned long long *E2;  // [4*qw]
};

// LDS layout for n positions, D records each, quads `qw` (spin capacity n*qw
// words) and energy accumulators for e2q quads (0: qw).
__host__ __device__ inline size_t sa_layout(int n, int D, int row_len, int qw, SaLds *L,
                                            unsigned char *base, int e2q = 0) {
    if (e2q < qw) e2q = qw;
    size_t o_nbr = 0;
    size_t o_h = o_nbr + (size_t)n * D * 4;
    size_t o_ord = o_h + (size_t)n * 4;
    size_t o_tab = o_ord + (size_t)n * 4;
    size_t o_S = o_tab + (size_t)2 * row_len * 4;
    size_t o_E = (o_S + (size_t)n * qw * 4 + 7) & ~(size_t)7;
    size_t end = o_E + (size_t)4 * e2q * 8;
    if (L) {
        L->nbr = reinterpret_cast<uint32_t *>(base + o_nbr);
        L->hpos = reinterpret_cast<int32_t *>(base + o_h);
        L->ord = reinterpret_cast<int32_t *>(base + o_ord);
        L->tab = reinterpret_cast<uint32_t *>(base + o_tab);
        L->S = reinterpret_cast<uint32_t *>(base + o_S);
        L->E2 = reinterpret_cast<unsigned long long *>(base + o_E);
    }
    return end;
}

// Layout when the instance stays in global memory (too large for the LDS beside
// the spins): LDS holds the two threshold rows, the spins and the accumulators.
__host__ __device__ inline size_t sa_big_layout(int n, int row_len, int qw, SaLds *L,
                                                unsigned char *base) {
    size_t o_tab = 0;
    size_t o_S = o_tab + (size_t)2 * row_len * 4;
    size_t o_E = (o_S + (size_t)n * qw * 4 + 7) & ~(size_t)7;
    size_t end = o_E + (size_t)4 * qw * 8;
    if (L) {
        L->nbr = nullptr;
        L->hpos = nullptr;
        L->ord = nullptr;
        L->tab = reinterpret_cast<uint32_t *>(base + o_tab);
        L->S = reinterpret_cast<uint32_t *>(base + o_S);
        L->E2 = reinterpret_cast<unsigned long long *>(base + o_E);
    }
    return end;
}

// One schedule over quads [q0, q0 + qw) of one instance.
struct SaItem {
    const int32_t *image;
    const uint32_t *tables;  // [sweeps][row_len]
    const int8_t *init;      // [reads][n] or null
    int8_t *out;             // [reads][n]
    int64_t *energies;       // [reads]
    int n, D, C, row_len, sweeps, reads, q0, qw;
    uint32_t sweep_offset, k0, k1;
    int wpl = 1;  // byte-parallel body: quad words per lane (1, or 2 when qw = 2)
    unsigned char *big = nullptr;  // byte-parallel body: instance in global memory (too large for LDS)
};

struct Fields {
    int32_t f[4];
};

// f_b = h_p + sum_k J_k s_kb for the four replicas of quad q at position p;
// nb points at record 0 of p, consecutive records `stride` apart.
__device__ __forceinline__ Fields local_fields(const uint32_t *__restrict__ nb,
                                               const uint32_t *__restrict__ S, int D, int qw,
                                               int q, int32_t hv, size_t stride) {
    Fields F;
#pragma unroll
    for (int b = 0; b < 4; ++b) F.f[b] = hv;
    for (int k = 0; k < D; ++k) {
        const uint32_t rec = nb[k * stride];
        const int32_t Jv = (int32_t)(int16_t)(rec & 0xffffu);
        const uint32_t w = S[__umul24(rec >> 16, (uint32_t)qw) + q];
#pragma unroll
        for (int b = 0; b < 4; ++b) F.f[b] += Jv * dev::spin_of(w, b);
    }
    return F;
}

// Xor mask (0xFE per accepted byte) of the Metropolis decisions for x[b] = -s f: a
// byte is accepted iff every nonzero digit of x passes its threshold (x <= 0 has
// none).  The first digit's block is drawn without a branch (some byte of a word
// almost always has a nonzero first digit), so the decisions stay lane masks; a
// later digit's block is drawn where some byte has that digit nonzero (a byte
// already rejected stays rejected, so testing it again changes nothing).
// Thresholds are loaded for every byte (a zero digit reads a valid entry it
// ignores), so the four LDS reads overlap the Philox block.
template <int ND>
__device__ __forceinline__ uint32_t metropolis_mask(const int32_t x[4], const uint32_t *tab,
                                                    uint32_t i, uint32_t t, uint32_t quad,
                                                    uint32_t k0, uint32_t k1) {
    uint32_t d[4], th[4], mask = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        d[b] = x[b] > 0 ? ((uint32_t)x[b] & (kDigitSize - 1)) : 0u;
        th[b] = tab[d[b]];
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
            th[b] = tab[j * kDigitSize + d[b]];
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

// Points the instance fields at the image in global memory (records position-major:
// record k of position p at nbr[p * D + k]) and loads the colour-class starts.
// Ends with a barrier.
__device__ inline void sa_bind_image(SaLds *L, const SaItem &a, int *cs) {
    const int32_t *img = a.image;
    const int n = a.n;
    if ((int)threadIdx.x <= a.C) cs[threadIdx.x] = img[3 + threadIdx.x];
    L->ord = const_cast<int32_t *>(img + kImgHeader);
    L->hpos = const_cast<int32_t *>(img + kImgHeader + 2 * n);
    L->nbr = reinterpret_cast<uint32_t *>(const_cast<int32_t *>(img + kImgHeader + 3 * n));
    __syncthreads();
}

// Copies the instance image into LDS (ELL records, biases, order).  Ends with a barrier.
__device__ inline void sa_load_instance(const SaLds &L, const SaItem &a, int *cs) {
    const int n = a.n, D = a.D, T = blockDim.x, tid = threadIdx.x;
    const int32_t *img = a.image;
    if (tid <= a.C) cs[tid] = img[3 + tid];
    const uint32_t *recs = reinterpret_cast<const uint32_t *>(img + kImgHeader + 3 * n);
    for (int idx = tid; idx < n * D; idx += T) {  // neighbour-major in LDS: nbr[k][p]
        const int p = idx / D, k = idx - p * D;
        L.nbr[(size_t)k * n + p] = recs[idx];
    }
    for (int k = tid; k < n; k += T) {
        L.hpos[k] = img[kImgHeader + 2 * n + k];
        L.ord[k] = img[kImgHeader + k];
    }
    __syncthreads();
}

// The whole schedule for quads [q0, q0+qw) of an instance resident in LDS
// (neighbour-major records), or in global memory when BIG (position-major).
// Starts and ends with a barrier, so LDS can be reused by the caller.
template <int ND, bool BIG = false>
__device__ void sa_run(const SaLds &L, const SaItem &a, const int *cs) {
    const int n = a.n, D = a.D, qw = a.qw, T = blockDim.x, tid = threadIdx.x;
    const int q0 = a.q0;
    const size_t rec_p = BIG ? (size_t)D : 1, rec_k = BIG ? 1 : (size_t)n;
    const int q = tid % qw, slot = tid / qw, nslots = T / qw;
    const bool active = slot < nslots;
    // (no sweeps: no table was uploaded, so none is read)
    for (int k = tid; a.sweeps > 0 && k < a.row_len; k += T) L.tab[k] = a.tables[k];
    for (int k = tid; k < 4 * qw; k += T) L.E2[k] = 0ull;
    // Initial state.
    if (a.init == nullptr) {
        for (int p = slot; active && p < n; p += nslots) {
            const dev::Words4 w =
                dev::philox((uint32_t)L.ord[p], 0u, (uint32_t)(q0 + q), 1u << 24, a.k0, a.k1);
            uint32_t word = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) word |= ((w.w[b] >> 31) ? 0x01u : 0xFFu) << (8 * b);
            L.S[(size_t)p * qw + q] = word;
        }
    } else {
        const int32_t *pos_of = a.image + kImgHeader + n;
        unsigned char *Sb = reinterpret_cast<unsigned char *>(L.S);
        for (int idx = tid; idx < 4 * qw * n; idx += T) {
            const int rl = idx / n, i = idx - rl * n;
            const int r = 4 * q0 + rl;
            int8_t v = 1;
            if (r < a.reads) v = a.init[(size_t)r * n + i] > 0 ? 1 : -1;
            const int p = pos_of[i];
            Sb[((size_t)p * qw + (rl >> 2)) * 4 + (rl & 3)] = (unsigned char)v;
        }
    }
    __syncthreads();
    const shadow::Pass sh = shadow::begin((uint32_t)n * (uint32_t)qw);
    // Debug build: the class pass's writes, then its neighbour reads, against the bitmap.
    auto shadow_pass = [&](int c, bool before) {
        const int pe = cs[c + 1];
        if (before) {
            for (int p = cs[c] + slot; active && p < pe; p += nslots) shadow::mark(sh, (uint32_t)(p * qw + q));
            shadow::barrier();
            for (int p = cs[c] + slot; active && p < pe; p += nslots)
                for (int k = 0; k < D; ++k) {
                    const uint32_t r = L.nbr[(size_t)p * rec_p + (size_t)k * rec_k];
                    if ((r & 0xffffu) == 0u) continue;  // padding or J = 0: the value read is unused
                    shadow::check(sh, (r >> 16) * (uint32_t)qw + (uint32_t)q);
                }
            shadow::count_pass(sh);
        } else {
            for (int p = cs[c] + slot; active && p < pe; p += nslots) shadow::unmark(sh, (uint32_t)(p * qw + q));
            shadow::barrier();
        }
    };

    for (int ls = 0; ls < a.sweeps; ++ls) {
        const uint32_t t = a.sweep_offset + (uint32_t)ls;
        const uint32_t *tcur = L.tab + (ls & 1) * a.row_len;
        uint32_t *tnext = L.tab + ((ls + 1) & 1) * a.row_len;
        if (ls + 1 < a.sweeps)
            for (int k = tid; k < a.row_len; k += T)
                tnext[k] = a.tables[(size_t)(ls + 1) * a.row_len + k];
        for (int c = 0; c < a.C; ++c) {
            if constexpr (shadow::kOn) shadow_pass(c, true);
            const int pe = cs[c + 1];
            for (int p = cs[c] + slot; active && p < pe; p += nslots) {
                const uint32_t self = L.S[(size_t)p * qw + q];
                const Fields F = local_fields(L.nbr + p * rec_p, L.S, D, qw, q, L.hpos[p], rec_k);
                int32_t x[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) x[b] = dev::spin_of(self, b) > 0 ? -F.f[b] : F.f[b];
                const uint32_t mask = metropolis_mask<ND>(x, tcur, (uint32_t)L.ord[p], t,
                                                          (uint32_t)(q0 + q), a.k0, a.k1);
                if (mask) L.S[(size_t)p * qw + q] = self ^ mask;
            }
            __syncthreads();
            if constexpr (shadow::kOn) shadow_pass(c, false);
        }
    }

    // Energies: 2E = sum_p s_p (h_p + f_p) per replica.
    {
        long long e2[4] = {0, 0, 0, 0};
        for (int p = slot; active && p < n; p += nslots) {
            const uint32_t self = L.S[(size_t)p * qw + q];
            const Fields F = local_fields(L.nbr + p * rec_p, L.S, D, qw, q, L.hpos[p], rec_k);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                e2[b] += (long long)dev::spin_of(self, b) * ((long long)L.hpos[p] + F.f[b]);
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
    // Spins, transposed back to [read][variable] in original variable order.
    const int32_t *pos_of = a.image + kImgHeader + n;
    const unsigned char *Sb = reinterpret_cast<const unsigned char *>(L.S);
    for (int idx = tid; idx < 4 * qw * n; idx += T) {
        const int rl = idx / n, i = idx - rl * n;
        const int r = 4 * q0 + rl;
        if (r < a.reads) {
            const int p = pos_of[i];
            a.out[(size_t)r * n + i] = (int8_t)Sb[((size_t)p * qw + (rl >> 2)) * 4 + (rl & 3)];
        }
    }
    __syncthreads();
}

}  // namespace core
}  // namespace spv
