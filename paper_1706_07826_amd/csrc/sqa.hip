// Simulated quantum annealing (Sec. III, "SQA": discrete-time path-integral
// Monte Carlo of the transverse-field Ising model over P Trotter slices, the
// Suzuki-Trotter mapping of Martonak, Santoro and Tosatti, PRB 66, 094203).
//
// One workgroup per read.  LDS holds the position-ordered instance (the same
// ELL image as the general SA body; read from global memory instead when it
// does not fit beside the slices), the acceptance rows of this sweep and the
// next (beta_t / P) and the read's P slices as P/4 words per site: slice
// k = 2m + parity lives in word parity * P/8 + m/4, byte m % 4, so a word holds
// four slices of one parity.  A sweep visits the colour classes in order and,
// inside a class, the even-slice words and then the odd-slice words: every
// update in such a pass reads only words the pass does not write (the
// neighbouring sites of the class are in other classes, the neighbouring slices
// have the other parity), and one Philox block serves the four slices of a word.
//
// Update of slice k at site i: g = f_i(s^k) - Jp_t (s^{k-1}_i + s^{k+1}_i) over
// the slice ring, x = -s g, accepted iff x <= 0 or every nonzero base-512 digit
// of x passes its threshold; the random words are Philox(i, t, quad, 6 << 24 |
// digit)[byte], quad = read * P/4 + word.  After the last sweep the read's
// sample is its lowest-energy slice (ties: lowest k).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "internal.hpp"
#include "lds_shadow.hpp"
#include "sa_core.hpp"
#include "swar_core.hpp"

namespace spv {

namespace {

constexpr uint32_t kTagSqa = 6u;

struct SqaArgs {
    const int32_t *image;
    const uint32_t *tables;  // [sweeps][row_len], thresholds for beta_t / P
    const int32_t *jp;       // [sweeps] inter-slice coupling, integer units
    int8_t *out;             // [reads][n]
    int64_t *energies;       // [reads]
    int n, D, C, row_len, sweeps, reads, P, x_bound;
    uint32_t k0, k1;
};

// Xor mask (0xFE per accepted byte) of the digit tests for x[b] (slice tag); digits
// from ndt on are zero for every x of this sweep (ndt is wave-uniform).  A byte is
// accepted iff every nonzero digit of x passes (x <= 0 has none).  The first digit's
// block is drawn without a branch (some byte of a word almost always has a nonzero
// first digit); a later digit's block is drawn where some byte has that digit nonzero
// (a byte already rejected stays rejected, so testing it again changes nothing).
template <int ND>
__device__ __forceinline__ uint32_t sqa_mask(const int32_t x[4], const uint32_t *tab, uint32_t i, uint32_t t,
                                             uint32_t quad, uint32_t k0, uint32_t k1, int ndt) {
    uint32_t d[4], th[4], mask = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        d[b] = x[b] > 0 ? ((uint32_t)x[b] & (kDigitSize - 1)) : 0u;
        th[b] = tab[d[b]];  // a zero digit reads a valid entry it ignores
    }
    {
        const dev::Words4 w = dev::philox(i, t, quad, kTagSqa << 24, k0, k1);
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if ((d[b] == 0) | (w.w[b] < th[b])) mask |= 0xFEu << (8 * b);
    }
#pragma unroll
    for (int j = 1; j < ND; ++j) {
        if (j >= ndt) break;
        bool need = false;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            d[b] = x[b] > 0 ? (((uint32_t)x[b] >> (kDigitBits * j)) & (kDigitSize - 1)) : 0u;
            need |= d[b] != 0;
            th[b] = tab[j * kDigitSize + d[b]];
        }
        if (need) {
            const dev::Words4 w = dev::philox(i, t, quad, (kTagSqa << 24) | (uint32_t)j, k0, k1);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if ((d[b] != 0) & (w.w[b] >= th[b])) mask &= ~(0xFEu << (8 * b));
        }
    }
    return mask;
}

// Classical fields of the four slices of one word from records expanded for the
// slice rows: record k of a position holds the LDS byte address of its neighbour's
// row of slice words and J sign-extended, so a neighbour costs one 8-byte read, one
// add and the four multiply-adds.  `w4` is the word's byte offset in a row.
__device__ __forceinline__ core::Fields sqa_fields(const uint2 *__restrict__ nb, int n, int D, uint32_t w4,
                                                   int32_t hv) {
    core::Fields F;
#pragma unroll
    for (int b = 0; b < 4; ++b) F.f[b] = hv;
    for (int k = 0; k < D; ++k) {
        const uint2 r = nb[(size_t)k * n];
        const uint32_t s = core::swar_ld32(r.x + w4);
        const int32_t J = (int32_t)r.y;
#pragma unroll
        for (int b = 0; b < 4; ++b) F.f[b] += __mul24(J, dev::spin_of(s, b));  // |J| < 2^15
    }
    return F;
}

// BIG: the instance stays in the global image (position-major records), LDS holds
// the acceptance rows and the slices only.
template <int ND, bool BIG = false>
__global__ __launch_bounds__(1024) void sqa_kernel(SqaArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cs[kMaxColours + 1];
    __shared__ int best_s;
    __shared__ long long bestE_s;
    const int n = a.n, D = a.D, P = a.P, qw = P / 4, G8 = P / 8, T = blockDim.x, tid = threadIdx.x;
    const int read = blockIdx.x;
    core::SaItem it;
    it.image = a.image;
    it.n = n;
    it.D = D;
    it.C = a.C;
    core::SaLds L;
    if constexpr (BIG) {
        core::sa_big_layout(n, a.row_len, qw, &L, smem);
        core::sa_bind_image(&L, it, cs);  // ends with a barrier
    } else {
        // the record area holds n * D expanded records of two words each
        core::sa_layout(n, 2 * D, a.row_len, qw, &L, smem);
        if (tid <= a.C) cs[tid] = a.image[3 + tid];
        const uint32_t *recs = reinterpret_cast<const uint32_t *>(a.image + kImgHeader + 3 * n);
        uint2 *nb2 = reinterpret_cast<uint2 *>(L.nbr);
        const uint32_t sb = core::swar_lds_addr(L.S), row_bytes = 4u * (uint32_t)qw;
        for (int idx = tid; idx < n * D; idx += T) {  // neighbour-major: record k of p at [k * n + p]
            const int p = idx / D, k = idx - p * D;
            const uint32_t r = recs[idx];
            nb2[(size_t)k * n + p] = make_uint2(sb + (r >> 16) * row_bytes, (uint32_t)(int32_t)(int16_t)(r & 0xffffu));
        }
        for (int k = tid; k < n; k += T) {
            L.hpos[k] = a.image[kImgHeader + 2 * n + k];
            L.ord[k] = a.image[kImgHeader + k];
        }
        __syncthreads();
    }
    const uint2 *const nb2 = reinterpret_cast<const uint2 *>(L.nbr);
    // record k of position p: nbr[p * rec_p + k * rec_k]
    const size_t rec_p = BIG ? (size_t)D : 1, rec_k = BIG ? 1 : (size_t)n;
    const uint32_t quad0 = (uint32_t)read * (uint32_t)qw;
    for (int k = tid; a.sweeps > 0 && k < a.row_len; k += T) L.tab[k] = a.tables[k];  // none uploaded without sweeps
    for (int k = tid; k < 4 * qw; k += T) L.E2[k] = 0ull;
    // Initial slices: replica r = read * P + parity * P/2 + m, i.e. quad quad0 + word.
    for (int idx = tid; idx < n * qw; idx += T) {
        const int p = idx / qw, w = idx - p * qw;
        const dev::Words4 r = dev::philox((uint32_t)L.ord[p], 0u, quad0 + (uint32_t)w, 1u << 24, a.k0, a.k1);
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) word |= ((r.w[b] >> 31) ? 0x01u : 0xFFu) << (8 * b);
        L.S[idx] = word;
    }
    __syncthreads();

    const int q = tid % G8, slot = tid / G8, nslots = T / G8;
    const bool active = slot < nslots;
    // Race-detection build: each (class, parity) pass's slice-word writes, then its
    // reads (the ring neighbours' words of the other parity and the classical
    // neighbours' words), against the LDS bitmap.
    const shadow::Pass sh = shadow::begin((uint32_t)n * (uint32_t)qw);
    auto shadow_pass = [&](int c, int par, bool before) {
        const int pe = cs[c + 1], w = par * G8 + q;
        const int wa = par ? q : G8 + q;
        const int wb = par ? (q + 1 == G8 ? 0 : q + 1) : G8 + (q == 0 ? G8 - 1 : q - 1);
        if (before) {
            for (int p = cs[c] + slot; active && p < pe; p += nslots) shadow::mark(sh, (uint32_t)(p * qw + w));
            shadow::barrier();
            for (int p = cs[c] + slot; active && p < pe; p += nslots) {
                shadow::check(sh, (uint32_t)(p * qw + wa));
                shadow::check(sh, (uint32_t)(p * qw + wb));
                for (int k = 0; k < D; ++k) {
                    if constexpr (BIG) {
                        const uint32_t rec = L.nbr[(size_t)p * rec_p + (size_t)k * rec_k];
                        if ((rec & 0xffffu) != 0u) shadow::check(sh, (rec >> 16) * (uint32_t)qw + (uint32_t)w);
                    } else {
                        const uint2 r = nb2[(size_t)k * n + p];
                        if (r.y != 0u) shadow::check(sh, (r.x - core::swar_lds_addr(L.S)) / 4u + (uint32_t)w);
                    }
                }
            }
            shadow::count_pass(sh);
        } else {
            for (int p = cs[c] + slot; active && p < pe; p += nslots) shadow::unmark(sh, (uint32_t)(p * qw + w));
            shadow::barrier();
        }
    };
    for (int ls = 0; ls < a.sweeps; ++ls) {
        const uint32_t t = (uint32_t)ls;
        const int32_t jp = a.jp[ls];
        // digits that |x| <= x_bound + 2 Jp can have in this sweep
        const int64_t xmax = (int64_t)a.x_bound + 2 * (int64_t)jp;
        int ndt = 1;
        while (ndt < ND && (xmax >> (kDigitBits * ndt)) != 0) ++ndt;
        const uint32_t *tcur = L.tab + (ls & 1) * a.row_len;
        uint32_t *tnext = L.tab + ((ls + 1) & 1) * a.row_len;
        if (ls + 1 < a.sweeps)
            for (int k = tid; k < a.row_len; k += T) tnext[k] = a.tables[(size_t)(ls + 1) * a.row_len + k];
        for (int c = 0; c < a.C; ++c) {
            const int pe = cs[c + 1];
#pragma unroll 1
            for (int par = 0; par < 2; ++par) {
                if constexpr (shadow::kOn) shadow_pass(c, par, true);
                const int w = par * G8 + q;
                // words of the other parity holding slices k - 1 and k + 1
                const int wa = par ? q : G8 + q;
                const int wb = par ? (q + 1 == G8 ? 0 : q + 1) : G8 + (q == 0 ? G8 - 1 : q - 1);
                for (int p = cs[c] + slot; active && p < pe; p += nslots) {
                    const uint32_t *row = L.S + (size_t)p * qw;
                    const uint32_t self = row[w], A = row[wa], B = row[wb];
                    core::Fields F;
                    if constexpr (BIG)
                        F = core::local_fields(L.nbr + p * rec_p, L.S, D, qw, w, L.hpos[p], rec_k);
                    else
                        F = sqa_fields(nb2 + p, n, D, 4u * (uint32_t)w, L.hpos[p]);
                    // even word: k-1 = odd slice m-1 (A byte b-1, or B byte 3), k+1 = odd slice m (A byte b);
                    // odd word: k-1 = even slice m (A byte b), k+1 = even slice m+1 (A byte b+1, or B byte 0)
                    const uint32_t up = par ? A : __builtin_amdgcn_alignbyte(A, B, 3);
                    const uint32_t dn = par ? __builtin_amdgcn_alignbyte(B, A, 1) : A;
                    int32_t x[4];
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int32_t g = F.f[b] - jp * (dev::spin_of(up, b) + dev::spin_of(dn, b));  // full 32-bit product: Jp <= 2^24
                        x[b] = dev::spin_of(self, b) > 0 ? -g : g;
                    }
                    const uint32_t mask =
                        sqa_mask<ND>(x, tcur, (uint32_t)L.ord[p], t, quad0 + (uint32_t)w, a.k0, a.k1, ndt);
                    if (mask) L.S[(size_t)p * qw + w] = self ^ mask;
                }
                __syncthreads();
                if constexpr (shadow::kOn) shadow_pass(c, par, false);
            }
        }
    }

    // Classical energy of every slice: 2E = sum_p s_p (h_p + f_p).
    {
        for (int idx = tid; idx < n * qw; idx += T) {
            const int p = idx / qw, w = idx - p * qw;
            const uint32_t self = L.S[idx];
            core::Fields F;
            if constexpr (BIG)
                F = core::local_fields(L.nbr + p * rec_p, L.S, D, qw, w, L.hpos[p], rec_k);
            else
                F = sqa_fields(nb2 + p, n, D, 4u * (uint32_t)w, L.hpos[p]);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                atomicAdd(&L.E2[w * 4 + b],
                          (unsigned long long)((long long)dev::spin_of(self, b) * ((long long)L.hpos[p] + F.f[b])));
        }
    }
    __syncthreads();
    if (tid == 0) {
        int best = 0;
        long long bestE = 0;
        for (int k = 0; k < P; ++k) {
            const int m = k >> 1, w = (k & 1) * G8 + (m >> 2), b = m & 3;
            const long long E = ((long long)L.E2[w * 4 + b]) / 2;
            if (k == 0 || E < bestE) {
                bestE = E;
                best = k;
            }
        }
        best_s = best;
        bestE_s = bestE;
    }
    __syncthreads();
    const int best = best_s, m = best >> 1, bw = (best & 1) * G8 + (m >> 2), bb = m & 3;
    if (tid == 0) a.energies[read] = bestE_s;
    const int32_t *pos_of = a.image + kImgHeader + n;
    const unsigned char *Sb = reinterpret_cast<const unsigned char *>(L.S);
    for (int i = tid; i < n; i += T)
        a.out[(size_t)read * n + i] = (int8_t)Sb[((size_t)pos_of[i] * qw + bw) * 4 + bb];
}

}  // namespace

size_t sqa_lds_bytes(int n, int D, int row_len, int P, bool big) {
    return big ? core::sa_big_layout(n, row_len, P / 4, nullptr, nullptr)
               : core::sa_layout(n, 2 * D, row_len, P / 4, nullptr, nullptr);  // expanded records
}

hipError_t launch_sqa(const SqaLaunch &L, hipStream_t s) {
    SqaArgs a;
    a.image = L.image;
    a.tables = L.tables;
    a.jp = L.jp;
    a.out = L.out;
    a.energies = L.energies;
    a.n = L.n;
    a.D = L.D;
    a.C = L.C;
    a.row_len = L.row_len;
    a.sweeps = L.sweeps;
    a.reads = L.reads;
    a.P = L.P;
    a.x_bound = L.x_bound;
    a.k0 = (uint32_t)L.seed;
    a.k1 = (uint32_t)(L.seed >> 32);
    const size_t lds = sqa_lds_bytes(L.n, L.D, L.row_len, L.P, L.global_instance);
    if (L.P % 8 != 0 || L.P < 8 || L.threads % (L.P / 8) != 0 || L.reads < 1) return hipErrorInvalidValue;
#define SPV_SQA(ND_)                                                                                  \
    do {                                                                                              \
        if (L.global_instance)                                                                        \
            hipLaunchKernelGGL((sqa_kernel<ND_, true>), dim3(L.reads), dim3(L.threads), lds, s, a);   \
        else                                                                                          \
            hipLaunchKernelGGL((sqa_kernel<ND_, false>), dim3(L.reads), dim3(L.threads), lds, s, a);  \
    } while (0)
    switch (L.nd) {
        case 1:
            SPV_SQA(1);
            break;
        case 2:
            SPV_SQA(2);
            break;
        case 3:
            SPV_SQA(3);
            break;
        default:
            return hipErrorInvalidValue;
    }
#undef SPV_SQA
    return hipGetLastError();
}

hipError_t shadow_stats_sqa(unsigned long long *out, bool reset) { return shadow::read_stats(out, reset); }

}  // namespace spv
