// Parallel tempering with each run's ladder split over several workgroups
// (Sec. III.D.1 "PTICM" at sizes where one run does not fit one workgroup, or
// where there are too few runs to fill the device).
//
// A run's K slots are cut into G groups of m consecutive slots, m a multiple
// of 4 (every quad of 4 replicas of the replica index r = (run * chains +
// chain) * K + slot lies inside one group), or m = 2 or 1 (a group owns half
// or a quarter of its quad: it draws the quad's whole random block and updates
// its own bytes; the other bytes of its LDS copy are never changed or read out).
// A group of one slot reading its instance from the global image keeps both
// chains' bytes of that slot in one word per site (byte c: chain c), each byte
// drawing from its own chain's quad block.
// Workgroup (run, g) holds the group's slots of EVERY chain, so the Houdayer
// partners (chain 0 and chain 1 at one slot) share its LDS.  A sweep is
//   1. Metropolis on the group's replicas (colour classes in order),
//   2. replica exchange of pairs (k, k+1), k = t mod 2.  Pairs inside the
//      group are decided from LDS energies and swapped byte-wise; a pair that
//      straddles a group boundary (on odd sweeps when m is even; the lower and
//      the upper boundary on alternate sweeps when m = 1) is decided by both
//      neighbours from the energies each publishes (with the edge
//      configuration) as sweep-tagged atomic words; an accepted pair copies
//      the partner's published configuration in,
//   3. Houdayer moves at the group's slots, up to four slot pairs at a time
//      with the whole workgroup (lock-free union-find over the disagreeing
//      sites; with one pair, the join scan also gathers each disagreeing
//      site's energy term, so the energy pass needs no neighbour reads),
//   4. the top-10 offers of the group's colder slots.
// The instance lives in LDS when it fits beside the replicas; otherwise the
// neighbour records, biases and orderings are read from the global image
// (shared by every workgroup, L2-resident).
//
// Waits for a neighbour's words are bounded: a workgroup whose neighbour does
// not publish within the spin limit stops and marks its lists with
// top_count = -1.  The host only launches grids that fit on the device at once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "internal.hpp"
#include "lds_shadow.hpp"
#include "pt_core.hpp"

namespace spv {

namespace {

using ptc::lanemask_lt;
using ptc::swap_test;
using ptc::wave_sum;

struct PtxArgs {
    const int32_t *image;
    const uint32_t *mtab;  // [K][row_len]
    const uint32_t *stab;  // [K-1][7*512]
    const int32_t *snd;    // [K-1]
    int8_t *final_spins;
    long long *final_E;
    int8_t *top_spins;
    long long *top_E;
    int32_t *top_count;
    int8_t *tops;          // [runs][Ls][10][n], position order
    uint32_t *xw;          // [runs][G][side 2][buf 2][chains][xmsg] tagged boundary messages
    PtResume rs;           // checkpoint to start from
    int n, D, C, K, chains, sweeps, row_len, icm_lo, icm_hi, nw_icm, G, m, xmsg, esum;
    uint32_t sweep_offset, k0, k1;
    unsigned spin_limit;
};

struct PtxLds {
    uint32_t *nbr;      // [D][n]   (LDS-resident instance)
    int32_t *hpos;      // [n]      (LDS-resident instance)
    int32_t *ord;       // [n]      (LDS-resident instance)
    int32_t *pos;       // [n]      (LDS-resident instance)
    uint32_t *tab;      // [m][row_len]
    uint32_t *S;        // [n][nq]
    unsigned char *Sb;
    long long *E;       // [chains*m]
    long long *LE;      // [chains*m][10]
    int32_t *Lwhen;     // [chains*m][10]
    int32_t *Lcnt;      // [chains*m]
    int32_t *Lbad;      // [chains*m] checkpoint count was outside 0..10
    int32_t *Lord;      // [chains*m][10]
    int32_t *Lins;      // [chains*m] entry a list's offer replaces this sweep (-1: none)
    long long *Lmax;    // [chains*m] a full list's largest energy (LLONG_MAX: not known)
    int32_t *snd;       // [m + 1] digit counts of the swap tables of pairs s0-1 .. s0+m-1
    int32_t *acc;       // [chains*m] accepted in-group pairs: their replicas' byte offsets
    int32_t *cin;       // [2*chains] accepted boundary pairs (side, chain)
    uint16_t *parent;          // [pairs][n rounded to even] union-find forests over positions
    unsigned long long *dmask; // [pairs][ceil(n / 64)] disagreement masks in variable order
    int32_t *misc;             // [4] broadcast scalars
    uint32_t *ubuf;            // [16 waves][kJoinBuf] pending joins: site | neighbour << 16
    unsigned char *ubj;        // [16 waves][kJoinBuf] their slot pair
    int32_t *esite;            // [n] one slot pair's cluster energy terms (esum)
};

// Pending-join buffer per wavefront (64 appended at most on top of < 64 pending).
constexpr int kJoinBuf = 128;

__host__ __device__ inline size_t ptx_layout(int n, int D, int m, int chains, int row_len, int nw_icm, bool big,
                                             bool esum, PtxLds *L, unsigned char *base) {
    const int nq = (big && m == 1 && chains == 2) ? 1 : chains * ((m + 3) / 4), nl = chains * m,
              vstride = 2 * ((n + 63) / 64);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = (o + bytes + 15) & ~(size_t)15;
        return at;
    };
    const size_t in_lds = big ? 0 : 1;
    const size_t o_nbr = take(in_lds * n * D * 4), o_h = take(in_lds * n * 4), o_ord = take(in_lds * n * 4),
                 o_pos = take(in_lds * n * 4), o_tab = take((size_t)m * row_len * 4), o_S = take((size_t)n * nq * 4),
                 o_E = take((size_t)nl * 8), o_LE = take((size_t)nl * 80), o_Lw = take((size_t)nl * 40),
                 o_Lc = take((size_t)nl * 4), o_Lb = take((size_t)nl * 4), o_Lo = take((size_t)nl * 40),
                 o_Li = take((size_t)nl * 4), o_Lm = take((size_t)nl * 8), o_snd = take((size_t)(m + 1) * 4),
                 o_acc = take((size_t)nl * 4),
                 o_cin = take((size_t)2 * chains * 4), o_par = take((size_t)nw_icm * ((n + 1) & ~1) * 2),
                 o_dm = take((size_t)nw_icm * vstride * 4), o_misc = take(16),
                 o_ub = take(nw_icm ? (size_t)16 * kJoinBuf * 4 : 0), o_uj = take(nw_icm ? (size_t)16 * kJoinBuf : 0),
                 o_es = take(esum ? (size_t)n * 4 : 0);
    if (L) {
        L->nbr = reinterpret_cast<uint32_t *>(base + o_nbr);
        L->hpos = reinterpret_cast<int32_t *>(base + o_h);
        L->ord = reinterpret_cast<int32_t *>(base + o_ord);
        L->pos = reinterpret_cast<int32_t *>(base + o_pos);
        L->tab = reinterpret_cast<uint32_t *>(base + o_tab);
        L->S = reinterpret_cast<uint32_t *>(base + o_S);
        L->Sb = base + o_S;
        L->E = reinterpret_cast<long long *>(base + o_E);
        L->LE = reinterpret_cast<long long *>(base + o_LE);
        L->Lwhen = reinterpret_cast<int32_t *>(base + o_Lw);
        L->Lcnt = reinterpret_cast<int32_t *>(base + o_Lc);
        L->Lbad = reinterpret_cast<int32_t *>(base + o_Lb);
        L->Lord = reinterpret_cast<int32_t *>(base + o_Lo);
        L->Lins = reinterpret_cast<int32_t *>(base + o_Li);
        L->Lmax = reinterpret_cast<long long *>(base + o_Lm);
        L->snd = reinterpret_cast<int32_t *>(base + o_snd);
        L->acc = reinterpret_cast<int32_t *>(base + o_acc);
        L->cin = reinterpret_cast<int32_t *>(base + o_cin);
        L->parent = reinterpret_cast<uint16_t *>(base + o_par);
        L->dmask = reinterpret_cast<unsigned long long *>(base + o_dm);
        L->misc = reinterpret_cast<int32_t *>(base + o_misc);
        L->ubuf = reinterpret_cast<uint32_t *>(base + o_ub);
        L->ubj = base + o_uj;
        L->esite = reinterpret_cast<int32_t *>(base + o_es);
    }
    return o;
}

// Slot pairs whose cluster moves run together (one forest and mask set each).
constexpr int kIcmBatch = 4;
// Boundary-message words a thread loads at once when copying a configuration in.
constexpr int kCopyBatch = 4;

__global__ void xw_zero_kernel(uint32_t *w, size_t count) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        w[i] = 0u;
}

// ND threshold digits; BIG: instance read from the global image; DK: records per
// site fixed at compile time (0: D at run time).
// a byte in LDS, addressed with 32-bit offsets
typedef __attribute__((address_space(3))) const unsigned char lds_u8;
typedef __attribute__((address_space(3))) unsigned char lds_mu8;

template <int ND, bool BIG, int DK>
__global__ __launch_bounds__(1024) void ptx_kernel(PtxArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cs[kMaxColours + 1];
    __shared__ int nacc;
    __shared__ int stop;
    const int n = a.n, D = a.D, K = a.K, chains = a.chains, G = a.G, row_len = a.row_len, xmsg = a.xmsg;
    PtxLds Lay;
    ptx_layout(n, D, a.m, chains, row_len, a.nw_icm, BIG, a.esum != 0, &Lay, smem);
    // LDS regions as plain locals (keeps the layout record out of scratch memory)
    auto *const L_nbr = Lay.nbr;
    auto *const L_hpos = Lay.hpos;
    auto *const L_ord = Lay.ord;
    auto *const L_pos = Lay.pos;
    auto *const L_tab = Lay.tab;
    auto *const L_S = Lay.S;
    auto *const L_Sb = Lay.Sb;
    auto *const L_E = Lay.E;
    auto *const L_LE = Lay.LE;
    auto *const L_Lwhen = Lay.Lwhen;
    auto *const L_Lcnt = Lay.Lcnt;
    auto *const L_Lbad = Lay.Lbad;
    auto *const L_Lord = Lay.Lord;
    auto *const L_Lins = Lay.Lins;
    auto *const L_Lmax = Lay.Lmax;
    auto *const L_snd = Lay.snd;
    auto *const L_acc = Lay.acc;
    auto *const L_cin = Lay.cin;
    auto *const L_parent = Lay.parent;
    auto *const L_dmask = Lay.dmask;
    auto *const L_misc = Lay.misc;
    auto *const L_ubuf = Lay.ubuf;
    auto *const L_ubj = Lay.ubj;
    auto *const L_es = Lay.esite;
    const int tid = threadIdx.x, T = blockDim.x, lane = dev::lane_id(), wid = tid >> 6, nw = T >> 6;
    const int run = blockIdx.x / G, g = blockIdx.x - run * G;
    // boff: byte of the quad word holding the group's first slot (0 when m is a
    // multiple of 4)
    const int s0 = g * a.m, mg = min(a.m, K - s0), boff = s0 & 3, qpc = (boff + mg + 3) >> 2;
    // pk: a group of one slot (cluster moves on, two chains) reading its instance from
    // the global image keeps both chains' bytes of its slot in one word per site,
    // chain c in byte c (with the instance in LDS the layout stays one word per chain)
    const bool pk = BIG && mg == 1 && chains == 2;
    const int nq = pk ? 1 : chains * qpc, nl = chains * mg;
    const int32_t *img = a.image;
    const uint32_t *gnbr = reinterpret_cast<const uint32_t *>(img + kImgHeader + 3 * n);
    const int32_t *gord = img + kImgHeader, *gpos = img + kImgHeader + n, *ghpos = img + kImgHeader + 2 * n;
#ifdef __OPTIMIZE__
    // Kept as values of their own: otherwise each use rebuilds them from the whole
    // argument block, which comes back from spill lanes sixteen registers at a time.
    asm volatile("" : "+s"(gnbr), "+s"(gord), "+s"(ghpos));
#endif
    const uint32_t *const lnbr = L_nbr;
    const int32_t *const lhpos = L_hpos, *const lord = L_ord, *const lpos = L_pos;
    unsigned char *const Sb = L_Sb;
    auto NBR = [=](int k, int p) __attribute__((always_inline)) -> uint32_t {
        return BIG ? gnbr[(size_t)p * D + k] : lnbr[(size_t)k * n + p];
    };
    auto HPOS = [=](int p) __attribute__((always_inline)) -> int32_t { return BIG ? ghpos[p] : lhpos[p]; };
    auto ORD = [=](int p) __attribute__((always_inline)) -> int32_t { return BIG ? gord[p] : lord[p]; };
    auto POS = [=](int i) __attribute__((always_inline)) -> int32_t { return BIG ? gpos[i] : lpos[i]; };
    // byte of local replica l = chain * mg + (slot - s0) at position p
    auto sbyte = [=](int l, int p) __attribute__((always_inline)) -> unsigned char * {
        if (pk) return Sb + (size_t)p * 4 + l;
        const int ch = l / mg, o = l - ch * mg + boff;
        return Sb + ((size_t)p * nq + ch * qpc + (o >> 2)) * 4 + (o & 3);
    };
    // a replica's bytes lie pst apart: loops over positions take sbyte(l, 0) once
    const uint32_t pst = (uint32_t)nq * 4u;

    if (tid <= a.C) cs[tid] = img[3 + tid];
    if (tid == 0) stop = 0;
    if (!BIG) {
        for (int idx = tid; idx < n * D; idx += T) {
            const int p = idx / D, k = idx - p * D;
            L_nbr[(size_t)k * n + p] = gnbr[idx];
        }
        for (int k = tid; k < n; k += T) {
            L_ord[k] = gord[k];
            L_pos[k] = gpos[k];
            L_hpos[k] = ghpos[k];
        }
    }
    for (int k = tid; k < mg * row_len; k += T) L_tab[k] = a.mtab[(size_t)s0 * row_len + k];
    // the swap tables' digit counts of the pairs this group decides, k = s0 - 1 .. s0 + mg - 1
    for (int i = tid; i <= mg; i += T) {
        const int k = s0 - 1 + i;
        L_snd[i] = k >= 0 && k < K - 1 ? a.snd[k] : 0;
    }
    const int half = K / 2, Ls = chains * half;
    // Local slot l = chain * mg + (slot - s0); slots k >= K - half hold list gl.
    auto list_of = [=](int l) __attribute__((always_inline)) -> int {
        const int ch = l / mg, k = s0 + (l - ch * mg);
        return k >= K - half ? ch * half + (k - (K - half)) : -1;
    };
    for (int k = tid; k < nl; k += T) {
        L_E[k] = 0;
        L_Lmax[k] = 0x7FFFFFFFFFFFFFFFll;
        const int gl = list_of(k);
        const int c = (gl >= 0 && a.rs.top_count) ? a.rs.top_count[(size_t)run * Ls + gl] : 0;
        const bool bad = c < 0 || c > 10;
        L_Lcnt[k] = bad ? 0 : c;
        L_Lbad[k] = bad ? 1 : 0;
    }
    __syncthreads();
    if (a.rs.top_count) {
        // Checkpoint entries, inserted before this launch's offers in list order.
        for (int le = tid; le < nl * 10; le += T) {
            const int l = le / 10, e = le - l * 10, gl = list_of(l);
            if (gl >= 0 && e < L_Lcnt[l]) {
                L_LE[le] = a.rs.top_E[((size_t)run * Ls + gl) * 10 + e];
                L_Lwhen[le] = e - 10;
            }
        }
        for (size_t idx = tid; idx < (size_t)nl * 10 * n; idx += T) {
            const int lr = (int)(idx / n), i = (int)(idx - (size_t)lr * n);
            const int l = lr / 10, e = lr - l * 10, gl = list_of(l);
            if (gl >= 0 && e < L_Lcnt[l]) {
                const size_t row = ((size_t)run * Ls + gl) * 10 + e;
                a.tops[row * n + POS(i)] = a.rs.top_spins[row * n + i] > 0 ? (int8_t)1 : (int8_t)-1;
            }
        }
    }

    const int q = tid % nq, pt = tid / nq, nstr = T / nq;
    const bool active = pt < nstr;
    const int chq = q / qpc, jq = q - chq * qpc;
    const uint32_t quad = (uint32_t)((((size_t)run * chains + chq) * K + s0) / 4 + jq);
    // pk: chain 1's quad (byte 1 of the word draws its word boff from that quad's block)
    const uint32_t quad1 = (uint32_t)((((size_t)run * chains + 1) * K + s0) / 4);
    auto wsel = [](const dev::Words4 &w, int i) __attribute__((always_inline)) -> uint32_t {
        return i == 0 ? w.w[0] : i == 1 ? w.w[1] : i == 2 ? w.w[2] : w.w[3];
    };
    // byte b of the thread's word is the group's local slot 4 jq + b - boff; own marks
    // (0xFE) the bytes that are the group's
    int loc[4];
    const uint32_t *tb[4];
    uint32_t own = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int o = 4 * jq + b - boff;
        const bool mine = o >= 0 && o < mg;
        own |= mine ? 0xFEu << (8 * b) : 0u;
        loc[b] = chq * mg + (mine ? o : 0);
        tb[b] = L_tab + (size_t)(mine ? o : 0) * row_len;
        if (pk) {
            // byte b < 2: chain b of the group's slot (local replica b), table row 0
            loc[b] = b < 2 ? b : 0;
            tb[b] = L_tab;
        }
    }
    if (pk) own = 0xFEFEu;
    const bool pow2 = (nq & (nq - 1)) == 0 && nq <= 64;
    // the group owns 1 or 2 bytes of each of its words (the same bytes in every word)
    const bool part = !pk && qpc == 1 && mg < 4;

    // Initial state and energies.
    for (int p = pt; active && p < n; p += nstr) {
        const dev::Words4 w = dev::philox((uint32_t)ORD(p), 0u, quad, 1u << 24, a.k0, a.k1);
        uint32_t word = 0;
        if (pk) {
            const dev::Words4 w1 = dev::philox((uint32_t)ORD(p), 0u, quad1, 1u << 24, a.k0, a.k1);
            word = ((wsel(w, boff) >> 31) ? 0x01u : 0xFFu) | (((wsel(w1, boff) >> 31) ? 0x01u : 0xFFu) << 8) |
                   0x01010000u;
        } else {
#pragma unroll
            for (int b = 0; b < 4; ++b) word |= ((w.w[b] >> 31) ? 0x01u : 0xFFu) << (8 * b);
        }
        L_S[(size_t)p * nq + q] = word;
    }
    __syncthreads();
    if (a.rs.spins) {
        // The group's replicas start from the checkpoint.
        for (int idx = tid; idx < nl * n; idx += T) {
            const int l = idx / n, i = idx - l * n;
            const int ch = l / mg, slot = s0 + (l - ch * mg);
            *sbyte(l, POS(i)) =
                a.rs.spins[(((size_t)run * chains + ch) * K + slot) * n + i] > 0 ? (unsigned char)0x01 : (unsigned char)0xFF;
        }
        __syncthreads();
    }
    {
        long long e2[4] = {0, 0, 0, 0};
        for (int p = pt; active && p < n; p += nstr) {
            const uint32_t self = L_S[(size_t)p * nq + q];
            const int32_t hp = HPOS(p);
            int32_t f[4];
            ptc::quad_fields<DK>(NBR, D, p, L_S, nq, q, hp, f);
#pragma unroll
            for (int b = 0; b < 4; ++b) e2[b] += (long long)dev::spin_of(self, b) * ((long long)hp + f[b]);
        }
        if (active)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (own & (0xFEu << (8 * b)))
                    atomicAdd(reinterpret_cast<unsigned long long *>(&L_E[loc[b]]), (unsigned long long)e2[b]);
    }
    __syncthreads();
    for (int l = tid; l < nl; l += T) L_E[l] /= 2;  // sum of s(h + f) counts every coupler twice
    __syncthreads();

    // Race-detection build: each class pass's spin-word writes, then its neighbour
    // reads, against the LDS bitmap (a word is (position, quad)).
    const shadow::Pass sh = shadow::begin((uint32_t)n * (uint32_t)nq);
    auto shadow_pass = [&](int c, bool before) {
        const int pe = cs[c + 1];
        if (before) {
            for (int p = cs[c] + pt; active && p < pe; p += nstr) shadow::mark(sh, (uint32_t)(p * nq + q));
            shadow::barrier();
            for (int p = cs[c] + pt; active && p < pe; p += nstr)
                for (int k = 0; k < D; ++k) {
                    const uint32_t rec = NBR(k, p);
                    if ((rec & 0xffffu) != 0u) shadow::check(sh, (rec >> 16) * (uint32_t)nq + (uint32_t)q);
                }
            shadow::count_pass(sh);
        } else {
            for (int p = cs[c] + pt; active && p < pe; p += nstr) shadow::unmark(sh, (uint32_t)(p * nq + q));
            shadow::barrier();
        }
    };

    for (int ls = 0; ls < a.sweeps; ++ls) {
        const uint32_t t = a.sweep_offset + (uint32_t)ls;
        // 1. Metropolis on the group's replicas.
        long long dE[4] = {0, 0, 0, 0}, dEp[2] = {0, 0};
        for (int c = 0; c < a.C; ++c) {
            if constexpr (shadow::kOn) shadow_pass(c, true);
            const int pe = cs[c + 1];
            auto update = [&](int p, auto rec, int32_t hp, uint32_t ord) __attribute__((always_inline)) {
                const uint32_t self = L_S[(size_t)p * nq + q];
                int32_t f[4];
                ptc::quad_fields<DK>(rec, D, p, L_S, nq, q, hp, f);
                int32_t x[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) x[b] = dev::spin_of(self, b) > 0 ? -f[b] : f[b];
                // The key enters each site's draws opaquely: otherwise the twenty round
                // keys are hoisted out of the loop, outgrow the scalar registers and
                // come back one vector-lane read at a time.  (Unoptimised device builds
                // keep it in vector registers, where a scalar operand cannot bind.)
                uint32_t k0 = a.k0, k1 = a.k1;
#ifdef __OPTIMIZE__
                asm volatile("" : "+s"(k0), "+s"(k1));
#endif
                const uint32_t mask = own & ptc::metropolis_mask4<ND>(x, tb, ord, t, quad, k0, k1);
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (mask & (0xFEu << (8 * b))) dE[b] += 2ll * x[b];
                if (mask) L_S[(size_t)p * nq + q] = self ^ mask;
            };
            // A group of 1 or 2 slots owns bytes boff.. of its words: those bytes alone are
            // updated (the quad's random blocks drawn whole, so the draws are the same).
            auto update_part = [&](int p, const uint32_t *rr, int32_t hp, uint32_t ord) __attribute__((always_inline)) {
                const uint32_t self = L_S[(size_t)p * nq + q];
                uint32_t wv[DK > 0 ? DK : 1];
#pragma unroll
                for (int u = 0; u < DK; ++u) wv[u] = L_S[__umul24(rr[u] >> 16, (uint32_t)nq) + (uint32_t)q];
                uint32_t k0 = a.k0, k1 = a.k1;
#ifdef __OPTIMIZE__
                asm volatile("" : "+s"(k0), "+s"(k1));
#endif
                int32_t x[2];
                uint32_t d[2], th[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const int sh = 24 - 8 * min(boff + i, 3);  // (i = 1 of a 1-slot group is unused)
                    int32_t f = hp;
#pragma unroll
                    for (int u = 0; u < DK; ++u)
                        f += (int32_t)(int16_t)(rr[u] & 0xffffu) * ((int32_t)(wv[u] << sh) >> 24);
                    x[i] = ((int32_t)(self << sh) >> 24) > 0 ? -f : f;
                    d[i] = x[i] > 0 ? ((uint32_t)x[i] & (kDigitSize - 1)) : 0u;
                    th[i] = L_tab[(size_t)min(i, mg - 1) * row_len + d[i]];
                }
                auto pick = [&](const dev::Words4 &w, int i) __attribute__((always_inline)) -> uint32_t {
                    const int bb = min(boff + i, 3);
                    return bb == 0 ? w.w[0] : bb == 1 ? w.w[1] : bb == 2 ? w.w[2] : w.w[3];
                };
                bool acc[2];
                {
                    const dev::Words4 w = dev::philox(ord, t, quad, 2u << 24, k0, k1);
#pragma unroll
                    for (int i = 0; i < 2; ++i) acc[i] = (d[i] == 0) | (pick(w, i) < th[i]);
                }
#pragma unroll
                for (int j = 1; j < ND; ++j) {
                    bool need = false;
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        d[i] = x[i] > 0 ? (((uint32_t)x[i] >> (kDigitBits * j)) & (kDigitSize - 1)) : 0u;
                        need |= i < mg && d[i] != 0;
                        th[i] = L_tab[(size_t)min(i, mg - 1) * row_len + j * kDigitSize + d[i]];
                    }
                    if (need) {
                        const dev::Words4 w = dev::philox(ord, t, quad, (2u << 24) | (uint32_t)j, k0, k1);
#pragma unroll
                        for (int i = 0; i < 2; ++i)
                            if ((d[i] != 0) & (pick(w, i) >= th[i])) acc[i] = false;
                    }
                }
                uint32_t mask = 0;
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    if (i < mg && acc[i]) {
                        mask |= 0xFEu << (8 * (boff + i));
                        dEp[i] += 2ll * x[i];
                    }
                if (mask) L_S[(size_t)p * nq + q] = self ^ mask;
            };
            // pk: bytes 0 and 1 of the site's word are chains 0 and 1 of the group's slot;
            // each draws word boff of its own chain's quad block, digit by digit.
            auto update_pk = [&](int p, auto rec, int32_t hp, uint32_t ord) __attribute__((always_inline)) {
                const uint32_t self = L_S[p];
                int32_t f[4];
                ptc::quad_fields<DK>(rec, D, p, L_S, 1, 0, hp, f);
                uint32_t k0 = a.k0, k1 = a.k1;
#ifdef __OPTIMIZE__
                asm volatile("" : "+s"(k0), "+s"(k1));
#endif
                int32_t x[2];
                uint32_t d[2], th[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    x[i] = dev::spin_of(self, i) > 0 ? -f[i] : f[i];
                    d[i] = x[i] > 0 ? ((uint32_t)x[i] & (kDigitSize - 1)) : 0u;
                    th[i] = L_tab[d[i]];
                }
                bool acc[2];
                {
                    const dev::Words4 w0 = dev::philox(ord, t, quad, 2u << 24, k0, k1);
                    const dev::Words4 w1 = dev::philox(ord, t, quad1, 2u << 24, k0, k1);
                    acc[0] = (d[0] == 0) | (wsel(w0, boff) < th[0]);
                    acc[1] = (d[1] == 0) | (wsel(w1, boff) < th[1]);
                }
#pragma unroll
                for (int j = 1; j < ND; ++j) {
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        d[i] = x[i] > 0 ? (((uint32_t)x[i] >> (kDigitBits * j)) & (kDigitSize - 1)) : 0u;
                        th[i] = L_tab[j * kDigitSize + d[i]];
                    }
                    if (d[0] != 0) {
                        const dev::Words4 w = dev::philox(ord, t, quad, (2u << 24) | (uint32_t)j, k0, k1);
                        if (wsel(w, boff) >= th[0]) acc[0] = false;
                    }
                    if (d[1] != 0) {
                        const dev::Words4 w = dev::philox(ord, t, quad1, (2u << 24) | (uint32_t)j, k0, k1);
                        if (wsel(w, boff) >= th[1]) acc[1] = false;
                    }
                }
                uint32_t mask = 0;
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    if (acc[i]) {
                        mask |= 0xFEu << (8 * i);
                        dEp[i] += 2ll * x[i];
                    }
                if (mask) L_S[p] = self ^ mask;
            };
            if constexpr (BIG && DK > 0) {
                // Records, h and index of a site come from global memory: those of the
                // thread's next site are in flight while the current one is updated.
                uint32_t rn[DK];
                int32_t hn = 0, on = 0;
                auto fetch = [&](int pp) __attribute__((always_inline)) {
#pragma unroll
                    for (int u = 0; u < DK; ++u) rn[u] = gnbr[(size_t)pp * DK + u];
                    hn = ghpos[pp];
                    on = gord[pp];
                };
                auto sites = [&](auto body) __attribute__((always_inline)) {
                    int p = cs[c] + pt;
                    if (active && p < pe) fetch(p);
                    for (; active && p < pe; p += nstr) {
                        uint32_t rr[DK];
#pragma unroll
                        for (int u = 0; u < DK; ++u) rr[u] = rn[u];
                        const int32_t hp = hn, od = on;
                        if (p + nstr < pe) fetch(p + nstr);
                        body(p, rr, hp, (uint32_t)od);
                    }
                };
                if (pk)
                    sites([&](int p, const uint32_t *rr, int32_t hp, uint32_t od) __attribute__((always_inline)) {
                        update_pk(p, [&](int u, int) __attribute__((always_inline)) { return rr[u]; }, hp, od);
                    });
                else if (part)
                    sites([&](int p, const uint32_t *rr, int32_t hp, uint32_t od)
                              __attribute__((always_inline)) { update_part(p, rr, hp, od); });
                else
                    sites([&](int p, const uint32_t *rr, int32_t hp, uint32_t od) __attribute__((always_inline)) {
                        update(p, [&](int u, int) __attribute__((always_inline)) { return rr[u]; }, hp, od);
                    });
            } else if (pk) {
                for (int p = cs[c] + pt; active && p < pe; p += nstr) update_pk(p, NBR, HPOS(p), (uint32_t)ORD(p));
            } else {
                for (int p = cs[c] + pt; active && p < pe; p += nstr) update(p, NBR, HPOS(p), (uint32_t)ORD(p));
            }
            __syncthreads();
            if constexpr (shadow::kOn) shadow_pass(c, false);
        }
        if (part)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (i < mg && boff + i == b) dE[b] += dEp[i];
        if (pk) {
            dE[0] += dEp[0];
            dE[1] += dEp[1];
        }
        if (pow2) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                for (int off = nq; off < 64; off <<= 1) dE[b] += __shfl_xor(dE[b], off, 64);
            if (active && lane < nq)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (dE[b]) atomicAdd(reinterpret_cast<unsigned long long *>(&L_E[loc[b]]), (unsigned long long)dE[b]);
        } else if (active) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (dE[b]) atomicAdd(reinterpret_cast<unsigned long long *>(&L_E[loc[b]]), (unsigned long long)dE[b]);
        }
        if (tid == 0) nacc = 0;
        if (tid < 2 * chains) L_cin[tid] = 0;
        __syncthreads();

        // 2. Replica exchange.
        // This sweep's pairs (k, k+1) have k of parity par: nin of them lie inside the
        // group from slot kin on; lo_act / hi_act: the pair across the lower / upper
        // boundary is one of them.  Each boundary pair comes every other sweep, so
        // a side publishes every other sweep and its two buffers alternate.
        const int par = (int)(t & 1u);
        const int kin = s0 + ((s0 ^ par) & 1), nin = max(0, (s0 + mg - kin) / 2);
        const bool lo_act = g > 0 && ((s0 - 1) & 1) == par, hi_act = g < G - 1 && ((s0 + mg - 1) & 1) == par;
        const bool edge = lo_act || hi_act;
        const int buf = (int)((t >> 1) & 1u);
        // Boundary messages: relaxed agent-scope atomic words, each 16 payload bits
        // under a 16-bit sweep tag (never 0; the area is cleared before the launch).
        // Per-word coherence of atomics makes a word with the expected tag carry
        // that sweep's payload, so no fence (and no L2 write-back) is needed.
        const uint32_t tag = ((((uint32_t)ls + 1u) & 0x7FFFu) | 0x8000u) << 16;
        auto msg = [=](int grp, int side, int ch) __attribute__((always_inline)) -> uint32_t * {
            return a.xw + ((((size_t)run * G + grp) * 2 + side) * 2 + buf) * chains * xmsg + (size_t)ch * xmsg;
        };
        auto recv = [=](const uint32_t *w) __attribute__((always_inline)) -> int {
            unsigned it = 0;
            for (;;) {
                const uint32_t v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((v & 0xFFFF0000u) == tag) return (int)(v & 0xFFFFu);
                if (++it > a.spin_limit) return -1;
                __builtin_amdgcn_s_sleep(1);
            }
        };
        if (edge) {
            // publish the first / last slot of every chain for an active lower / upper
            // boundary pair (pre-exchange states, energies)
            for (int side = 0; side < 2; ++side) {
                if (side == 0 ? !lo_act : !hi_act) continue;
                for (int ch = 0; ch < chains; ++ch) {
                    const int l = ch * mg + (side ? mg - 1 : 0);
                    const unsigned char *rb = sbyte(l, 0);
                    uint32_t *dst = msg(g, side, ch);
                    const unsigned long long El = (unsigned long long)L_E[l];
                    for (int w = tid; w < xmsg; w += T) {
                        uint32_t pay;
                        if (w < 4) {
                            pay = (uint32_t)((El >> (16 * w)) & 0xFFFFu);
                        } else {
                            const uint32_t p = 2u * (uint32_t)(w - 4);
                            pay = (uint32_t)rb[p * pst] | ((int)p + 1 < n ? (uint32_t)rb[(p + 1u) * pst] << 8 : 0u);
                        }
                        __hip_atomic_store(dst + w, tag | pay, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
            __syncthreads();
        }
        {
            const int per = nin + (edge ? 2 : 0);      // + the straddling pairs
            if (tid < chains * per) {
                const int ch = tid / per, e = tid - ch * per;
                const uint32_t cctr = (uint32_t)(run * chains + ch);
                if (e < nin) {
                    const int k = kin + 2 * e;
                    const int la = ch * mg + (k - s0);
                    const long long Dd = L_E[la] - L_E[la + 1];
                    if (swap_test(Dd, a.stab + (size_t)k * 7 * kDigitSize, L_snd[k - s0 + 1], (uint32_t)k, t, cctr, a.k0,
                                  a.k1)) {
                        const long long x = L_E[la];
                        L_E[la] = L_E[la + 1];
                        L_E[la + 1] = x;
                        // the pair's byte offsets of its two replicas (at position 0)
                        const int ix = atomicAdd(&nacc, 1);
                        L_acc[2 * ix] = (int)(sbyte(la, 0) - Sb);
                        L_acc[2 * ix + 1] = (int)(sbyte(la + 1, 0) - Sb);
                    }
                } else if ((e == nin && lo_act) || (e == nin + 1 && hi_act)) {
                    // the pair straddling a group boundary: (s0 - 1, s0) against the lower
                    // neighbour's last slot, (s0 + mg - 1, s0 + mg) against the upper one's first
                    const int side = e - nin;
                    const uint32_t *m = msg(side == 0 ? g - 1 : g + 1, side == 0 ? 1 : 0, ch);
                    // the four energy words are loaded together (one round trip when the
                    // message is there); a word without the expected tag is waited for
                    uint32_t ew[4];
#pragma unroll
                    for (int w = 0; w < 4; ++w) ew[w] = __hip_atomic_load(m + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    unsigned long long eu = 0;
                    bool ok = true;
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        const int v = (ew[w] & 0xFFFF0000u) == tag ? (int)(ew[w] & 0xFFFFu) : recv(m + w);
                        ok = ok && v >= 0;
                        eu |= (unsigned long long)(v < 0 ? 0 : v) << (16 * w);
                    }
                    if (!ok) {
                        stop = 1;
                    } else {
                        const long long En = (long long)eu;
                        const int lo = ch * mg + (side == 0 ? 0 : mg - 1);
                        const int k = side == 0 ? s0 - 1 : s0 + mg - 1;
                        const long long Dd = side == 0 ? En - L_E[lo] : L_E[lo] - En;
                        if (swap_test(Dd, a.stab + (size_t)k * 7 * kDigitSize, L_snd[k - s0 + 1], (uint32_t)k, t, cctr,
                                      a.k0, a.k1)) {
                            L_E[lo] = En;
                            L_cin[side * chains + ch] = 1;
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (stop) break;
        {
            // accepted pairs swap their bytes four pairs at a time, every load before
            // the stores (the pairs' replicas are distinct)
            const int na = nacc;
            for (int pr0 = 0; pr0 < na; pr0 += 4) {
                const int nb = min(4, na - pr0);
                uint32_t oa[4], ob[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int pr = pr0 + min(u, nb - 1);
                    oa[u] = (uint32_t)L_acc[2 * pr];
                    ob[u] = (uint32_t)L_acc[2 * pr + 1];
                }
                lds_mu8 *const S3 = (lds_mu8 *)Sb;
                for (int p = tid; p < n; p += T) {
                    const uint32_t o = (uint32_t)p * pst;
                    unsigned char x[4], y[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        x[u] = S3[oa[u] + o];
                        y[u] = S3[ob[u] + o];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (u < nb) {
                            S3[oa[u] + o] = y[u];
                            S3[ob[u] + o] = x[u];
                        }
                }
            }
            if (edge) {
                // an accepted straddling pair takes the neighbour's published configuration
                // (kCopyBatch words per thread loaded together; a word whose tag is not
                // yet the expected one is waited for)
                const int nwd = xmsg - 4;
                for (int sc = 0; sc < 2 * chains; ++sc) {
                    if (!L_cin[sc]) continue;
                    const int side = sc / chains, ch = sc - side * chains;
                    const uint32_t *src = msg(side == 0 ? g - 1 : g + 1, side == 0 ? 1 : 0, ch) + 4;
                    unsigned char *rb = sbyte(ch * mg + (side ? mg - 1 : 0), 0);
                    for (int w0 = tid; w0 < nwd; w0 += kCopyBatch * T) {
                        uint32_t v[kCopyBatch];
#pragma unroll
                        for (int u = 0; u < kCopyBatch; ++u) {
                            const int w = w0 + u * T;
                            v[u] = w < nwd ? __hip_atomic_load(src + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
                        }
#pragma unroll
                        for (int u = 0; u < kCopyBatch; ++u) {
                            const int w = w0 + u * T;
                            if (w >= nwd) continue;
                            const int pay = (v[u] & 0xFFFF0000u) == tag ? (int)(v[u] & 0xFFFFu) : recv(src + w);
                            if (pay < 0) {
                                stop = 1;
                                continue;
                            }
                            const uint32_t p = 2u * (uint32_t)w;
                            rb[p * pst] = (unsigned char)(pay & 0xFF);
                            if ((int)p + 1 < n) rb[(p + 1u) * pst] = (unsigned char)(pay >> 8);
                        }
                    }
                }
            }
            __syncthreads();
            if (stop) break;
        }

        // 3. Houdayer cluster moves between chains 0 and 1 at the group's slots, up to
        // kIcmBatch slot pairs at a time with the whole workgroup: each cluster is the
        // connected component of its seed in the graph of J != 0 edges between sites
        // where the pair's replicas disagree, found with a lock-free union-find in LDS
        // (the pairs share every neighbour-record fetch).
        const int kb = max(a.icm_lo, s0), ke = min(a.icm_hi, s0 + mg);
        const int nchunks = (n + 63) / 64, vstr = 2 * nchunks, n16 = (n + 1) & ~1;
        // records per site (compile-time when DK > 0, so record batches stay in registers)
        const int Dn = DK > 0 ? DK : D;
        // One slot pair per pass (esum): the join scan also gathers, for every
        // disagreeing site v, E_v = sum of J s_v s_u over its agreeing neighbours u in
        // replica A, so the energy pass needs no neighbour reads (a cluster's change is
        // -2 sum over its sites of s_v h_v + E_v, as in the general pass below).
        const bool esum = a.esum != 0;
        constexpr int KB = DK > 0 ? DK : ptc::kRecBatch;
        const size_t pstride = (size_t)nq * 4;
        for (int kq = kb; a.nw_icm > 0 && kq < ke; kq += a.nw_icm) {
            const int nb = min(a.nw_icm, ke - kq);
            unsigned char *pa[kIcmBatch], *pb[kIcmBatch];
#pragma unroll
            for (int j = 0; j < kIcmBatch; ++j) {
                const int o = min(kq + j, ke - 1) - s0 + boff;
                pa[j] = pk ? Sb : Sb + (size_t)(o >> 2) * 4 + (o & 3);
                pb[j] = pk ? Sb + 1 : Sb + (size_t)(qpc + (o >> 2)) * 4 + (o & 3);
            }
            auto dis = [=](int j, int p) __attribute__((always_inline)) -> bool {
                return pa[j][(size_t)p * pstride] != pb[j][(size_t)p * pstride];
            };
            // The batch's disagreements at position p as bits (bit j: pair j).  When its
            // pairs lie in one quad word per chain, one XOR of the two words gives them all
            // (a byte is 0xFE where the replicas differ and 0 where they agree).
            const int o0 = kq - s0 + boff, qa0 = o0 >> 2, off0 = o0 & 3;
            const bool word_dis = off0 + nb <= 4;
            const uint32_t pmask = (1u << nb) - 1u;
            // Chain 0's spin bytes of the batch's pairs at position p (byte j: pair j) and
            // their disagreement bits.
            auto pair_bytes = [=](int p, uint32_t &wa, uint32_t &db) __attribute__((always_inline)) {
                if (pk) {
                    // one word: chain 0's byte, then chain 1's
                    const uint32_t w = L_S[p];
                    wa = w & 0xFFu;
                    db = ((w ^ (w >> 8)) >> 1) & 1u;
                    return;
                }
                if (word_dis) {
                    const uint32_t w0 = L_S[(size_t)p * nq + qa0], w1 = L_S[(size_t)p * nq + qpc + qa0];
                    wa = w0 >> (8 * off0);
                    uint32_t m = (((w0 ^ w1) >> (8 * off0)) >> 1) & 0x01010101u;
                    m |= m >> 7;
                    m |= m >> 14;
                    db = m & pmask;
                    return;
                }
                wa = 0;
                db = 0;
#pragma unroll
                for (int j = 0; j < kIcmBatch; ++j) {
                    const unsigned char x = pa[j][(size_t)p * pstride], y = pb[j][(size_t)p * pstride];
                    wa |= (uint32_t)x << (8 * j);
                    if (j < nb && x != y) db |= 1u << j;
                }
            };
            auto dis_bits = [=](int p) __attribute__((always_inline)) -> uint32_t {
                if (pk) {
                    const uint32_t w = L_S[p];
                    return ((w ^ (w >> 8)) >> 1) & 1u;
                }
                if (word_dis) {
                    const uint32_t x =
                        (L_S[(size_t)p * nq + qa0] ^ L_S[(size_t)p * nq + qpc + qa0]) >> (8 * off0);
                    uint32_t m = (x >> 1) & 0x01010101u;
                    m |= m >> 7;
                    m |= m >> 14;
                    return m & pmask;
                }
                uint32_t m = 0;
#pragma unroll
                for (int j = 0; j < kIcmBatch; ++j)
                    if (j < nb && dis(j, p)) m |= 1u << j;
                return m;
            };
            // disagreement masks in variable-index order, 64 variables per chunk
            for (int c0 = wid; c0 < nchunks; c0 += 4 * nw) {
                int pp[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = (c0 + u * nw) * 64 + lane;
                    pp[u] = (c0 + u * nw < nchunks && i < n) ? POS(i) : -1;
                }
                uint32_t db[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) db[u] = pp[u] >= 0 ? dis_bits(pp[u]) : 0u;
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int j = 0; j < kIcmBatch; ++j) {
                        if (j >= nb) break;
                        const unsigned long long m = __ballot((db[u] >> j) & 1u);
                        if (lane == 0 && c0 + u * nw < nchunks) L_dmask[(size_t)j * nchunks + c0 + u * nw] = m;
                    }
            }
            __syncthreads();
            if (wid < nb) {
                // seed of pair wid = the target-th disagreeing variable
                const int j = wid, k = kq + j;
                const unsigned long long *dm = L_dmask + (size_t)j * nchunks;
                int n_neg = 0;
                for (int c = lane; c < nchunks; c += 64) n_neg += __popcll(dm[c]);
                for (int d = 32; d >= 1; d >>= 1) n_neg += __shfl_xor(n_neg, d, 64);
                int seed_p = -1;
                if (n_neg > 0) {
                    const uint32_t w = dev::philox((uint32_t)k, t, (uint32_t)run, 4u << 24, a.k0, a.k1).w[0];
                    const int target = (int)(((unsigned long long)w * (unsigned long long)n_neg) >> 32);
                    int seen = 0;
                    for (int c0 = 0; c0 < nchunks && seed_p < 0; c0 += 64) {
                        const int c = c0 + lane;
                        const unsigned long long m = c < nchunks ? dm[c] : 0ull;
                        const int cnt = __popcll(m);
                        int incl = cnt;
                        for (int d = 1; d < 64; d <<= 1) {
                            const int y = __shfl_up(incl, d, 64);
                            if (lane >= d) incl += y;
                        }
                        const int excl = seen + incl - cnt;
                        const unsigned long long who = __ballot(target >= excl && target < excl + cnt);
                        if (who) {
                            const int src = __ffsll((long long)who) - 1;
                            const unsigned long long ms = __shfl(m, src, 64);
                            const int rest = target - __shfl(excl, src, 64);
                            const bool mine = ((ms >> lane) & 1ull) && __popcll(ms & lanemask_lt()) == rest;
                            const int bitl = __ffsll((long long)__ballot(mine)) - 1;
                            seed_p = POS((c0 + src) * 64 + bitl);
                        }
                        seen += __shfl(incl, 63, 64);
                    }
                }
                if (lane == 0) L_misc[j] = seed_p;
            }
            // fresh forests and energy terms, written by the other wavefronts while the
            // seeds are searched (by all of them when every wavefront searches a seed)
            const int iw = T > 64 * nb ? nb : 0;
            if (wid >= iw) {
                const int t0 = tid - 64 * iw, ts = T - 64 * iw;
                for (int j = 0; j < nb; ++j)
                    for (int p = t0; p < n16; p += ts) L_parent[(size_t)j * n16 + p] = (uint16_t)p;
                if (esum)
                    for (int p = t0; p < n; p += ts) L_es[p] = 0;
            }
            __syncthreads();
            // The masks are consumed: their words now collect cluster membership.
            uint32_t *const memb = reinterpret_cast<uint32_t *>(L_dmask);
            if (!esum)
                for (int wd = tid; wd < nb * vstr; wd += T) memb[wd] = 0u;
            // join the endpoints of every J != 0 edge between disagreeing sites.  Each
            // wavefront scans 64 sites at a time and appends the qualifying
            // (pair, site, neighbour) joins to its own LDS buffer; whenever 64 are
            // pending, every lane performs one (full lanes instead of the ~1 in 4 that
            // a per-site loop would keep busy).  Join order does not change the sets.
            {
                uint32_t *const wb = L_ubuf + wid * kJoinBuf;
                unsigned char *const wj = L_ubj + wid * kJoinBuf;
                int cnt = 0;
                auto run_joins = [&](int m) __attribute__((always_inline)) {
                    __builtin_amdgcn_wave_barrier();
                    if (lane < m) {
                        const uint32_t it = wb[cnt - m + lane];
                        ptc::uf_union(L_parent + (size_t)wj[cnt - m + lane] * n16, it & 0xFFFFu, it >> 16);
                    }
                    cnt -= m;
                    __builtin_amdgcn_wave_barrier();
                };
                // Every edge is taken from its smaller end, and the last colour class (the
                // highest positions; no edge joins two sites of one class) has none: the
                // scan stops where that class begins.
                const int scan_end = a.C > 0 ? min(n, cs[a.C - 1]) : 0;
                auto scan_site = [&](int p, auto rec) __attribute__((always_inline)) {
                    uint32_t dp = 0, ap = 0;
                    if (esum) {
                        if (p < n) pair_bytes(p, ap, dp);
                    } else {
                        dp = p < n ? dis_bits(p) : 0u;
                    }
                    // with esum every site's edges are read (an agreeing site may border a
                    // disagreeing one)
                    const bool need = esum ? p < n : dp != 0u;
                    for (int k0 = 0; k0 < Dn; k0 += KB) {
                        uint32_t rr[KB];
#pragma unroll
                        for (int uu = 0; uu < KB; ++uu) rr[uu] = (need && k0 + uu < Dn) ? rec(k0 + uu, p) : 0u;
                        // the pairs each edge joins, every neighbour's words read before the joins
                        uint32_t fb[KB];
#pragma unroll
                        for (int uu = 0; uu < KB; ++uu) {
                            const int u = (int)(rr[uu] >> 16);
                            const bool edge_ok = k0 + uu < Dn && (rr[uu] & 0xffffu) != 0u && u > p;
                            if (esum) {
                                uint32_t au = 0, du = 0;
                                if (edge_ok) pair_bytes(u, au, du);
                                fb[uu] = dp & du;
                                if (edge_ok && ((dp ^ du) & 1u)) {
                                    // an edge with one disagreeing end: its term goes to that end
                                    const int32_t Jv = (int32_t)(int16_t)(rr[uu] & 0xffffu);
                                    const int32_t prod = Jv * (int32_t)(int8_t)(ap & 0xFFu) * (int32_t)(int8_t)(au & 0xFFu);
                                    atomicAdd(&L_es[(dp & 1u) ? p : u], prod);
                                }
                            } else {
                                fb[uu] = edge_ok ? (dp & dis_bits(u)) : 0u;
                            }
                        }
#pragma unroll
                        for (int uu = 0; uu < KB; ++uu) {
                            if (k0 + uu >= Dn) break;
                            const int u = (int)(rr[uu] >> 16);
#pragma unroll
                            for (int j = 0; j < kIcmBatch; ++j) {
                                if (j >= nb) break;
                                const bool f = (fb[uu] >> j) & 1u;
                                const unsigned long long msk = __ballot(f);
                                if (f) {
                                    const int at = cnt + __popcll(msk & lanemask_lt());
                                    wb[at] = (uint32_t)p | ((uint32_t)u << 16);
                                    wj[at] = (unsigned char)j;
                                }
                                cnt += __popcll(msk);
                                if (cnt >= 64) run_joins(64);
                            }
                        }
                    }
                };
                if constexpr (BIG && DK > 0) {
                    // the records of the wavefront's next 64 sites are in flight while
                    // the current ones are scanned
                    uint32_t rn[DK];
                    auto fetch = [&](int pp) __attribute__((always_inline)) {
#pragma unroll
                        for (int u = 0; u < DK; ++u) rn[u] = pp < n ? gnbr[(size_t)pp * DK + u] : 0u;
                    };
                    int p0 = wid * 64;
                    if (p0 < scan_end) fetch(p0 + lane);
                    for (; p0 < scan_end; p0 += nw * 64) {
                        uint32_t rr[DK];
#pragma unroll
                        for (int u = 0; u < DK; ++u) rr[u] = rn[u];
                        if (p0 + nw * 64 < scan_end) fetch(p0 + nw * 64 + lane);
                        scan_site(p0 + lane, [&](int k, int) __attribute__((always_inline)) { return rr[k]; });
                    }
                } else {
                    for (int p0 = wid * 64; p0 < scan_end; p0 += nw * 64) scan_site(p0 + lane, NBR);
                }
                if (cnt > 0) run_joins(cnt);
            }
            __syncthreads();
            // energy change of flipping each seed's component: -2 s_v (h_v + sum over
            // agreeing neighbours J s_u) per site (a neighbour across a J != 0 edge is in
            // the cluster exactly when it disagrees); the replicas are only written after
            // every site has been read
            uint32_t root[kIcmBatch];
#pragma unroll
            for (int j = 0; j < kIcmBatch; ++j) {
                const int sp = j < nb ? L_misc[j] : -1;
                root[j] = sp >= 0 ? ptc::uf_find(L_parent + (size_t)j * n16, (uint32_t)sp) : 0xffffffffu;
            }
            long long dA[kIcmBatch];
#pragma unroll
            for (int j = 0; j < kIcmBatch; ++j) dA[j] = 0;
            auto energy_site = [&](int p, auto rec, int32_t hp) __attribute__((always_inline)) {
                unsigned in = 0;
                const uint32_t dpb = dis_bits(p);
#pragma unroll
                for (int j = 0; j < kIcmBatch; ++j)
                    if (root[j] != 0xffffffffu && ((dpb >> j) & 1u) &&
                        ptc::uf_find(L_parent + (size_t)j * n16, (uint32_t)p) == root[j])
                        in |= 1u << j;
                if (!in) return;
                // f = h + sum of J s over the neighbours that agree (those outside the
                // cluster); replica B's field is the same (it agrees with A there) and its
                // spin at p is -s_A, so its energy change is -dA: the pair energy is
                // conserved exactly
                int32_t fA[kIcmBatch];
#pragma unroll
                for (int j = 0; j < kIcmBatch; ++j) fA[j] = hp;
                for (int k0 = 0; k0 < Dn; k0 += KB) {
                    uint32_t rr[KB];
#pragma unroll
                    for (int uu = 0; uu < KB; ++uu) rr[uu] = k0 + uu < Dn ? rec(k0 + uu, p) : 0u;
                    uint32_t wa[KB], db[KB];
#pragma unroll
                    for (int uu = 0; uu < KB; ++uu) pair_bytes((int)(rr[uu] >> 16), wa[uu], db[uu]);
#pragma unroll
                    for (int uu = 0; uu < KB; ++uu) {
                        const int32_t Jv = (int32_t)(int16_t)(rr[uu] & 0xffffu);
                        if (k0 + uu >= Dn || Jv == 0) continue;
#pragma unroll
                        for (int j = 0; j < kIcmBatch; ++j)
                            if (((in >> j) & 1u) && !((db[uu] >> j) & 1u))
                                fA[j] += Jv * (int32_t)(int8_t)(wa[uu] >> (8 * j));
                    }
                }
                uint32_t wp, dbp;
                pair_bytes(p, wp, dbp);
#pragma unroll
                for (int j = 0; j < kIcmBatch; ++j)
                    if ((in >> j) & 1u) {
                        atomicOr(&memb[(size_t)j * vstr + (p >> 5)], 1u << (p & 31));
                        dA[j] += -2ll * (int32_t)(int8_t)(wp >> (8 * j)) * (long long)fA[j];
                    }
            };
            if (esum) {
                // the seed's cluster: its disagreeing sites whose root is the seed's
                auto esite = [&](int p, int32_t hp) __attribute__((always_inline)) {
                    uint32_t wp, dbp;
                    pair_bytes(p, wp, dbp);
                    if (root[0] == 0xffffffffu || !(dbp & 1u)) return;
                    if (ptc::uf_find(L_parent, (uint32_t)p) != root[0]) return;
                    dA[0] += -2ll * ((long long)(int8_t)(wp & 0xFFu) * hp + (long long)L_es[p]);
                    // no other thread reads this site's bytes in this pass: flip it here
                    pa[0][(size_t)p * pstride] = (unsigned char)(-(int)(int8_t)pa[0][(size_t)p * pstride]);
                    pb[0][(size_t)p * pstride] = (unsigned char)(-(int)(int8_t)pb[0][(size_t)p * pstride]);
                };
                if constexpr (BIG) {
                    // the next site's bias is in flight while the current one is tested
                    int p = tid;
                    int32_t hn = p < n ? ghpos[p] : 0;
                    for (; p < n; p += T) {
                        const int32_t hp = hn;
                        if (p + T < n) hn = ghpos[p + T];
                        esite(p, hp);
                    }
                } else {
                    for (int p = tid; p < n; p += T) esite(p, HPOS(p));
                }
            } else {
                if constexpr (BIG && DK > 0) {
                    // the records and h of the thread's next site are in flight while the
                    // current one is tested and summed
                    uint32_t rn[DK];
                    int32_t hn = 0;
                    auto fetch = [&](int pp) __attribute__((always_inline)) {
#pragma unroll
                        for (int u = 0; u < DK; ++u) rn[u] = gnbr[(size_t)pp * DK + u];
                        hn = ghpos[pp];
                    };
                    int p = tid;
                    if (p < n) fetch(p);
                    for (; p < n; p += T) {
                        uint32_t rr[DK];
#pragma unroll
                        for (int u = 0; u < DK; ++u) rr[u] = rn[u];
                        const int32_t hp = hn;
                        if (p + T < n) fetch(p + T);
                        energy_site(p, [&](int k, int) __attribute__((always_inline)) { return rr[k]; }, hp);
                    }
                } else {
                    for (int p = tid; p < n; p += T) energy_site(p, NBR, HPOS(p));
                }
            }
#pragma unroll
            for (int j = 0; j < kIcmBatch; ++j) {
                if (j >= nb) break;
                const long long sa = wave_sum(dA[j]), sb = -sa;
                const int la = kq + j - s0, lb = mg + la;
                if (lane == 0) {
                    if (sa) atomicAdd(reinterpret_cast<unsigned long long *>(&L_E[la]), (unsigned long long)sa);
                    if (sb) atomicAdd(reinterpret_cast<unsigned long long *>(&L_E[lb]), (unsigned long long)sb);
                }
            }
            __syncthreads();
            // flip the clusters in both replicas (the gathered-terms pass flipped its own)
            for (int p = tid; !esum && p < n; p += T)
#pragma unroll
                for (int j = 0; j < kIcmBatch; ++j)
                    if (j < nb && ((memb[(size_t)j * vstr + (p >> 5)] >> (p & 31)) & 1u)) {
                        pa[j][(size_t)p * pstride] = (unsigned char)(-(int)(int8_t)pa[j][(size_t)p * pstride]);
                        pb[j][(size_t)p * pstride] = (unsigned char)(-(int)(int8_t)pb[j][(size_t)p * pstride]);
                    }
            __syncthreads();
        }

        // 4. Top-10 lists of the group's colder slots: a wavefront per list decides the
        // offer (candidate test, duplicate check, victim entry) and updates the list;
        // the inserted state is stored by that wavefront, or for long states (where one
        // wavefront's copy outlasts a barrier) by the whole workgroup afterwards.
        const int kc = max(K - half, s0), ncold = max(0, s0 + mg - kc);
        const bool wide_copy = n >= 2048;
        // replica l's state into dst by threads first, first + step, ...
        auto store_state = [&](int l, int8_t *dst, int first, int step) __attribute__((always_inline)) {
            if (pk && (n & 3) == 0) {
                // chain l's byte of four consecutive sites' words per thread, one word store
                const int sh = 8 * l;
                for (int w = first; w < (n >> 2); w += step) {
                    const uint4 v = *reinterpret_cast<const uint4 *>(L_S + 4 * w);
                    *reinterpret_cast<uint32_t *>(dst + 4 * w) =
                        ((v.x >> sh) & 0xFFu) | (((v.y >> sh) & 0xFFu) << 8) | (((v.z >> sh) & 0xFFu) << 16) |
                        (((v.w >> sh) & 0xFFu) << 24);
                }
            } else {
                // 32-bit LDS offsets stepped by addition (no 64-bit address arithmetic)
                const lds_u8 *rb = (const lds_u8 *)sbyte(l, 0);
                const uint32_t ostep = (uint32_t)step * pst;
                uint32_t o = (uint32_t)first * pst;
                for (uint32_t p = (uint32_t)first; p < (uint32_t)n; p += (uint32_t)step, o += ostep)
                    dst[p] = (int8_t)rb[o];
            }
        };
        for (int li = wid; li < chains * ncold; li += nw) {
            const int ch = li / ncold, k = kc + (li - ch * ncold);
            const int l = ch * mg + (k - s0);
            const int gl = ch * half + (k - (K - half));
            const long long Ec = L_E[l];
            const int cnt = L_Lcnt[l];
            // a full list whose largest energy is known and not above the offered one
            // fails the candidate test without reading its entries
            if (cnt == 10 && Ec >= L_Lmax[l]) {
                if (wide_copy && lane == 0) L_Lins[li] = -1;
                continue;
            }
            long long *LE = L_LE + (size_t)l * 10;
            int32_t *LW = L_Lwhen + (size_t)l * 10;
            int8_t *base = a.tops + ((size_t)run * Ls + gl) * 10 * n;
            int victim = -1;
            // lane e holds entry e: one butterfly over 16 lanes gives the entry ordered
            // last by (energy, insertion stamp), the worst one and a full list's victim
            // (stamps are distinct, so the order is strict)
            const bool held = lane < cnt;
            const long long le = held ? LE[lane] : (long long)0x8000000000000000ll;
            const int32_t lw = held ? LW[lane] : (int32_t)0x80000000;
            long long bk = le;
            int32_t bw = lw, bi = lane;
#pragma unroll
            for (int off = 8; off >= 1; off >>= 1) {
                const long long ok = __shfl_xor(bk, off, 64);
                const int32_t ow = __shfl_xor(bw, off, 64), oi = __shfl_xor(bi, off, 64);
                if (ok > bk || (ok == bk && ow > bw)) {
                    bk = ok;
                    bw = ow;
                    bi = oi;
                }
            }
            const long long worst = __shfl(bk, 0, 64);
            const bool cand = cnt < 10 || Ec < worst;
            if (cand) {
                const lds_u8 *rb = (const lds_u8 *)sbyte(l, 0);
                bool dup = false;
                // entries of equal energy get a full comparison of their states
                for (unsigned long long eq = __ballot(held && le == Ec); eq && !dup; eq &= eq - 1) {
                    const int8_t *ent = base + (size_t)(__ffsll((long long)eq) - 1) * n;
                    bool diff = false;
                    uint32_t o = (uint32_t)lane * pst;
                    for (uint32_t p = (uint32_t)lane; p < (uint32_t)n; p += 64u, o += 64u * pst)
                        diff |= ent[p] != (int8_t)rb[o];
                    dup = !__any(diff);
                }
                if (!dup) {
                    victim = __builtin_amdgcn_readfirstlane(cnt < 10 ? cnt : __shfl(bi, 0, 64));
                    if (!wide_copy) store_state(l, base + (size_t)victim * n, lane, 64);
                }
            }
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) {
                if (wide_copy) L_Lins[li] = victim;
                if (victim >= 0) {
                    LE[victim] = Ec;
                    LW[victim] = ls;
                    if (cnt < 10) L_Lcnt[l] = cnt + 1;
                }
                // the largest energy stays known while the entries do not change
                L_Lmax[l] = victim < 0 && cnt == 10 ? worst : 0x7FFFFFFFFFFFFFFFll;
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (wide_copy && ncold > 0) {
            __syncthreads();
            for (int li = 0; li < chains * ncold; ++li) {
                const int victim = L_Lins[li];
                if (victim < 0) continue;
                const int ch = li / ncold, k = kc + (li - ch * ncold);
                const int l = ch * mg + (k - s0);
                const int gl = ch * half + (k - (K - half));
                store_state(l, a.tops + (((size_t)run * Ls + gl) * 10 + victim) * n, tid, T);
            }
        }
        __syncthreads();
    }

    const int kc = max(K - half, s0), ncold = max(0, s0 + mg - kc);
    if (stop) {
        // A neighbour never published: mark the group's lists as invalid.
        if (a.top_count)
            for (int li = tid; li < chains * ncold; li += T) {
                const int ch = li / ncold, k = kc + (li - ch * ncold);
                a.top_count[(size_t)run * Ls + ch * half + (k - (K - half))] = -1;
            }
        return;
    }
    // Outputs of the group's replicas.
    if (a.final_E)
        for (int l = tid; l < nl; l += T) {
            const int ch = l / mg, slot = s0 + (l - ch * mg);
            a.final_E[((size_t)run * chains + ch) * K + slot] = L_E[l];
        }
    if (a.final_spins)
        for (int idx = tid; idx < nl * n; idx += T) {
            const int l = idx / n, i = idx - l * n;
            const int ch = l / mg, slot = s0 + (l - ch * mg);
            a.final_spins[(((size_t)run * chains + ch) * K + slot) * n + i] = (int8_t)*sbyte(l, POS(i));
        }
    if (a.top_E || a.top_spins || a.top_count) {
        // Rank of entry e of a list = number of entries ordered before it by (E, insertion).
        const int nlist = chains * ncold;
        for (int le = tid; le < nlist * 10; le += T) L_Lord[le] = -1;
        __syncthreads();
        for (int le = tid; le < nlist * 10; le += T) {
            const int li = le / 10, e = le - li * 10;
            const int ch = li / ncold, k = kc + (li - ch * ncold);
            const int l = ch * mg + (k - s0);
            const long long *LE = L_LE + (size_t)l * 10;
            const int32_t *LW = L_Lwhen + (size_t)l * 10;
            const int cnt = L_Lcnt[l];
            if (e < cnt) {
                int rank = 0;
                for (int o = 0; o < cnt; ++o) rank += (LE[o] < LE[e] || (LE[o] == LE[e] && LW[o] < LW[e])) ? 1 : 0;
                L_Lord[li * 10 + rank] = e;
            }
            if (e == 0 && a.top_count)
                a.top_count[(size_t)run * Ls + ch * half + (k - (K - half))] = L_Lbad[l] ? -1 : cnt;
        }
        __syncthreads();
        if (a.top_E)
            for (int le = tid; le < nlist * 10; le += T) {
                const int li = le / 10, rank = le - li * 10;
                const int ch = li / ncold, k = kc + (li - ch * ncold);
                const int l = ch * mg + (k - s0), gl = ch * half + (k - (K - half));
                const int e = L_Lord[le];
                a.top_E[((size_t)run * Ls + gl) * 10 + rank] = e >= 0 ? L_LE[(size_t)l * 10 + e] : 0x7FFFFFFFFFFFFFFFll;
            }
        if (a.top_spins)
            for (size_t idx = tid; idx < (size_t)nlist * 10 * n; idx += T) {
                const int lr = (int)(idx / n), i = (int)(idx - (size_t)lr * n);
                const int li = lr / 10, rank = lr - li * 10;
                const int ch = li / ncold, k = kc + (li - ch * ncold);
                const int gl = ch * half + (k - (K - half));
                const int e = L_Lord[li * 10 + rank];
                a.top_spins[((size_t)run * Ls + gl) * 10 * n + (size_t)rank * n + i] =
                    e >= 0 ? a.tops[(((size_t)run * Ls + gl) * 10 + e) * n + POS(i)] : (int8_t)0;
            }
    }
}

template <int ND, bool BIG>
void *ptx_entry(int D) {
    if (D == 6) return reinterpret_cast<void *>(ptx_kernel<ND, BIG, 6>);
    return reinterpret_cast<void *>(ptx_kernel<ND, BIG, 0>);
}

void *ptx_fn(int nd, bool big, int D) {
    switch (nd) {
        case 1:
            return big ? ptx_entry<1, true>(D) : ptx_entry<1, false>(D);
        case 2:
            return big ? ptx_entry<2, true>(D) : ptx_entry<2, false>(D);
        case 3:
            return big ? ptx_entry<3, true>(D) : ptx_entry<3, false>(D);
        default:
            return nullptr;
    }
}

}  // namespace

int ptx_msg_words(int n) { return 4 + (n + 1) / 2; }

size_t ptx_lds_bytes(int n, int D, int m, int chains, int row_len, int nw_icm, bool big, bool esum) {
    return ptx_layout(n, D, m, chains, row_len, nw_icm, big, esum, nullptr, nullptr);
}

hipError_t ptx_max_groups_resident(int nd, bool big, int D, int threads, size_t lds, int *blocks_per_cu) {
    void *f = ptx_fn(nd, big, D);
    if (!f) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, threads, lds);
}

hipError_t launch_ptx(const PtxLaunch &P, hipStream_t s) {
    PtxArgs a;
    a.image = P.image;
    a.mtab = P.mtab;
    a.stab = P.stab;
    a.snd = P.snd;
    a.final_spins = P.out->final_spins;
    a.final_E = reinterpret_cast<long long *>(P.out->final_E);
    a.top_spins = P.out->top_spins;
    a.top_E = reinterpret_cast<long long *>(P.out->top_E);
    a.top_count = P.out->top_count;
    a.tops = P.tops;
    a.rs = P.resume;
    a.xw = P.xw;
    a.xmsg = ptx_msg_words(P.n);
    a.n = P.n;
    a.D = P.D;
    a.C = P.C;
    a.K = P.K;
    a.chains = P.chains;
    a.sweeps = P.sweeps;
    a.row_len = P.row_len;
    a.icm_lo = P.icm_lo;
    a.icm_hi = P.icm_hi;
    a.nw_icm = P.nw_icm;
    a.esum = P.esum ? 1 : 0;
    a.G = P.G;
    a.m = P.m;
    a.sweep_offset = P.sweep_offset;
    a.k0 = (uint32_t)P.seed;
    a.k1 = (uint32_t)(P.seed >> 32);
    a.spin_limit = P.spin_limit;
    if (P.G > 1) {
        const size_t words = (size_t)P.runs * P.G * 4 * P.chains * ptx_msg_words(P.n);
        hipLaunchKernelGGL(xw_zero_kernel, dim3((unsigned)std::min<size_t>((words + 255) / 256, 4096)), dim3(256), 0,
                           s, P.xw, words);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const size_t lds = ptx_lds_bytes(P.n, P.D, P.m, P.chains, P.row_len, P.nw_icm, P.big, P.esum);
    void *f = ptx_fn(P.nd, P.big, P.D);
    if (!f) return hipErrorInvalidValue;
    void *args[] = {&a};
    return hipLaunchKernel(f, dim3(P.runs * P.G), dim3(P.threads), args, lds, s);
}

hipError_t shadow_stats_ptx(unsigned long long *out, bool reset) { return shadow::read_stats(out, reset); }

}  // namespace spv
