// Parallel tempering with replica exchange, Houdayer isoenergetic cluster
// moves and the top-10 sample (Sec. III.D.1, "PTICM" sample formation).
//
// One workgroup owns one run: its `chains` ladders of K slots live in LDS as
// S[p][q] words (4 replicas per word, replica r = (run * chains + chain) * K +
// slot), together with the position-ordered instance, one Metropolis
// threshold row per slot and the run's energies.  A sweep is
//   1. Metropolis on every slot (colour classes in order; lane = position x
//      quad, per-replica table row, one Philox block per quad),
//   2. replica exchange of pairs (k, k+1), k = t mod 2, decided from the
//      energies held in LDS, configurations swapped byte-wise,
//   3. Houdayer moves (chains 0/1): a wavefront per slot picks the seed with
//      ballots, grows the cluster with a wavefront BFS (LDS visited bitset +
//      queue, ballot/mbcnt compaction) and flips it in both replicas,
//   4. the colder half is offered to per-slot lists of the 10 lowest-energy
//      distinct states (a wavefront per list: ballot compare, byte copy).
// Replicas of a quad that belong to a neighbouring run (when chains*K is not
// a multiple of 4) are carried along but never read back.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "internal.hpp"
#include "lds_shadow.hpp"
#include "pt_core.hpp"

namespace spv {

namespace {

using ptc::lanemask_lt;
using ptc::swap_test;
using ptc::wave_sum;

struct PtArgs {
    const int32_t *image;
    const uint32_t *mtab;  // [K][row_len]
    const uint32_t *stab;  // [K-1][7*512]
    const int32_t *snd;    // [K-1]
    int8_t *final_spins;
    long long *final_E;
    int8_t *top_spins;
    long long *top_E;
    int32_t *top_count;
    int8_t *tops;  // [runs][L][10][n], position order
    PtResume rs;   // checkpoint to start from
    int n, D, C, K, chains, sweeps, row_len, nqa, icm_lo, icm_hi, nw_icm;
    uint32_t sweep_offset, k0, k1;
};

struct PtLds {
    uint32_t *nbr;
    int32_t *hpos, *ord, *pos;
    uint32_t *tab;
    uint32_t *S;
    unsigned char *Sb;
    long long *E;      // [cK]
    long long *LE;     // [L][10]
    int32_t *Lwhen;    // [L][10]
    int32_t *Lcnt;     // [L]
    int32_t *Lbad;     // [L] checkpoint count was outside 0..10
    int32_t *Lord;     // [L][10]
    int32_t *acc;      // [cK]
    uint32_t *vis;     // [nw_icm][nwords]
    uint16_t *queue;   // [nw_icm][n]
};

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t pt_layout(int n, int D, int K, int chains, int row_len, int nqa,
                                            int nw_icm, PtLds *L, unsigned char *base) {
    const int cK = chains * K, Ls = chains * (K / 2), nwords = (n + 31) / 32;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = al16(o + bytes);
        return at;
    };
    const size_t o_nbr = take((size_t)n * D * 4), o_h = take((size_t)n * 4), o_ord = take((size_t)n * 4),
                 o_pos = take((size_t)n * 4), o_tab = take((size_t)K * row_len * 4),
                 o_S = take((size_t)n * nqa * 4), o_E = take((size_t)cK * 8), o_LE = take((size_t)Ls * 80),
                 o_Lw = take((size_t)Ls * 40), o_Lc = take((size_t)Ls * 4), o_Lb = take((size_t)Ls * 4),
                 o_Lo = take((size_t)Ls * 40),
                 o_acc = take((size_t)cK * 4 + 4), o_vis = take((size_t)nw_icm * nwords * 4),
                 o_q = take((size_t)nw_icm * n * 2);
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
        L->acc = reinterpret_cast<int32_t *>(base + o_acc);
        L->vis = reinterpret_cast<uint32_t *>(base + o_vis);
        L->queue = reinterpret_cast<uint16_t *>(base + o_q);
    }
    return o;
}

template <int ND>
__global__ __launch_bounds__(1024) void pt_kernel(PtArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cs[kMaxColours + 1];
    __shared__ int nacc;
    PtLds L;
    const int n = a.n, D = a.D, K = a.K, chains = a.chains, nqa = a.nqa;
    pt_layout(n, D, K, chains, a.row_len, nqa, a.nw_icm, &L, smem);
    const int tid = threadIdx.x, T = blockDim.x, lane = dev::lane_id(), wid = tid >> 6, nw = T >> 6;
    const int run = blockIdx.x;
    const int cK = chains * K, half = K / 2, Ls = chains * half, nwords = (n + 31) / 32;
    const int r0 = run * cK;
    const int qf = r0 >> 2;  // first quad of the run's window
    const int32_t *img = a.image;

    if (tid <= a.C) cs[tid] = img[3 + tid];
    for (int idx = tid; idx < n * D; idx += T) {  // neighbour-major in LDS: nbr[k][p]
        const int p = idx / D, k = idx - p * D;
        L.nbr[(size_t)k * n + p] = reinterpret_cast<const uint32_t *>(img + kImgHeader + 3 * n)[idx];
    }
    for (int k = tid; k < n; k += T) {
        L.ord[k] = img[kImgHeader + k];
        L.pos[k] = img[kImgHeader + n + k];
        L.hpos[k] = img[kImgHeader + 2 * n + k];
    }
    for (int k = tid; k < K * a.row_len; k += T) L.tab[k] = a.mtab[k];
    for (int k = tid; k < cK; k += T) L.E[k] = 0;
    for (int k = tid; k < Ls; k += T) {
        const int c = a.rs.top_count ? a.rs.top_count[(size_t)run * Ls + k] : 0;
        const bool bad = c < 0 || c > 10;
        L.Lcnt[k] = bad ? 0 : c;
        L.Lbad[k] = bad ? 1 : 0;
    }
    __syncthreads();
    if (a.rs.top_count) {
        // Checkpoint entries, inserted before this launch's offers in list order.
        for (int le = tid; le < Ls * 10; le += T) {
            const int li = le / 10, e = le - li * 10;
            if (e < L.Lcnt[li]) {
                L.LE[le] = a.rs.top_E[(size_t)run * Ls * 10 + le];
                L.Lwhen[le] = e - 10;
            }
        }
        for (size_t idx = tid; idx < (size_t)Ls * 10 * n; idx += T) {
            const int lr = (int)(idx / n), i = (int)(idx - (size_t)lr * n);
            if (lr % 10 < L.Lcnt[lr / 10]) {
                const size_t row = (size_t)run * Ls * 10 + lr;
                a.tops[row * n + L.pos[i]] = a.rs.top_spins[row * n + i] > 0 ? (int8_t)1 : (int8_t)-1;
            }
        }
    }

    const int q = tid % nqa, slot_t = tid / nqa, nslots = T / nqa;
    const bool active = slot_t < nslots;
    // Replicas of this thread's quad: owned flag, local index l = r - r0, slot.
    bool own[4];
    int loc[4];
    const uint32_t *tb[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int r = 4 * (qf + q) + b;
        own[b] = active && r >= r0 && r < r0 + cK;
        loc[b] = r - r0;
        const int sl = own[b] ? loc[b] % K : 0;
        tb[b] = L.tab + (size_t)sl * a.row_len;
    }
    const uint32_t quad = (uint32_t)(qf + q);
    auto nbr_rec = [=](int k, int p) __attribute__((always_inline)) -> uint32_t { return L.nbr[(size_t)k * n + p]; };
    const bool pow2 = (nqa & (nqa - 1)) == 0 && nqa <= 64;

    // Initial state and energies.
    for (int p = slot_t; active && p < n; p += nslots) {
        const dev::Words4 w = dev::philox((uint32_t)L.ord[p], 0u, quad, 1u << 24, a.k0, a.k1);
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) word |= ((w.w[b] >> 31) ? 0x01u : 0xFFu) << (8 * b);
        L.S[(size_t)p * nqa + q] = word;
    }
    __syncthreads();
    if (a.rs.spins) {
        // The run's own replicas start from the checkpoint (a neighbouring run's
        // bytes of a shared quad keep their Philox values; they are never read back).
        for (int idx = tid; idx < cK * n; idx += T) {
            const int l = idx / n, i = idx - l * n;
            const int r = r0 + l;
            L.Sb[((size_t)L.pos[i] * nqa + ((r >> 2) - qf)) * 4 + (r & 3)] =
                a.rs.spins[(size_t)r * n + i] > 0 ? (unsigned char)0x01 : (unsigned char)0xFF;
        }
        __syncthreads();
    }
    {
        long long e2[4] = {0, 0, 0, 0};
        for (int p = slot_t; active && p < n; p += nslots) {
            const uint32_t self = L.S[(size_t)p * nqa + q];
            int32_t f[4];
            ptc::quad_fields(nbr_rec, D, p, L.S, nqa, q, L.hpos[p], f);
#pragma unroll
            for (int b = 0; b < 4; ++b) e2[b] += (long long)dev::spin_of(self, b) * ((long long)L.hpos[p] + f[b]);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if (own[b]) atomicAdd(reinterpret_cast<unsigned long long *>(&L.E[loc[b]]), (unsigned long long)e2[b]);
    }
    __syncthreads();
    for (int l = tid; l < cK; l += T) L.E[l] /= 2;  // sum of s(h + f) counts every coupler twice
    __syncthreads();

    // Race-detection build: each class pass's spin-word writes, then its neighbour
    // reads, against the LDS bitmap (a word is (position, quad)).
    const shadow::Pass sh = shadow::begin((uint32_t)n * (uint32_t)nqa);
    auto shadow_pass = [&](int c, bool before) {
        const int pe = cs[c + 1];
        if (before) {
            for (int p = cs[c] + slot_t; active && p < pe; p += nslots) shadow::mark(sh, (uint32_t)(p * nqa + q));
            shadow::barrier();
            for (int p = cs[c] + slot_t; active && p < pe; p += nslots)
                for (int k = 0; k < D; ++k) {
                    const uint32_t rec = nbr_rec(k, p);
                    if ((rec & 0xffffu) != 0u) shadow::check(sh, (rec >> 16) * (uint32_t)nqa + (uint32_t)q);
                }
            shadow::count_pass(sh);
        } else {
            for (int p = cs[c] + slot_t; active && p < pe; p += nslots) shadow::unmark(sh, (uint32_t)(p * nqa + q));
            shadow::barrier();
        }
    };

    for (int ls = 0; ls < a.sweeps; ++ls) {
        const uint32_t t = a.sweep_offset + (uint32_t)ls;
        // 1. Metropolis on every slot.
        long long dE[4] = {0, 0, 0, 0};
        for (int c = 0; c < a.C; ++c) {
            if constexpr (shadow::kOn) shadow_pass(c, true);
            const int pe = cs[c + 1];
            for (int p = cs[c] + slot_t; active && p < pe; p += nslots) {
                const uint32_t self = L.S[(size_t)p * nqa + q];
                int32_t f[4];
                ptc::quad_fields(nbr_rec, D, p, L.S, nqa, q, L.hpos[p], f);
                int32_t x[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) x[b] = dev::spin_of(self, b) > 0 ? -f[b] : f[b];
                const uint32_t mask =
                    ptc::metropolis_mask4<ND>(x, tb, (uint32_t)L.ord[p], t, quad, a.k0, a.k1);
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (mask & (0xFEu << (8 * b))) dE[b] += 2ll * x[b];
                if (mask) L.S[(size_t)p * nqa + q] = self ^ mask;
            }
            __syncthreads();
            if constexpr (shadow::kOn) shadow_pass(c, false);
        }
        // Fold the energy changes of the sweep.
        if (pow2) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                for (int off = nqa; off < 64; off <<= 1) dE[b] += __shfl_xor(dE[b], off, 64);
            if (lane < nqa)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (own[b] && dE[b]) atomicAdd(reinterpret_cast<unsigned long long *>(&L.E[loc[b]]), (unsigned long long)dE[b]);
        } else {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (own[b] && dE[b]) atomicAdd(reinterpret_cast<unsigned long long *>(&L.E[loc[b]]), (unsigned long long)dE[b]);
        }
        if (tid == 0) nacc = 0;
        __syncthreads();
        // 2. Replica exchange.
        {
            const int par = (int)(t & 1u);
            const int npairs = (K - par) / 2;
            if (tid < chains * npairs) {
                const int ch = tid / npairs, m = tid - ch * npairs, k = par + 2 * m;
                const long long Dd = L.E[ch * K + k] - L.E[ch * K + k + 1];
                if (swap_test(Dd, a.stab + (size_t)k * 7 * kDigitSize, a.snd[k], (uint32_t)k, t,
                              (uint32_t)(run * chains + ch), a.k0, a.k1)) {
                    const long long e = L.E[ch * K + k];
                    L.E[ch * K + k] = L.E[ch * K + k + 1];
                    L.E[ch * K + k + 1] = e;
                    L.acc[atomicAdd(&nacc, 1)] = ch * K + k;
                }
            }
        }
        __syncthreads();
        const int na = nacc;
        if (na) {
            for (int idx = tid; idx < n * na; idx += T) {
                const int pr = idx / n, p = idx - pr * n;
                const int la = L.acc[pr], lb = la + 1;
                const int ra = r0 + la, rb = r0 + lb;
                unsigned char *A = L.Sb + ((size_t)p * nqa + ((ra >> 2) - qf)) * 4 + (ra & 3);
                unsigned char *B = L.Sb + ((size_t)p * nqa + ((rb >> 2) - qf)) * 4 + (rb & 3);
                const unsigned char x = *A;
                *A = *B;
                *B = x;
            }
            __syncthreads();
        }
        // 3. Houdayer cluster moves between chains 0 and 1.
        if (a.nw_icm > 0 && wid < a.nw_icm) {
            uint32_t *vis = L.vis + (size_t)wid * nwords;
            uint16_t *queue = L.queue + (size_t)wid * n;
            for (int k = a.icm_lo + wid; k < a.icm_hi; k += a.nw_icm) {
                const int la = k, lb = K + k;
                const int ra = r0 + la, rb = r0 + lb;
                const size_t qa_ = (size_t)((ra >> 2) - qf), qb_ = (size_t)((rb >> 2) - qf);
                const int ba = ra & 3, bb = rb & 3;
                auto byteA = [=](int p) __attribute__((always_inline)) -> unsigned char * { return L.Sb + ((size_t)p * nqa + qa_) * 4 + ba; };
                auto byteB = [=](int p) __attribute__((always_inline)) -> unsigned char * { return L.Sb + ((size_t)p * nqa + qb_) * 4 + bb; };
                // sites where the replicas disagree, counted in variable-index order
                int n_neg = 0;
                for (int i0 = 0; i0 < n; i0 += 64) {
                    const int i = i0 + lane;
                    bool f = false;
                    if (i < n) {
                        const int p = L.pos[i];
                        f = *byteA(p) != *byteB(p);
                    }
                    n_neg += __popcll(__ballot(f));
                }
                if (n_neg == 0) continue;
                const uint32_t w = dev::philox((uint32_t)k, t, (uint32_t)run, 4u << 24, a.k0, a.k1).w[0];
                const int target = (int)(((unsigned long long)w * (unsigned long long)n_neg) >> 32);
                int seed_p = -1, seen = 0;
                for (int i0 = 0; i0 < n && seed_p < 0; i0 += 64) {
                    const int i = i0 + lane;
                    bool f = false;
                    int p = 0;
                    if (i < n) {
                        p = L.pos[i];
                        f = *byteA(p) != *byteB(p);
                    }
                    const unsigned long long m = __ballot(f);
                    const int cnt = __popcll(m);
                    if (target < seen + cnt) {
                        const bool me = f && (seen + __popcll(m & lanemask_lt())) == target;
                        const unsigned long long who = __ballot(me);
                        const int src = __ffsll((long long)who) - 1;
                        seed_p = __shfl(p, src, 64);
                    }
                    seen += cnt;
                }
                for (int wd = lane; wd < nwords; wd += 64) vis[wd] = 0u;
                __builtin_amdgcn_wave_barrier();
                if (lane == 0) {
                    vis[seed_p >> 5] = 1u << (seed_p & 31);
                    queue[0] = (uint16_t)seed_p;
                }
                __builtin_amdgcn_wave_barrier();
                int head = 0, tail = 1;
                while (head < tail) {
                    const int chunk = min(64, tail - head);
                    const bool act = lane < chunk;
                    const int v = act ? (int)queue[head + lane] : 0;
                    int newtail = tail;
                    for (int kk = 0; kk < D; ++kk) {
                        bool added = false;
                        int u = 0;
                        if (act) {
                            const uint32_t rec = L.nbr[(size_t)kk * n + v];
                            u = (int)(rec >> 16);
                            if ((rec & 0xffffu) != 0u && *byteA(u) != *byteB(u)) {
                                const uint32_t bit = 1u << (u & 31);
                                const uint32_t old = atomicOr(&vis[u >> 5], bit);
                                added = !(old & bit);
                            }
                        }
                        const unsigned long long m = __ballot(added);
                        if (added) queue[newtail + __popcll(m & lanemask_lt())] = (uint16_t)u;
                        newtail += __popcll(m);
                    }
                    head += chunk;
                    tail = newtail;
                    __builtin_amdgcn_wave_barrier();
                }
                // energy change of flipping the cluster, then the flips
                long long dA = 0, dB = 0;
                for (int e = lane; e < tail; e += 64) {
                    const int v = queue[e];
                    const int sA = (int)(int8_t)*byteA(v), sB = (int)(int8_t)*byteB(v);
                    dA += -2ll * L.hpos[v] * sA;
                    dB += -2ll * L.hpos[v] * sB;
                    for (int kk = 0; kk < D; ++kk) {
                        const uint32_t rec = L.nbr[(size_t)kk * n + v];
                        const int u = (int)(rec >> 16);
                        if (!((vis[u >> 5] >> (u & 31)) & 1u)) {
                            const long long Jv = (int16_t)(rec & 0xffffu);
                            dA += -2ll * Jv * sA * (int)(int8_t)*byteA(u);
                            dB += -2ll * Jv * sB * (int)(int8_t)*byteB(u);
                        }
                    }
                }
                dA = wave_sum(dA);
                dB = wave_sum(dB);
                __builtin_amdgcn_wave_barrier();
                for (int e = lane; e < tail; e += 64) {
                    const int v = queue[e];
                    *byteA(v) = (unsigned char)(-(int)(int8_t)*byteA(v));
                    *byteB(v) = (unsigned char)(-(int)(int8_t)*byteB(v));
                }
                if (lane == 0) {
                    L.E[la] += dA;
                    L.E[lb] += dB;
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (a.nw_icm > 0) __syncthreads();
        // 4. Top-10 lists of the colder half.
        for (int li = wid; li < Ls; li += nw) {
            const int ch = li / half, k = (K - half) + (li - ch * half);
            const int l = ch * K + k;
            const int r = r0 + l;
            const size_t qq = (size_t)((r >> 2) - qf);
            const int bq = r & 3;
            const long long Ec = L.E[l];
            const int cnt = L.Lcnt[li];
            long long *LE = L.LE + (size_t)li * 10;
            int32_t *LW = L.Lwhen + (size_t)li * 10;
            bool cand = cnt < 10;
            if (!cand) {
                long long worst = LE[0];
                for (int e = 1; e < 10; ++e) worst = LE[e] > worst ? LE[e] : worst;
                cand = Ec < worst;
            }
            if (!cand) continue;
            int8_t *base = a.tops + (size_t)(run * Ls + li) * 10 * n;
            bool dup = false;
            for (int e = 0; e < cnt && !dup; ++e) {
                if (LE[e] != Ec) continue;
                bool diff = false;
                for (int p = lane; p < n; p += 64)
                    diff |= base[(size_t)e * n + p] != (int8_t)L.Sb[((size_t)p * nqa + qq) * 4 + bq];
                dup = !__any(diff);
            }
            if (dup) continue;
            int victim = cnt;
            if (cnt == 10) {
                victim = 0;
                for (int e = 1; e < 10; ++e)
                    if (LE[e] > LE[victim] || (LE[e] == LE[victim] && LW[e] > LW[victim])) victim = e;
            }
            for (int p = lane; p < n; p += 64)
                base[(size_t)victim * n + p] = (int8_t)L.Sb[((size_t)p * nqa + qq) * 4 + bq];
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) {
                LE[victim] = Ec;
                LW[victim] = ls;
                if (cnt < 10) L.Lcnt[li] = cnt + 1;
            }
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
    }

    // Outputs.
    if (a.final_E)
        for (int l = tid; l < cK; l += T) a.final_E[(size_t)r0 + l] = L.E[l];
    if (a.final_spins)
        for (int idx = tid; idx < cK * n; idx += T) {
            const int l = idx / n, i = idx - l * n;
            const int r = r0 + l;
            a.final_spins[(size_t)r * n + i] =
                (int8_t)L.Sb[((size_t)L.pos[i] * nqa + ((r >> 2) - qf)) * 4 + (r & 3)];
        }
    if (a.top_E || a.top_spins || a.top_count) {
        // Rank of entry e of a list = number of entries ordered before it by (E, insertion).
        for (int le = tid; le < Ls * 10; le += T) L.Lord[le] = -1;
        __syncthreads();
        for (int le = tid; le < Ls * 10; le += T) {
            const int li = le / 10, e = le - li * 10;
            const long long *LE = L.LE + (size_t)li * 10;
            const int32_t *LW = L.Lwhen + (size_t)li * 10;
            const int cnt = L.Lcnt[li];
            if (e < cnt) {
                int rank = 0;
                for (int o = 0; o < cnt; ++o)
                    rank += (LE[o] < LE[e] || (LE[o] == LE[e] && LW[o] < LW[e])) ? 1 : 0;
                L.Lord[li * 10 + rank] = e;
            }
            if (e == 0 && a.top_count) a.top_count[(size_t)run * Ls + li] = L.Lbad[li] ? -1 : cnt;
        }
        __syncthreads();
        if (a.top_E)
            for (int le = tid; le < Ls * 10; le += T) {
                const int e = L.Lord[le];
                a.top_E[(size_t)run * Ls * 10 + le] = e >= 0 ? L.LE[(le / 10) * 10 + e] : 0x7FFFFFFFFFFFFFFFll;
            }
        if (a.top_spins)
            for (size_t idx = tid; idx < (size_t)Ls * 10 * n; idx += T) {
                const int lr = (int)(idx / n), i = (int)(idx - (size_t)lr * n);
                const int li = lr / 10, rank = lr - li * 10;
                const int e = L.Lord[li * 10 + rank];
                a.top_spins[((size_t)run * Ls + li) * 10 * n + (size_t)rank * n + i] =
                    e >= 0 ? a.tops[((size_t)(run * Ls + li) * 10 + e) * n + L.pos[i]] : (int8_t)0;
            }
    }
}

}  // namespace

size_t pt_lds_bytes(int n, int D, int K, int chains, int row_len, int nqa, int nw_icm) {
    return pt_layout(n, D, K, chains, row_len, nqa, nw_icm, nullptr, nullptr);
}

hipError_t launch_pt(const PtLaunch &P, hipStream_t s) {
    PtArgs a;
    a.image = P.image;
    a.mtab = P.mtab;
    a.stab = P.stab;
    a.snd = P.snd;
    a.final_spins = P.out->final_spins;
    a.final_E = reinterpret_cast<long long *>(P.out->final_E);
    a.top_spins = P.out->top_spins;
    a.top_E = reinterpret_cast<long long *>(P.out->top_E);
    a.top_count = P.out->top_count;
    a.tops = static_cast<int8_t *>(P.scratch);
    a.rs = P.resume;
    a.n = P.n;
    a.D = P.D;
    a.C = P.C;
    a.K = P.K;
    a.chains = P.chains;
    a.sweeps = P.sweeps;
    a.row_len = P.row_len;
    a.nqa = P.nqa;
    a.icm_lo = P.icm_lo;
    a.icm_hi = P.icm_hi;
    a.nw_icm = P.nw_icm;
    a.sweep_offset = P.sweep_offset;
    a.k0 = (uint32_t)P.seed;
    a.k1 = (uint32_t)(P.seed >> 32);
    const size_t lds = pt_lds_bytes(P.n, P.D, P.K, P.chains, P.row_len, P.nqa, P.nw_icm);
    switch (P.nd) {
        case 1:
            hipLaunchKernelGGL(pt_kernel<1>, dim3(P.runs), dim3(P.threads), lds, s, a);
            break;
        case 2:
            hipLaunchKernelGGL(pt_kernel<2>, dim3(P.runs), dim3(P.threads), lds, s, a);
            break;
        case 3:
            hipLaunchKernelGGL(pt_kernel<3>, dim3(P.runs), dim3(P.threads), lds, s, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t shadow_stats_pt(unsigned long long *out, bool reset) { return shadow::read_stats(out, reset); }

}  // namespace spv
