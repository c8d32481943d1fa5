// Instance packing, the one-instance simulated-annealing launch and the energy kernel.
//
// Sampler (Sec. III.A, "SA"): every read starts from its own Philox state (or
// a caller state) and performs one Metropolis sweep per entry of the beta
// schedule; the sample is the final state of every read.  A sweep visits the
// colour classes in order; a class is an independent set, so all of its
// spins are updated in parallel with the same result as any sequential order.
//
// Layout: the instance is renumbered by position p (colour-major, index order
// inside a class) and held in LDS as an ELL table of 32-bit records
// (neighbour position << 16 | int16 coupling).  Spins live in LDS as S[p][q]:
// one 32-bit word per (position, quad of 4 replicas), a byte per replica.  A
// lane owns one (position, quad) task: it forms the four local fields, draws
// one Philox block that serves the four replicas, and applies the integer
// threshold test, so instance data is shared by the replicas of a quad and
// every random word is used.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "device.hpp"
#include "internal.hpp"
#include "sa_core.hpp"
#include "swar_core.hpp"

namespace spv {

namespace {

__global__ __launch_bounds__(1024) void prep_order_kernel(const uint8_t *__restrict__ colour,
                                                          int n, int D, int C,
                                                          int32_t *__restrict__ image) {
    __shared__ int cnt[kMaxColours];
    __shared__ int cs[kMaxColours + 1];
    __shared__ int tmp[1024 / 64 + 1];
    int32_t *order = image + kImgHeader;
    int32_t *pos_of = order + n;
    const int tid = threadIdx.x;
    if (tid < kMaxColours) cnt[tid] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
        int c = colour[i];
        c = c < C ? c : C - 1;
        atomicAdd(&cnt[c], 1);
    }
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int c = 0; c < C; ++c) {
            cs[c] = acc;
            acc += cnt[c];
        }
        cs[C] = acc;
        image[0] = n;
        image[1] = D;
        image[2] = C;
        for (int c = 0; c <= C; ++c) image[3 + c] = cs[c];
    }
    __syncthreads();
    for (int c = 0; c < C; ++c) {
        int base = cs[c];
        for (int start = 0; start < n; start += blockDim.x) {
            const int i = start + tid;
            int ci = 0;
            if (i < n) {
                ci = colour[i];
                ci = ci < C ? ci : C - 1;
            }
            const bool flag = (i < n) && ci == c;
            int tot;
            const int pre = dev::block_exclusive_scan(flag ? 1 : 0, tmp, &tot);
            if (flag) {
                order[base + pre] = i;
                pos_of[i] = base + pre;
            }
            base += tot;
        }
    }
}

__global__ __launch_bounds__(256) void prep_nbr_kernel(const int32_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ col,
                                                       const int32_t *__restrict__ J,
                                                       const int32_t *__restrict__ h, int n,
                                                       int nnz, int D, int32_t *__restrict__ image) {
    const int32_t *order = image + kImgHeader;
    const int32_t *pos_of = order + n;
    int32_t *hpos = image + kImgHeader + 2 * n;
    uint32_t *nbr = reinterpret_cast<uint32_t *>(image + kImgHeader + 3 * n);
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int i = order[p];
    i = i < 0 ? 0 : (i >= n ? n - 1 : i);
    int rb = row_ptr[i], re = row_ptr[i + 1];
    rb = rb < 0 ? 0 : (rb > nnz ? nnz : rb);
    re = re < rb ? rb : (re > nnz ? nnz : re);
    const int deg = (re - rb) < D ? (re - rb) : D;
    for (int k = 0; k < D; ++k) {
        uint32_t rec = (uint32_t)p << 16;
        if (k < deg) {
            int j = col[rb + k];
            j = j < 0 ? 0 : (j >= n ? n - 1 : j);
            int v = J[rb + k];
            v = v > 32767 ? 32767 : (v < -32767 ? -32767 : v);
            rec = ((uint32_t)pos_of[j] << 16) | (uint32_t)(uint16_t)(int16_t)v;
        }
        nbr[(size_t)p * D + k] = rec;
    }
    hpos[p] = h[i];
}

// ND = number of threshold digits; ND = 0 selects the byte-parallel path, whose
// neighbour loop is straight-line code for a record count DK (0: any).
// BIG: the instance lives in global memory, LDS holds the tables and the spins.
// The byte-parallel body reads its own records from a.big (built beforehand by
// big_prep_kernel); the general body reads the prepared image itself.
template <int ND, int DK = 0, bool BIG = false>
__global__ __launch_bounds__(1024) void sa_kernel(core::SaItem a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cs[kMaxColours + 1];
    a.q0 = blockIdx.x * a.qw;
    if constexpr (ND == 0) {
        core::SwarLds L;
        if constexpr (BIG) {
            core::swar_big_layout(a.n, a.qw, &L, smem);
            core::swar_bind_big(&L, a.big, a.n, a.D);
            core::swar_load_colours(a, cs);
        } else {
            core::swar_layout(a.n, a.D, a.row_len, a.qw, &L, smem);
            core::swar_load_instance(L, a, cs);
        }
        if (a.wpl == 2 && a.qw == 2)
            core::swar_run<DK, 2, BIG>(L, a, cs);
        else
            core::swar_run<DK, 1, BIG>(L, a, cs);
    } else if constexpr (BIG) {
        core::SaLds L;
        core::sa_big_layout(a.n, a.row_len, a.qw, &L, smem);
        core::sa_bind_image(&L, a, cs);
        core::sa_run<ND, true>(L, a, cs);
    } else {
        core::SaLds L;
        core::sa_layout(a.n, a.D, a.row_len, a.qw, &L, smem);
        core::sa_load_instance(L, a, cs);
        core::sa_run<ND>(L, a, cs);
    }
}

// Streamed byte-parallel SA: resident workgroups take (group of qw quads, chunk of
// sweeps) tasks from a counter in chunk-major order, so that the replicas are
// spread over the whole device however their count divides into workgroups.  A
// group's spin words pass from one chunk to the next through global memory as
// self-validating 32-bit words {tag, spins}, stored and polled with relaxed
// device-scope atomics (tag = chunks done, plus an abandoned-wait bit; the
// words are cleared before every launch), so no cache-wide fence is needed.  A
// spin byte of the byte-parallel body is a mask (0xFF or 0), so a word carries 4
// spin words as 4-bit nibbles under a 16-bit tag.  A task polls (bounded) until
// every word of its group carries the previous chunk's tag.  Every task uses the
// same counters as the one-launch schedule, so the sample is bit-identical.
struct StreamArgs {
    core::SaItem a;
    int G, K, Lc;    // groups, chunks per group, sweeps per chunk
    int *counter;
    uint32_t *state;  // [G][ceil(n qw / 4)] {tag << 16, 4 spin words as nibbles}
    int spin_limit;
};

constexpr uint32_t kTagPoison = 1u << 8;  // tags are chunk counts <= 255 plus this bit

// Spin word (4 mask bytes) <-> nibble (bit b = byte b).
__device__ __forceinline__ uint32_t spin_nibble(uint32_t w) {
    uint32_t m = w & 0x01010101u;
    m |= m >> 7;
    m |= m >> 14;
    return m & 0xFu;
}
__device__ __forceinline__ uint32_t spin_word(uint32_t nib) { return ((nib * 0x00204081u) & 0x01010101u) * 0xFFu; }

// Every branch of the task loop depends on wave-uniform values only (the task
// index is read back with readfirstlane), so that no lane can be split from its
// wave across loop iterations and barriers.
template <int DK, int W, bool BIG = false>
__global__ __launch_bounds__(1024) void sa_stream_kernel(StreamArgs s) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cs[kMaxColours + 1];
    __shared__ int task_s, late_s, poison_s;
    core::SwarLds L;
    if constexpr (BIG) {
        core::swar_big_layout(s.a.n, s.a.qw, &L, smem);
        core::swar_bind_big(&L, s.a.big, s.a.n, s.a.D);
        core::swar_load_colours(s.a, cs);
    } else {
        core::swar_layout(s.a.n, s.a.D, s.a.row_len, s.a.qw, &L, smem);
        core::swar_load_instance(L, s.a, cs);
    }
    const int ntask = s.G * s.K, T = blockDim.x, tid = threadIdx.x;
    const int words = s.a.n * s.a.qw, hw = (words + 3) / 4;
    const uint32_t inv = (uint32_t)words;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (;;) {
        if (wave == 0) {
            // one increment per workgroup: lane 0 adds 1, the others 0
            const int v = __hip_atomic_fetch_add(s.counter, threadIdx.x == 0 ? 1 : 0, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            if (threadIdx.x == 0) {
                task_s = v;
                late_s = 0;
                poison_s = 0;
            }
        }
        __syncthreads();
        const int tau = __builtin_amdgcn_readfirstlane(task_s);
        if (tau >= ntask) break;
        const int g = tau % s.G, k = tau / s.G;
        uint32_t *st = s.state + (size_t)g * (size_t)hw;
        if (k > 0) {
            // resume: every word must carry this launch's tag for k chunks done
            const uint32_t want = (uint32_t)k;
            bool late = false, poison = false;
            for (int h = tid; h < hw; h += T) {
                uint32_t v = 0;
                for (int spins = 0;; ++spins) {
                    v = __hip_atomic_load(st + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (((v >> 16) & ~kTagPoison) == want) break;
                    if (spins >= s.spin_limit) {
                        late = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                poison |= ((v >> 16) & kTagPoison) != 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int w = 4 * h + q;
                    if (w < words) {
                        const uint32_t word = spin_word((v >> (4 * q)) & 0xFu);
                        L.S[w] = word;
                        L.S[w + inv] = ~word;
                    }
                }
            }
            if (late) late_s = 1;
            if (poison) poison_s = 1;
        }
        __syncthreads();
        const bool poisoned = (__builtin_amdgcn_readfirstlane(late_s) | __builtin_amdgcn_readfirstlane(poison_s)) != 0;
        const bool late = __builtin_amdgcn_readfirstlane(late_s) != 0;
        core::SaItem it = s.a;
        it.q0 = g * s.a.qw;
        core::SwarChunk ch;
        ch.ls0 = k * s.Lc;
        ch.count = min(s.Lc, s.a.sweeps - ch.ls0);
        // An abandoned wait restarts the group from its initial state: words that may
        // still be in flight are not used.
        ch.resume = k > 0 && !late;
        ch.keep = k + 1 < s.K;
        ch.poisoned = poisoned;
        core::swar_run<DK, W, BIG>(L, it, cs, ch);  // ends with a barrier
        if (ch.keep) {
            const uint32_t tag = (poisoned ? kTagPoison : 0u) | (uint32_t)(k + 1);
            for (int h = tid; h < hw; h += T) {
                uint32_t pay = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (4 * h + q < words) pay |= spin_nibble(L.S[4 * h + q]) << (4 * q);
                __hip_atomic_store(st + h, (tag << 16) | pay, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// Task counter and tags back to zero (no word then matches a chunk tag >= 1).
__global__ void stream_reset_kernel(int *counter, uint32_t *state, size_t words) {
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) *counter = 0;
    for (size_t i = i0; i < words; i += (size_t)gridDim.x * blockDim.x) state[i] = 0u;
}

// The global-memory instance of the byte-parallel body (record addresses relative
// to the spin words).
__global__ __launch_bounds__(256) void big_prep_kernel(core::SaItem a) {
    core::SwarLds L;
    core::swar_bind_big(&L, a.big, a.n, a.D);
    core::swar_build(L.rec, L.co, L.hpos, a, 0u, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// Energies of arbitrary states: one workgroup per 64 rows... one thread per (row, variable).
__global__ __launch_bounds__(256) void energy_kernel(const int32_t *__restrict__ image, int n,
                                                     int D, const int8_t *__restrict__ spins,
                                                     int R, long long *__restrict__ E) {
    // 2E = sum_i s_i (2 h_i + sum_j J_ij s_j); each workgroup handles one row.
    const int r = blockIdx.x;
    if (r >= R) return;
    const int32_t *order = image + kImgHeader;
    const int32_t *pos_of = order + n;
    const int32_t *hpos = order + 2 * n;
    const uint32_t *nbr = reinterpret_cast<const uint32_t *>(order + 3 * n);
    const int8_t *s = spins + (size_t)r * n;
    long long acc = 0;
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
        const int i = order[p];
        long long f = 2ll * hpos[p];
        for (int k = 0; k < D; ++k) {
            const uint32_t rec = nbr[(size_t)p * D + k];
            const int jp = (int)(rec >> 16);
            f += (long long)(int16_t)(rec & 0xffffu) * s[order[jp]];
        }
        acc += (long long)s[i] * f;
    }
    (void)pos_of;
    __shared__ long long part[256 / 64];
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_down(acc, d, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long tot = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += part[w];
        E[r] = tot / 2;
    }
}

}  // namespace

hipError_t launch_prep(const Inst *P, int32_t *image, hipStream_t s) {
    hipLaunchKernelGGL(prep_order_kernel, dim3(1), dim3(1024), 0, s, P->colour, P->n,
                       P->max_degree, P->n_colours, image);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (P->n > 0) {
        hipLaunchKernelGGL(prep_nbr_kernel, dim3((P->n + 255) / 256), dim3(256), 0, s,
                           P->row_ptr, P->col, P->J, P->h, P->n, P->nnz, P->max_degree, image);
        e = hipGetLastError();
    }
    return e;
}

// The byte-parallel path serves single-digit tables of at most 256 entries
// (x_bound <= 255); SPVAR_NO_SWAR=1 forces the general path (for comparisons).
bool sa_use_swar(int nd, int row_len) {
    static const bool off = [] {
        const char *v = getenv("SPVAR_NO_SWAR");
        return v && v[0] == '1';
    }();
    return nd == 1 && row_len <= 256 && !off;
}

size_t sa_lds_bytes(int n, int D, int row_len, int qw, bool big) {
    if (sa_use_swar(1 + (row_len > kDigitSize ? 1 : 0), row_len))
        return big ? core::swar_big_lds_bytes(n, qw) : core::swar_layout(n, D, row_len, qw, nullptr, nullptr);
    return big ? core::sa_big_layout(n, row_len, qw, nullptr, nullptr)
               : core::sa_layout(n, D, row_len, qw, nullptr, nullptr);
}

size_t sa_big_bytes(int n, int D) { return core::swar_big_bytes(n, D); }

static hipError_t launch_big_prep(const core::SaItem &a, hipStream_t s) {
    const size_t work = (size_t)a.n * (size_t)core::swar_rec_stride(a.D);
    const int grid = (int)std::min<size_t>(4096, std::max<size_t>(1, (work + 255) / 256));
    hipLaunchKernelGGL(big_prep_kernel, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sa(const SaLaunch &L, hipStream_t s, size_t lds_limit) {
    core::SaItem a;
    a.image = L.image;
    a.tables = L.tables;
    a.init = L.init;
    a.out = L.out;
    a.energies = L.energies;
    a.n = L.n;
    a.D = L.D;
    a.C = L.C;
    a.row_len = L.row_len;
    a.sweeps = L.sweeps;
    a.reads = L.reads;
    a.q0 = 0;
    a.qw = L.qw;
    a.sweep_offset = L.sweep_offset;
    a.wpl = (L.wpl == 2 && L.qw == 2) ? 2 : 1;
    a.k0 = (uint32_t)L.seed;
    a.k1 = (uint32_t)(L.seed >> 32);
    a.big = L.big;
    const bool swar = sa_use_swar(L.nd, L.row_len);
    const bool big = L.global_instance;
    const size_t lds = sa_lds_bytes(L.n, L.D, L.row_len, L.qw, big);
    if (lds > lds_limit || (big && swar && L.big == nullptr)) return hipErrorInvalidValue;
    const int quads = (L.reads + 3) / 4;
    const int grid = (quads + L.qw - 1) / L.qw;
    if (big && !swar) {
        switch (L.nd) {
            case 1:
                hipLaunchKernelGGL((sa_kernel<1, 0, true>), dim3(grid), dim3(L.threads), lds, s, a);
                break;
            case 2:
                hipLaunchKernelGGL((sa_kernel<2, 0, true>), dim3(grid), dim3(L.threads), lds, s, a);
                break;
            case 3:
                hipLaunchKernelGGL((sa_kernel<3, 0, true>), dim3(grid), dim3(L.threads), lds, s, a);
                break;
            default:
                return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (big) {
        hipError_t e = launch_big_prep(a, s);
        if (e != hipSuccess) return e;
        if (L.D == 6)
            hipLaunchKernelGGL((sa_kernel<0, 6, true>), dim3(grid), dim3(L.threads), lds, s, a);
        else
            hipLaunchKernelGGL((sa_kernel<0, 0, true>), dim3(grid), dim3(L.threads), lds, s, a);
        return hipGetLastError();
    }
    switch (sa_use_swar(L.nd, L.row_len) ? 0 : L.nd) {
        case 0:
            if (L.D == 6)
                hipLaunchKernelGGL((sa_kernel<0, 6>), dim3(grid), dim3(L.threads), lds, s, a);
            else if (L.D == 4)
                hipLaunchKernelGGL((sa_kernel<0, 4>), dim3(grid), dim3(L.threads), lds, s, a);
            else if (L.D == 8)
                hipLaunchKernelGGL((sa_kernel<0, 8>), dim3(grid), dim3(L.threads), lds, s, a);
            else
                hipLaunchKernelGGL(sa_kernel<0>, dim3(grid), dim3(L.threads), lds, s, a);
            break;
        case 1:
            hipLaunchKernelGGL(sa_kernel<1>, dim3(grid), dim3(L.threads), lds, s, a);
            break;
        case 2:
            hipLaunchKernelGGL(sa_kernel<2>, dim3(grid), dim3(L.threads), lds, s, a);
            break;
        case 3:
            hipLaunchKernelGGL(sa_kernel<3>, dim3(grid), dim3(L.threads), lds, s, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int DK, int W, bool BIG>
static hipError_t stream_occupancy(int threads, size_t lds, int *per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, sa_stream_kernel<DK, W, BIG>, threads, lds);
}

// Chunks per group: the fewest (sweeps per chunk >= kStreamMinSweeps) whose tasks
// fill the resident workgroups to kStreamFill, else the best filling count.  Every
// chunk boundary moves a group's spin words through global memory once each way.
static int stream_chunks(int G, int sweeps, int resident) {
    constexpr int kStreamMinSweeps = 64, kStreamMaxChunks = 32;
    constexpr double kStreamFill = 0.985;
    int best = 1;
    double best_eff = 0.0;
    for (int K = 1; K <= kStreamMaxChunks && (K == 1 || sweeps / K >= kStreamMinSweeps); ++K) {
        const long long tasks = (long long)G * K;
        const long long rounds = (tasks + resident - 1) / resident;
        const double eff = (double)tasks / (double)(rounds * resident);
        if (eff >= kStreamFill) return K;
        if (eff > best_eff + 1e-3) {
            best_eff = eff;
            best = K;
        }
    }
    return best;
}

size_t sa_stream_bytes(int n, int reads, int qw) {
    const size_t G = (size_t)((reads + 3) / 4 + qw - 1) / (size_t)qw;
    return 256 + G * (((size_t)n * (size_t)qw + 3) / 4) * 4;
}

// Chunks per group for a streamed launch of L, or 1 when the plain launch is used
// (not the byte-parallel body, one wave of workgroups covers the replicas, or a
// short schedule).
int sa_stream_plan(const SaLaunch &L, int num_cus, int force_grid) {
    if (!sa_use_swar(L.nd, L.row_len)) return 1;
    if (force_grid > 0) {  // tests: a given grid, chunk dependencies whatever the shape
        const int K = std::max(2, std::min(32, L.sweeps / 16));
        return L.sweeps >= 2 ? (K | (force_grid << 8)) : 1;
    }
    if (L.sweeps < 128) return 1;
    const int quads = (L.reads + 3) / 4;
    const int G = (quads + L.qw - 1) / L.qw;
    const int W = (L.wpl == 2 && L.qw == 2) ? 2 : 1;
    const bool big = L.global_instance;
    const size_t lds = sa_lds_bytes(L.n, L.D, L.row_len, L.qw, big);
    const int dk = (L.D == 6 || L.D == 4 || L.D == 8) ? L.D : 0;
    int per_cu = 0;
    hipError_t e;
#define SPV_OCC(D_, W_) e = stream_occupancy<D_, W_, false>(L.threads, lds, &per_cu)
    if (big) {
        if (dk == 6) {
            if (W == 2) e = stream_occupancy<6, 2, true>(L.threads, lds, &per_cu);
            else e = stream_occupancy<6, 1, true>(L.threads, lds, &per_cu);
        } else {
            if (W == 2) e = stream_occupancy<0, 2, true>(L.threads, lds, &per_cu);
            else e = stream_occupancy<0, 1, true>(L.threads, lds, &per_cu);
        }
    } else if (W == 2) {
        if (dk == 6) SPV_OCC(6, 2); else if (dk == 4) SPV_OCC(4, 2); else if (dk == 8) SPV_OCC(8, 2); else SPV_OCC(0, 2);
    } else {
        if (dk == 6) SPV_OCC(6, 1); else if (dk == 4) SPV_OCC(4, 1); else if (dk == 8) SPV_OCC(8, 1); else SPV_OCC(0, 1);
    }
#undef SPV_OCC
    const int resident = per_cu * num_cus;
    if (e != hipSuccess || resident <= 0 || G <= resident) return 1;
    const char *kv = getenv("SPVAR_SA_CHUNKS");  // tuning: a fixed chunk count
    const int K = kv && atoi(kv) > 0 ? std::min(255, atoi(kv)) : stream_chunks(G, L.sweeps, resident);
    return K <= 1 ? 1 : (K | (resident << 8));
}

int sa_stream_chunks_of(const SaLaunch &L, int plan) {
    const int K0 = plan & 0xff;
    const int Lc = (L.sweeps + K0 - 1) / K0;
    return (L.sweeps + Lc - 1) / Lc;
}

hipError_t launch_sa_stream(const SaLaunch &L, int plan, void *buf, hipStream_t s) {
    const int K0 = plan & 0xff, resident = plan >> 8;
    const int quads = (L.reads + 3) / 4;
    const int G = (quads + L.qw - 1) / L.qw;
    const int W = (L.wpl == 2 && L.qw == 2) ? 2 : 1;
    const bool big = L.big != nullptr;
    const size_t lds = sa_lds_bytes(L.n, L.D, L.row_len, L.qw, big);
    const int dk = (L.D == 6 || L.D == 4 || L.D == 8) ? L.D : 0;
    StreamArgs a;
    a.a.image = L.image;
    a.a.tables = L.tables;
    a.a.init = L.init;
    a.a.out = L.out;
    a.a.energies = L.energies;
    a.a.n = L.n;
    a.a.D = L.D;
    a.a.C = L.C;
    a.a.row_len = L.row_len;
    a.a.sweeps = L.sweeps;
    a.a.reads = L.reads;
    a.a.q0 = 0;
    a.a.qw = L.qw;
    a.a.sweep_offset = L.sweep_offset;
    a.a.k0 = (uint32_t)L.seed;
    a.a.k1 = (uint32_t)(L.seed >> 32);
    a.a.wpl = W;
    a.a.big = L.big;
    a.G = G;
    a.Lc = (L.sweeps + K0 - 1) / K0;
    a.K = (L.sweeps + a.Lc - 1) / a.Lc;
    unsigned char *b = static_cast<unsigned char *>(buf);
    a.counter = reinterpret_cast<int *>(b);
    a.state = reinterpret_cast<uint32_t *>(b + 256);
    a.spin_limit = L.spin_limit;
    const size_t words = (size_t)G * (((size_t)L.n * (size_t)L.qw + 3) / 4);
    const int rgrid = (int)std::min<size_t>(1024, std::max<size_t>(1, (words + 255) / 256));
    hipLaunchKernelGGL(stream_reset_kernel, dim3(rgrid), dim3(256), 0, s, a.counter, a.state, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int grid = std::min(resident, G * a.K);
    if (big) {
        e = launch_big_prep(a.a, s);
        if (e != hipSuccess) return e;
        if (dk == 6) {
            if (W == 2) hipLaunchKernelGGL((sa_stream_kernel<6, 2, true>), dim3(grid), dim3(L.threads), lds, s, a);
            else hipLaunchKernelGGL((sa_stream_kernel<6, 1, true>), dim3(grid), dim3(L.threads), lds, s, a);
        } else {
            if (W == 2) hipLaunchKernelGGL((sa_stream_kernel<0, 2, true>), dim3(grid), dim3(L.threads), lds, s, a);
            else hipLaunchKernelGGL((sa_stream_kernel<0, 1, true>), dim3(grid), dim3(L.threads), lds, s, a);
        }
        return hipGetLastError();
    }
#define SPV_GO(D_, W_) hipLaunchKernelGGL((sa_stream_kernel<D_, W_>), dim3(grid), dim3(L.threads), lds, s, a)
    if (W == 2) {
        if (dk == 6) SPV_GO(6, 2); else if (dk == 4) SPV_GO(4, 2); else if (dk == 8) SPV_GO(8, 2); else SPV_GO(0, 2);
    } else {
        if (dk == 6) SPV_GO(6, 1); else if (dk == 4) SPV_GO(4, 1); else if (dk == 8) SPV_GO(8, 1); else SPV_GO(0, 1);
    }
#undef SPV_GO
    return hipGetLastError();
}

hipError_t launch_energy(const int32_t *image, int n, int D, const int8_t *spins, int R,
                         int64_t *E, hipStream_t s) {
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL(energy_kernel, dim3(R), dim3(256), 0, s, image, n, D, spins, R,
                       reinterpret_cast<long long *>(E));
    return hipGetLastError();
}

hipError_t shadow_stats_sa(unsigned long long *out, bool reset) { return shadow::read_stats(out, reset); }

}  // namespace spv
