// Persistence and reduction (Algorithm 1: elite selection, per-variable
// agreement, fixing, "Update J and h"), with the zero-bias gauge of Sec. II.C.
//
// Pipeline (all stream-ordered, no host round trip):
//   1. elite_kernel   one workgroup: radix-selects the m-th smallest (E, row)
//                     key and emits the elite rows in row order.
//   2. bitmap_kernel  a wavefront takes 64 elite rows; for each variable a
//                     ballot of "s = +1" over the 64 lanes is one 64-bit word
//                     of that variable's column bitmap P_i (W = ceil(m/64)
//                     words per variable).  Counts are popcounts of P_i.
//   3. gauge kernels  (optional) hash every canonical column (P_i, or its
//                     complement when the first elite row holds -1) into an
//                     open-addressing table; the largest class (ties: lower
//                     minimum index) gives the pivot p; members of the pivot
//                     class are verified word by word.
//   4. fix_reduce     one workgroup: c_i = 2 popc(P_i) - m, or with the gauge
//                     c_i = m - 2 popc(P_i xor P_p); fix iff |c_i| >= k_min;
//                     scans for the new numbering, emits the reduced CSR,
//                     folds fixed neighbours into h', reduces the offset.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device.hpp"
#include "internal.hpp"

namespace spv {

// Scratch of the allocation-free persistence entry point: one copy per device,
// alive until the process ends.  Host code never passes this name to a kernel
// (on the host it is only a stand-in); it uses the per-device address that
// noalloc_scratch looks up.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(int device, void **ptr) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // `device` is current
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

namespace {

// Scratch layout (bytes, all 8-aligned):
//   int64 status, pivot, m-info ... (header, 64 bytes)
//   int32 elite[R]
//   uint64 bits[n][W]
//   uint64 hash[n]
//   uint64 tab_key[TS], int32 tab_cnt[TS], int32 tab_min[TS]
//   int32 newid[n], int32 kept[n]
struct FixScratch {
    long long *hdr;  // [0] status, [1] pivot, [2] all-h-zero flag
    int32_t *elite;
    unsigned long long *bits;
    unsigned long long *hash;
    unsigned long long *tkey;
    int32_t *tcnt;
    int32_t *tmin;
    int32_t *newid;
    int32_t *kept;
    int TS;
    int W;
};

inline size_t align8(size_t x) { return (x + 7) & ~(size_t)7; }

inline int table_size(int n) {
    int ts = 64;
    while (ts < 2 * n) ts <<= 1;
    return ts;
}

FixScratch carve(void *base, int n, int R, int m) {
    FixScratch f;
    unsigned char *p = static_cast<unsigned char *>(base);
    const int W = (m + 63) / 64;
    const int TS = table_size(n);
    f.hdr = reinterpret_cast<long long *>(p);
    p += 64;
    f.elite = reinterpret_cast<int32_t *>(p);
    p += align8((size_t)R * 4);
    f.bits = reinterpret_cast<unsigned long long *>(p);
    p += (size_t)n * W * 8;
    f.hash = reinterpret_cast<unsigned long long *>(p);
    p += (size_t)n * 8;
    f.tkey = reinterpret_cast<unsigned long long *>(p);
    p += (size_t)TS * 8;
    f.tcnt = reinterpret_cast<int32_t *>(p);
    p += (size_t)TS * 4;
    f.tmin = reinterpret_cast<int32_t *>(p);
    p += (size_t)TS * 4;
    f.newid = reinterpret_cast<int32_t *>(p);
    p += align8((size_t)n * 4);
    f.kept = reinterpret_cast<int32_t *>(p);
    f.TS = TS;
    f.W = W;
    return f;
}

__device__ __forceinline__ unsigned long long order_key(long long e) {
    return (unsigned long long)e ^ 0x8000000000000000ull;
}

// 1. Elite selection: the first m rows in (E, row) order, emitted by row.
// The m-th smallest key is found by a radix select, most significant byte
// first, that starts at the highest byte in which the smallest and largest keys
// differ (the bytes above are common to every key, so every pass over them
// would keep all keys and the rank unchanged).  Each wavefront counts into its
// own histogram, so keys sharing a byte value do not serialise on one counter.
__global__ __launch_bounds__(1024) void elite_kernel(const long long *__restrict__ E, int R, int m,
                                                     FixScratch f) {
    constexpr int kWaves = 1024 / 64;
    __shared__ unsigned int hist[kWaves][256];
    __shared__ unsigned long long kmin_w[kWaves], kmax_w[kWaves];
    __shared__ unsigned long long prefix_s;
    __shared__ int need_s, pass0_s;
    __shared__ int tmp[1024 / 64 + 1];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
    {
        unsigned long long lo = ~0ull, hi = 0ull;
        for (int r = tid; r < R; r += blockDim.x) {
            const unsigned long long key = order_key(E[r]);
            lo = key < lo ? key : lo;
            hi = key > hi ? key : hi;
        }
        for (int d = 32; d >= 1; d >>= 1) {
            const unsigned long long ol = __shfl_xor(lo, d, 64), oh = __shfl_xor(hi, d, 64);
            lo = ol < lo ? ol : lo;
            hi = oh > hi ? oh : hi;
        }
        if (lane == 0) {
            kmin_w[wid] = lo;
            kmax_w[wid] = hi;
        }
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long lo = kmin_w[0], hi = kmax_w[0];
        for (int w = 1; w < nw; ++w) {
            lo = kmin_w[w] < lo ? kmin_w[w] : lo;
            hi = kmax_w[w] > hi ? kmax_w[w] : hi;
        }
        const unsigned long long x = lo ^ hi;
        const int p0 = x == 0ull ? -1 : (63 - __clzll((long long)x)) / 8;
        pass0_s = p0;
        prefix_s = p0 < 0 ? lo : (p0 == 7 ? 0ull : lo & (~0ull << (8 * p0 + 8)));
        need_s = m;  // rank (1-based) of the wanted key among the candidates
        // INT64_MIN is no energy (|E| <= sum |J| + sum |h| < 2^62): it marks the reads of an
        // abandoned streamed sample, which must not be fixed from.
        f.hdr[0] = lo == 0ull ? (long long)SPV_EINVAL : 0;
    }
    __syncthreads();
    for (int pass = pass0_s; pass >= 0; --pass) {
        for (int k = tid; k < kWaves * 256; k += blockDim.x) (&hist[0][0])[k] = 0u;
        __syncthreads();
        const unsigned long long prefix = prefix_s;
        const int shift = 8 * pass;
        const unsigned long long hi_mask = (pass == 7) ? 0ull : (~0ull << (shift + 8));
        for (int r = tid; r < R; r += blockDim.x) {
            const unsigned long long key = order_key(E[r]);
            if ((key & hi_mask) == prefix) atomicAdd(&hist[wid][(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (tid < 256) {
            unsigned int c = 0;
            for (int w = 0; w < nw; ++w) c += hist[w][tid];
            hist[0][tid] = c;
        }
        __syncthreads();
        if (wid == 0) {
            // lane l holds bins 4l..4l+3; the first lane whose inclusive count
            // reaches the rank holds the wanted bin
            const int need = need_s;
            unsigned int c[4], sum = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c[u] = hist[0][4 * lane + u];
                sum += c[u];
            }
            unsigned int incl = sum;
            for (int d = 1; d < 64; d <<= 1) {
                const unsigned int y = __shfl_up(incl, d, 64);
                if (lane >= d) incl += y;
            }
            const unsigned long long hit = __ballot(incl >= (unsigned int)need);
            const int src = __ffsll((long long)hit) - 1;
            if (lane == src) {
                unsigned int acc = incl - sum;
                int b = 4 * lane;
#pragma unroll
                for (int u = 0; u < 3; ++u)
                    if (acc + c[u] < (unsigned int)need && b == 4 * lane + u) {
                        acc += c[u];
                        ++b;
                    }
                need_s = need - (int)acc;
                prefix_s = prefix | ((unsigned long long)b << shift);
            }
        }
        __syncthreads();
    }
    const unsigned long long kstar = prefix_s;
    const int need_eq = need_s;  // rows with key == kstar that enter the elite (lowest rows)
    // Emit, in row order: key < kstar, or key == kstar and among the first need_eq such rows.
    int out_base = 0, eq_base = 0;
    for (int start = 0; start < R; start += blockDim.x) {
        const int r = start + tid;
        unsigned long long key = 0;
        bool lt = false, eq = false;
        if (r < R) {
            key = order_key(E[r]);
            lt = key < kstar;
            eq = key == kstar;
        }
        // one scan of both counts (lt in the low 16 bits, eq in the high 16; a chunk
        // holds at most 1024 rows); the chunk takes its lt rows and its first `rem`
        // eq rows, so a taken row's slot is lt_pre + min(eq_pre, rem)
        int tot;
        const int pre = dev::block_exclusive_scan((lt ? 1 : 0) | (eq ? 1 << 16 : 0), tmp, &tot);
        const int lt_pre = pre & 0xFFFF, eq_pre = pre >> 16, lt_tot = tot & 0xFFFF, eq_tot = tot >> 16;
        const int rem = need_eq - eq_base > 0 ? need_eq - eq_base : 0;
        const bool take = lt || (eq && eq_pre < rem);
        if (take) f.elite[out_base + lt_pre + min(eq_pre, rem)] = r;
        out_base += lt_tot + min(eq_tot, rem);
        eq_base += eq_tot;
    }
}

// 2. Column bitmaps: word w of variable i = ballot over elite rows 64w..64w+63 of s = +1.
__global__ __launch_bounds__(64) void bitmap_kernel(const int8_t *__restrict__ S, int n, int m,
                                                    FixScratch f, int cols_per_block) {
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    const int e = w * 64 + lane;
    const bool valid = e < m;
    const int row = valid ? f.elite[e] : 0;
    const int8_t *srow = S + (size_t)row * n;
    const int i0 = blockIdx.y * cols_per_block;
    const int i1 = min(n, i0 + cols_per_block);
    bool bad = false;
    int i = i0;
    // rows read 4 columns at a time when every row starts on a 4-byte boundary
    // (cols_per_block is a multiple of 4, so i0 keeps that alignment)
    if ((n & 3) == 0 && (reinterpret_cast<uintptr_t>(S) & 3) == 0) {
        for (; i + 4 <= i1; i += 4) {
            const uint32_t v4 = valid ? *reinterpret_cast<const uint32_t *>(srow + i) : 0x01010101u;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int8_t v = (int8_t)(v4 >> (8 * b));
                bad |= (v != 1 && v != -1);
                const unsigned long long word = __ballot(valid && v > 0);
                if (lane == 0) f.bits[(size_t)(i + b) * f.W + w] = word;
            }
        }
    }
    for (; i < i1; ++i) {
        const int8_t v = valid ? srow[i] : (int8_t)1;
        bad |= (v != 1 && v != -1);
        const unsigned long long word = __ballot(valid && v > 0);
        if (lane == 0) f.bits[(size_t)i * f.W + w] = word;
    }
    if (__any(bad) && lane == 0) atomicMin(reinterpret_cast<long long *>(&f.hdr[0]), (long long)SPV_EINVAL);
}

__device__ __forceinline__ unsigned long long canon_word(const unsigned long long *bi, int w, int W,
                                                         int m) {
    // Canonical column: the bitmap itself when the first elite row holds +1,
    // else its complement; bits beyond m are zero.
    unsigned long long x = bi[w];
    if (!(bi[0] & 1ull)) x = ~x;
    if (w == W - 1 && (m & 63)) x &= (1ull << (m & 63)) - 1ull;
    return x;
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// 3a. Hash canonical columns into the open-addressing table.
__global__ __launch_bounds__(256) void gauge_hash_kernel(int n, int m, FixScratch f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const unsigned long long *bi = f.bits + (size_t)i * f.W;
    unsigned long long hsh = 0x6A09E667F3BCC909ull;
    for (int w = 0; w < f.W; ++w) hsh = mix64(hsh ^ mix64(canon_word(bi, w, f.W, m) + (unsigned long long)w));
    if (hsh == 0ull) hsh = 1ull;
    f.hash[i] = hsh;
    unsigned int slot = (unsigned int)(hsh & (unsigned long long)(f.TS - 1));
    for (int probe = 0; probe < f.TS; ++probe) {
        const unsigned long long prev = atomicCAS(&f.tkey[slot], 0ull, hsh);
        if (prev == 0ull || prev == hsh) {
            atomicAdd(&f.tcnt[slot], 1);
            atomicMin(&f.tmin[slot], i);
            return;
        }
        slot = (slot + 1) & (unsigned int)(f.TS - 1);
    }
}

// 3b. Largest class -> pivot; verify the pivot class exactly.
__global__ __launch_bounds__(1024) void gauge_pivot_kernel(const int32_t *__restrict__ h, int n,
                                                           int m, int mode, FixScratch f) {
    __shared__ unsigned long long best[1024 / 64];
    __shared__ int nonzero_h;
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) {
        nonzero_h = 0;
        bad = 0;
    }
    __syncthreads();
    if (mode == 2)
        for (int i = tid; i < n; i += blockDim.x)
            if (h[i] != 0) nonzero_h = 1;
    // key = count << 32 | (0xFFFFFFFF - min): larger is better (ties: lower min index)
    unsigned long long mine = 0ull;
    for (int s = tid; s < f.TS; s += blockDim.x) {
        if (f.tkey[s] != 0ull) {
            const unsigned long long k =
                ((unsigned long long)(unsigned int)f.tcnt[s] << 32) |
                (unsigned long long)(0xFFFFFFFFu - (unsigned int)f.tmin[s]);
            mine = k > mine ? k : mine;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long o = __shfl_down(mine, d, 64);
        mine = o > mine ? o : mine;
    }
    if ((tid & 63) == 0) best[tid >> 6] = mine;
    __syncthreads();
    if (tid == 0) {
        unsigned long long b = 0ull;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) b = best[w] > b ? best[w] : b;
        best[0] = b;
    }
    __syncthreads();
    const bool off = (mode == 2 && nonzero_h) || n == 0;
    const int pivot = off ? -1 : (int)(0xFFFFFFFFu - (unsigned int)(best[0] & 0xFFFFFFFFull));
    if (pivot >= 0) {
        const unsigned long long key = f.hash[pivot];
        const unsigned long long *bp = f.bits + (size_t)pivot * f.W;
        for (int i = tid; i < n; i += blockDim.x) {
            if (f.hash[i] != key) continue;
            const unsigned long long *bi = f.bits + (size_t)i * f.W;
            for (int w = 0; w < f.W; ++w)
                if (canon_word(bi, w, f.W, m) != canon_word(bp, w, f.W, m)) bad = 1;
        }
    }
    __syncthreads();
    if (tid == 0) {
        f.hdr[1] = pivot;
        if (bad) atomicMin(reinterpret_cast<long long *>(&f.hdr[0]), (long long)SPV_EINTERNAL);
    }
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ int count_of(const FixScratch &f, int i, int pivot, int m) {
    const unsigned long long *bi = f.bits + (size_t)i * f.W;
    int pos = 0;
    if (pivot < 0) {
        for (int w = 0; w < f.W; ++w) pos += __popcll(bi[w]);
        return 2 * pos - m;
    }
    const unsigned long long *bp = f.bits + (size_t)pivot * f.W;
    int diff = 0;
    for (int w = 0; w < f.W; ++w) diff += __popcll(bi[w] ^ bp[w]);  // bits beyond m are 0 in both
    return m - 2 * diff;
}

struct ReduceArgs {
    const int32_t *row_ptr;
    const int32_t *col;
    const int32_t *J;
    const int32_t *h;
    const uint8_t *colour;
    int n, nnz, m, kmin, use_pivot;
    uint8_t *fixed_mask;
    int8_t *fixed_val;
    int32_t *row_ptr_o;
    int32_t *col_o;
    int32_t *J_o;
    int32_t *h_o;
    uint8_t *colour_o;
    int32_t *orig_o;
    long long *info;
};

// 4. Fix and reduce (one workgroup; phases separated by barriers).
__global__ __launch_bounds__(1024) void fix_reduce_kernel(ReduceArgs a, FixScratch f) {
    __shared__ int tmp[1024 / 64 + 1];
    __shared__ long long part[1024 / 64];
    __shared__ int range_bad;
    const int tid = threadIdx.x, T = blockDim.x, n = a.n;
    const int pivot = a.use_pivot ? (int)f.hdr[1] : -1;
    if (tid == 0) range_bad = 0;
    // Phase A: decisions and the new numbering.
    int base = 0;
    for (int start = 0; start < n; start += T) {
        const int i = start + tid;
        bool fixed = false;
        if (i < n) {
            const int c = count_of(f, i, pivot, a.m);
            fixed = (c >= a.kmin) || (-c >= a.kmin);
            a.fixed_mask[i] = fixed ? 1 : 0;
            a.fixed_val[i] = fixed ? (c > 0 ? 1 : -1) : 0;
        }
        int tot;
        const int pre = dev::block_exclusive_scan((i < n && !fixed) ? 1 : 0, tmp, &tot);
        if (i < n) {
            f.newid[i] = fixed ? -1 : base + pre;
            if (!fixed) a.orig_o[base + pre] = i;
        }
        base += tot;
    }
    const int n_free = base;
    __syncthreads();
    // Phase B: per free row, kept entries and folded bias; offset terms.
    long long off = 0;
    for (int i = tid; i < n; i += T) {
        const int rb = clampi(a.row_ptr[i], 0, a.nnz), re = clampi(a.row_ptr[i + 1], rb, a.nnz);
        const int u = f.newid[i];
        if (u < 0) {
            const long long vi = a.fixed_val[i];
            off += (long long)a.h[i] * vi;
            for (int k = rb; k < re; ++k) {
                const int j = clampi(a.col[k], 0, n - 1);
                if (j > i && f.newid[j] < 0) off += (long long)a.J[k] * vi * a.fixed_val[j];
            }
        } else {
            long long hv = a.h[i];
            int kept = 0;
            for (int k = rb; k < re; ++k) {
                const int j = clampi(a.col[k], 0, n - 1);
                if (f.newid[j] < 0)
                    hv += (long long)a.J[k] * a.fixed_val[j];
                else
                    ++kept;
            }
            if (hv > 2147483647ll || hv < -2147483648ll) range_bad = 1;
            a.h_o[u] = (int32_t)hv;
            a.colour_o[u] = a.colour[i];
            f.kept[u] = kept;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) off += __shfl_down(off, d, 64);
    if ((tid & 63) == 0) part[tid >> 6] = off;
    __syncthreads();
    // Phase C: row pointers of the reduced CSR.
    int rbase = 0;
    if (tid == 0) a.row_ptr_o[0] = 0;
    for (int start = 0; start < n_free; start += T) {
        const int u = start + tid;
        const int v = u < n_free ? f.kept[u] : 0;
        int tot;
        const int pre = dev::block_exclusive_scan(v, tmp, &tot);
        if (u < n_free) a.row_ptr_o[u + 1] = rbase + pre + v;
        rbase += tot;
    }
    const int nnz_free = rbase;
    __syncthreads();
    // Phase D: entries of the reduced CSR.
    for (int u = tid; u < n_free; u += T) {
        const int i = a.orig_o[u];
        int o = a.row_ptr_o[u];
        const int rb = clampi(a.row_ptr[i], 0, a.nnz), re = clampi(a.row_ptr[i + 1], rb, a.nnz);
        for (int k = rb; k < re; ++k) {
            const int nj = f.newid[clampi(a.col[k], 0, n - 1)];
            if (nj >= 0) {
                a.col_o[o] = nj;
                a.J_o[o] = a.J[k];
                ++o;
            }
        }
    }
    if (tid == 0) {
        long long offset = 0;
        for (int w = 0; w < (T >> 6); ++w) offset += part[w];
        long long status = f.hdr[0];
        if (range_bad && status == 0) status = SPV_ERANGE;
        a.info[0] = n_free;
        a.info[1] = nnz_free;
        a.info[2] = offset;
        a.info[3] = n - n_free;
        a.info[4] = pivot;
        a.info[5] = a.m;
        a.info[6] = a.kmin;
        a.info[7] = status;
    }
}

__global__ void zero_kernel(unsigned long long *p, size_t words, int32_t *mins, int nmins) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < words) p[k] = 0ull;
    if (k < (size_t)nmins) mins[k] = 0x7FFFFFFF;
}

// Iterated rounds: fold a round's fixes into original indices and compose the
// reduced -> original map.
__global__ void compose_kernel(int n_cur, const uint8_t *__restrict__ fm_round,
                               const int8_t *__restrict__ fv_round,
                               const int32_t *__restrict__ orig_cur, uint8_t *__restrict__ fixed_mask,
                               int8_t *__restrict__ fixed_val, const long long *__restrict__ info,
                               const int32_t *__restrict__ orig_out, int32_t *__restrict__ orig_new) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n_cur && fm_round[u]) {
        fixed_mask[orig_cur[u]] = 1;
        fixed_val[orig_cur[u]] = fv_round[u];
    }
    if (u < (int)info[0]) orig_new[u] = orig_cur[orig_out[u]];
}

__global__ void iota_kernel(int n, int32_t *__restrict__ a, uint8_t *__restrict__ fm,
                            int8_t *__restrict__ fv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        a[i] = i;
        fm[i] = 0;
        fv[i] = 0;
    }
}

}  // namespace

hipError_t launch_compose(int n_cur, const uint8_t *fm_round, const int8_t *fv_round,
                          const int32_t *orig_cur, uint8_t *fixed_mask, int8_t *fixed_val,
                          const int64_t *info, const int32_t *orig_out, int32_t *orig_new,
                          hipStream_t s) {
    if (n_cur <= 0) return hipSuccess;
    hipLaunchKernelGGL(compose_kernel, dim3((n_cur + 255) / 256), dim3(256), 0, s, n_cur, fm_round,
                       fv_round, orig_cur, fixed_mask, fixed_val,
                       reinterpret_cast<const long long *>(info), orig_out, orig_new);
    return hipGetLastError();
}

// Sample assembly of a tempering run: the filled entries of every top-10 list,
// concatenated in list order (one workgroup per list; off = exclusive prefix of
// the counts).
__global__ __launch_bounds__(256) void top_gather_kernel(const int8_t *__restrict__ ts,
                                                         const long long *__restrict__ te,
                                                         const int32_t *__restrict__ cnt,
                                                         const int32_t *__restrict__ off, int n,
                                                         int8_t *__restrict__ S, long long *__restrict__ E) {
    const int l = blockIdx.x;
    const int c = cnt[l];
    const size_t src = (size_t)l * 10, dst = (size_t)off[l];
    for (int k = threadIdx.x; k < c; k += blockDim.x) E[dst + k] = te[src + k];
    const size_t bytes = (size_t)c * n;
    for (size_t b = threadIdx.x; b < bytes; b += blockDim.x) S[dst * n + b] = ts[src * n + b];
}

hipError_t launch_top_gather(const int8_t *ts, const int64_t *te, const int32_t *cnt, const int32_t *off,
                             int lists, int n, int8_t *S, int64_t *E, hipStream_t s) {
    if (lists <= 0) return hipSuccess;
    hipLaunchKernelGGL(top_gather_kernel, dim3(lists), dim3(256), 0, s, ts, (const long long *)te, cnt,
                       off, n, S, (long long *)E);
    return hipGetLastError();
}

hipError_t launch_iota(int n, int32_t *a, uint8_t *fm, int8_t *fv, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(iota_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, a, fm, fv);
    return hipGetLastError();
}

size_t fix_scratch_bytes(int n, int R, int m) {
    const int W = (m + 63) / 64;
    const int TS = table_size(n);
    return 64 + align8((size_t)R * 4) + (size_t)n * W * 8 + (size_t)n * 8 + (size_t)TS * 16 +
           2 * align8((size_t)n * 4) + 64;
}

hipError_t launch_persist_fix(const FixLaunch &L, hipStream_t s) {
    const spv_problem *P = L.P;
    const int n = P->n;
    FixScratch f = carve(L.scratch, n, L.R, L.m);
    hipLaunchKernelGGL(elite_kernel, dim3(1), dim3(1024), 0, s,
                       reinterpret_cast<const long long *>(L.energies), L.R, L.m, f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int cols = 64;  // a multiple of 4 (the kernel's 4-column reads)
    if (n > 0) {
        hipLaunchKernelGGL(bitmap_kernel, dim3(f.W, (n + cols - 1) / cols), dim3(64), 0, s,
                           L.samples, n, L.m, f, cols);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (L.gauge_mode != 0) {
        // table words: keys (TS u64) followed by counts and mins (TS int32 each)
        const size_t words = (size_t)f.TS + (size_t)f.TS / 2;
        const size_t total = words > (size_t)f.TS ? words : (size_t)f.TS;
        hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                           f.tkey, words, f.tmin, f.TS);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (n > 0) {
            hipLaunchKernelGGL(gauge_hash_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, L.m, f);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        hipLaunchKernelGGL(gauge_pivot_kernel, dim3(1), dim3(1024), 0, s, P->h, n, L.m,
                           L.gauge_mode, f);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    ReduceArgs a;
    a.row_ptr = P->row_ptr;
    a.col = P->col;
    a.J = P->J;
    a.h = P->h;
    a.colour = P->colour;
    a.n = n;
    a.nnz = P->nnz;
    a.m = L.m;
    a.kmin = L.kmin;
    a.use_pivot = L.gauge_mode != 0;
    a.fixed_mask = L.out->fixed_mask;
    a.fixed_val = L.out->fixed_val;
    a.row_ptr_o = L.out->row_ptr;
    a.col_o = L.out->col;
    a.J_o = L.out->J;
    a.h_o = L.out->h;
    a.colour_o = L.out->colour;
    a.orig_o = L.out->orig_index;
    a.info = reinterpret_cast<long long *>(L.out->info);
    hipLaunchKernelGGL(fix_reduce_kernel, dim3(1), dim3(1024), 0, s, a, f);
    return hipGetLastError();
}

}  // namespace spv
