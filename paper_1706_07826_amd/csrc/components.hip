// Disconnected problems (Sec. II.C, special considerations): connected
// components of the coupler graph and the sorted-merge recombination of a
// sample over them.
//
// Components: one workgroup runs a lock-free union-find over 16-bit parents
// in LDS, always keeping the smaller root, so every root is its component's
// smallest variable index; labels are the prefix count of roots, i.e. the
// components numbered in order of their smallest variable.
//
// Recombination: partial energies E_c(r) (one workgroup per row, accumulated
// per component in LDS), then per component a stable LSD radix sort of the
// rows by E_c (one workgroup per component, 4-bit digits, as many passes as
// the component's energy range needs), then the merged rows are gathered.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "internal.hpp"
#include "pt_core.hpp"

namespace spv {

namespace {

__global__ __launch_bounds__(1024) void comp_kernel(const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col,
                                                    const int32_t *__restrict__ J, int n, int nnz,
                                                    int32_t *__restrict__ comp, int32_t *__restrict__ count) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int scan_tmp[1024 / 64 + 1];
    __shared__ int base;
    uint16_t *parent = reinterpret_cast<uint16_t *>(smem);
    const int tid = threadIdx.x, T = blockDim.x;
    for (int i = tid; i < n; i += T) parent[i] = (uint16_t)i;
    if (tid == 0) base = 0;
    __syncthreads();
    for (int i = tid; i < n; i += T) {
        int rb = row_ptr[i], re = row_ptr[i + 1];
        rb = rb < 0 ? 0 : (rb > nnz ? nnz : rb);
        re = re < rb ? rb : (re > nnz ? nnz : re);
        for (int k = rb; k < re; ++k) {
            const int j = col[k];
            if (j > i && j < n && J[k] != 0) ptc::uf_union(parent, (uint32_t)i, (uint32_t)j);
        }
    }
    __syncthreads();
    // every variable's root (its component's smallest index) into comp[]
    for (int i = tid; i < n; i += T) comp[i] = (int32_t)ptc::uf_find(parent, (uint32_t)i);
    __syncthreads();
    // label of each root = number of roots before it (parents no longer needed)
    for (int i0 = 0; i0 < n; i0 += T) {
        const int i = i0 + tid;
        const int is_root = (i < n && comp[i] == i) ? 1 : 0;
        int tot;
        const int ex = dev::block_exclusive_scan(is_root, scan_tmp, &tot);
        if (is_root) parent[i] = (uint16_t)(base + ex);
        __syncthreads();
        if (tid == 0) base += tot;
        __syncthreads();
    }
    for (int i = tid; i < n; i += T) comp[i] = parent[comp[i]];
    if (tid == 0) *count = base;
}

// Partial energies, component-major: pe[c * R + r] = E_c(r).
constexpr int kPeLdsComps = 8192;

__global__ __launch_bounds__(256) void partial_energy_kernel(const int32_t *__restrict__ row_ptr,
                                                             const int32_t *__restrict__ col,
                                                             const int32_t *__restrict__ J,
                                                             const int32_t *__restrict__ h, int n,
                                                             const int32_t *__restrict__ comp, int C,
                                                             const int8_t *__restrict__ S, int R,
                                                             long long *__restrict__ pe) {
    extern __shared__ __align__(16) unsigned char smem[];
    long long *acc = reinterpret_cast<long long *>(smem);  // [C] when C <= kPeLdsComps
    const int r = blockIdx.x, tid = threadIdx.x, T = blockDim.x;
    const bool lds = C <= kPeLdsComps;
    if (lds)
        for (int c = tid; c < C; c += T) acc[c] = 0;
    __syncthreads();
    const int8_t *s = S + (size_t)r * n;
    for (int i = tid; i < n; i += T) {
        const long long si = s[i];
        long long e = (long long)h[i] * si;
        for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const int j = col[k];
            if (j > i) e += (long long)J[k] * si * s[j];
        }
        if (e == 0) continue;
        if (lds)
            atomicAdd(reinterpret_cast<unsigned long long *>(&acc[comp[i]]), (unsigned long long)e);
        else
            atomicAdd(reinterpret_cast<unsigned long long *>(&pe[(size_t)comp[i] * R + r]), (unsigned long long)e);
    }
    __syncthreads();
    if (lds)
        for (int c = tid; c < C; c += T) pe[(size_t)c * R + r] = acc[c];
}

__global__ void fill_i64_kernel(long long *p, size_t count) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Stable sort of one component's rows by partial energy (one workgroup per
// component): keys k = E - min as unsigned, 4-bit LSD passes; thread t owns a
// contiguous chunk of the current order, so scattering each digit's rows in
// (digit, thread, position) order keeps equal keys in row order.
constexpr int kSortThreads = 1024;

__global__ __launch_bounds__(kSortThreads) void component_sort_kernel(long long *__restrict__ keyA,
                                                                      long long *__restrict__ keyB,
                                                                      int32_t *__restrict__ idxA,
                                                                      int32_t *__restrict__ idxB, int R,
                                                                      int32_t *__restrict__ inv,
                                                                      long long *__restrict__ part_E) {
    extern __shared__ __align__(16) unsigned char smem[];
    int *cnt = reinterpret_cast<int *>(smem);  // [16][T]
    __shared__ int scan_tmp[kSortThreads / 64 + 1];
    __shared__ long long red_min[kSortThreads / 64], red_max[kSortThreads / 64];
    const int c = blockIdx.x, tid = threadIdx.x, T = blockDim.x, lane = dev::lane_id(), wid = tid >> 6;
    long long *ka = keyA + (size_t)c * R, *kb = keyB + (size_t)c * R;
    int32_t *ia = idxA + (size_t)c * R, *ib = idxB + (size_t)c * R;
    // range of the keys
    long long mn = 0x7FFFFFFFFFFFFFFFll, mx = -0x7FFFFFFFFFFFFFFFll - 1;
    for (int r = tid; r < R; r += T) {
        const long long e = ka[r];
        mn = e < mn ? e : mn;
        mx = e > mx ? e : mx;
        ia[r] = r;
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const long long a = __shfl_xor(mn, d, 64), b = __shfl_xor(mx, d, 64);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    if (lane == 0) {
        red_min[wid] = mn;
        red_max[wid] = mx;
    }
    __syncthreads();
    mn = red_min[0];
    mx = red_max[0];
    for (int w = 1; w < T / 64; ++w) {
        mn = red_min[w] < mn ? red_min[w] : mn;
        mx = red_max[w] > mx ? red_max[w] : mx;
    }
    const unsigned long long range = R > 0 ? (unsigned long long)(mx - mn) : 0ull;
    const int bits = range ? 64 - __clzll((long long)range) : 0;
    for (int r = tid; r < R; r += T) ka[r] = (long long)((unsigned long long)(ka[r] - mn));
    __syncthreads();
    const int chunk = (R + T - 1) / T;
    const int r0 = min(R, tid * chunk), r1 = min(R, r0 + chunk);
    for (int shift = 0; shift < bits; shift += 4) {
        int h[16];
#pragma unroll
        for (int d = 0; d < 16; ++d) h[d] = 0;
        for (int r = r0; r < r1; ++r) ++h[((unsigned long long)ka[r] >> shift) & 15u];
#pragma unroll
        for (int d = 0; d < 16; ++d) cnt[d * T + tid] = h[d];
        __syncthreads();
        // exclusive scan of cnt in (digit, thread) order: 16 consecutive entries per thread
        int loc[16], sum = 0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            loc[u] = sum;
            sum += cnt[tid * 16 + u];
        }
        int tot;
        const int ex = dev::block_exclusive_scan(sum, scan_tmp, &tot);
#pragma unroll
        for (int u = 0; u < 16; ++u) cnt[tid * 16 + u] = ex + loc[u];
        __syncthreads();
#pragma unroll
        for (int d = 0; d < 16; ++d) h[d] = cnt[d * T + tid];
        for (int r = r0; r < r1; ++r) {
            const long long k = ka[r];
            const int d = (int)(((unsigned long long)k >> shift) & 15u);
            const int at = h[d]++;
            kb[at] = k;
            ib[at] = ia[r];
        }
        __syncthreads();
        long long *tk = ka;
        ka = kb;
        kb = tk;
        int32_t *ti = ia;
        ia = ib;
        ib = ti;
    }
    for (int k = tid; k < R; k += T) {
        inv[(size_t)c * R + k] = ia[k];
        if (part_E) part_E[(size_t)c * R + k] = ka[k] + mn;
    }
}

__global__ void merge_rows_kernel(const int8_t *__restrict__ S, int n, int R, const int32_t *__restrict__ comp,
                                  const int32_t *__restrict__ inv, int8_t *__restrict__ merged) {
    const size_t total = (size_t)R * n;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < total; x += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(x / n), i = (int)(x - (size_t)k * n);
        const int r = inv[(size_t)comp[i] * R + k];
        merged[x] = S[(size_t)r * n + i];
    }
}

__global__ void merge_energy_kernel(const long long *__restrict__ sorted_E, int C, int R,
                                    long long *__restrict__ merged_E) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= R) return;
    long long e = 0;
    for (int c = 0; c < C; ++c) e += sorted_E[(size_t)c * R + k];
    merged_E[k] = e;
}

}  // namespace

size_t components_lds_bytes(int n) { return ((size_t)((n + 1) & ~1)) * 2 + 16; }

hipError_t launch_components(const spv_problem *P, int32_t *comp, int32_t *count, hipStream_t s) {
    hipLaunchKernelGGL(comp_kernel, dim3(1), dim3(1024), components_lds_bytes(P->n), s, P->row_ptr, P->col, P->J,
                       P->n, P->nnz, comp, count);
    return hipGetLastError();
}

// Scratch of one recombination: keys and row indices (two of each for the
// radix passes), the inverse orders and, when the caller does not want the
// sorted partial energies, a buffer for them.
size_t merge_scratch_bytes(int C, int R) {
    const size_t cr = (size_t)C * R;
    return cr * (8 + 8) + ((cr * 12 + 7) & ~(size_t)7) + cr * 8 + 256;
}

hipError_t launch_merge(const spv_problem *P, const int32_t *comp, int C, const int8_t *S, int R, int8_t *merged,
                        int64_t *merged_E, int64_t *part_E, void *scratch, hipStream_t s) {
    if (R <= 0 || C <= 0) return hipSuccess;
    const size_t cr = (size_t)C * R;
    long long *keyA = static_cast<long long *>(scratch);
    long long *keyB = keyA + cr;
    int32_t *idxA = reinterpret_cast<int32_t *>(keyB + cr);
    int32_t *idxB = idxA + cr;
    int32_t *inv = idxB + cr;
    long long *own_sorted = reinterpret_cast<long long *>(reinterpret_cast<unsigned char *>(scratch) + cr * 16 +
                                                          ((cr * 12 + 7) & ~(size_t)7));
    long long *sortedE = part_E ? reinterpret_cast<long long *>(part_E) : own_sorted;
    const bool lds = C <= kPeLdsComps;
    if (!lds)
        hipLaunchKernelGGL(fill_i64_kernel, dim3((unsigned)std::min<size_t>((cr + 255) / 256, 4096)), dim3(256), 0, s,
                           keyA, cr);
    hipLaunchKernelGGL(partial_energy_kernel, dim3(R), dim3(256), lds ? (size_t)C * 8 : 0, s, P->row_ptr, P->col,
                       P->J, P->h, P->n, comp, C, S, R, keyA);
    hipLaunchKernelGGL(component_sort_kernel, dim3(C), dim3(kSortThreads), (size_t)16 * kSortThreads * 4, s, keyA,
                       keyB, idxA, idxB, R, inv, sortedE);
    const size_t total = (size_t)R * P->n;
    if (total)
        hipLaunchKernelGGL(merge_rows_kernel, dim3((unsigned)std::min<size_t>((total + 255) / 256, 16384)), dim3(256),
                           0, s, S, P->n, R, comp, inv, merged);
    hipLaunchKernelGGL(merge_energy_kernel, dim3((R + 255) / 256), dim3(256), 0, s, sortedE, C, R,
                       reinterpret_cast<long long *>(merged_E));
    return hipGetLastError();
}

}  // namespace spv
