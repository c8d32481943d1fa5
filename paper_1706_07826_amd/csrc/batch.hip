// Batched simulated annealing over many instances of uneven size (residual
// problems left after fixing, Sec. II.C / Sec. III.C) in one persistent launch.
//
// Every instance is packed into its own image by two batched prep kernels.
// The persistent kernel then pops work items -- (instance, block of quads) in
// largest-instance-first order -- from a device counter; a workgroup reloads
// the instance image into LDS only when the instance changes, and runs the
// same schedule body as the one-instance launch, so results are bit-identical
// to one launch per instance whatever the shape.  Every workgroup exits when
// the counter passes the item count.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.hpp"
#include "internal.hpp"
#include "sa_core.hpp"
#include "swar_core.hpp"

namespace spv {

namespace {

__global__ __launch_bounds__(1024) void batch_prep_order_kernel(const BatchInst *__restrict__ insts,
                                                                int32_t *__restrict__ images) {
    __shared__ int cnt[kMaxColours];
    __shared__ int cs[kMaxColours + 1];
    __shared__ int tmp[1024 / 64 + 1];
    const BatchInst in = insts[blockIdx.x];
    const int n = in.n, C = in.C, tid = threadIdx.x;
    int32_t *image = images + in.image_off;
    int32_t *order = image + kImgHeader;
    int32_t *pos_of = order + n;
    if (tid < kMaxColours) cnt[tid] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
        int c = in.colour[i];
        atomicAdd(&cnt[c < C ? c : C - 1], 1);
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
        image[1] = in.D;
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
                ci = in.colour[i];
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

__global__ __launch_bounds__(256) void batch_prep_nbr_kernel(const BatchInst *__restrict__ insts,
                                                             int32_t *__restrict__ images) {
    const BatchInst in = insts[blockIdx.y];
    const int n = in.n, D = in.D, nnz = in.nnz;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int32_t *image = images + in.image_off;
    const int32_t *order = image + kImgHeader;
    const int32_t *pos_of = order + n;
    int32_t *hpos = image + kImgHeader + 2 * n;
    uint32_t *nbr = reinterpret_cast<uint32_t *>(image + kImgHeader + 3 * n);
    int i = order[p];
    i = i < 0 ? 0 : (i >= n ? n - 1 : i);
    int rb = in.row_ptr[i], re = in.row_ptr[i + 1];
    rb = rb < 0 ? 0 : (rb > nnz ? nnz : rb);
    re = re < rb ? rb : (re > nnz ? nnz : re);
    const int deg = (re - rb) < D ? (re - rb) : D;
    for (int k = 0; k < D; ++k) {
        uint32_t rec = (uint32_t)p << 16;
        if (k < deg) {
            int j = in.col[rb + k];
            j = j < 0 ? 0 : (j >= n ? n - 1 : j);
            int v = in.J[rb + k];
            v = v > 32767 ? 32767 : (v < -32767 ? -32767 : v);
            rec = ((uint32_t)pos_of[j] << 16) | (uint32_t)(uint16_t)(int16_t)v;
        }
        nbr[(size_t)p * D + k] = rec;
    }
    hpos[p] = in.h[i];
}

__global__ void batch_reset_kernel(int *counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

struct BatchArgs {
    const BatchInst *insts;
    const int32_t *items;  // [n_items][2]: instance, first quad
    int n_items;
    int *counter;
    const int32_t *images;
    const uint32_t *tables;
    int row_len, sweeps, qw, n_max, D_max;
    uint32_t sweep_offset;
    int pairs_qw;  // paired body: the spin area holds 2 n_max pairs_qw words (every item's 4 n copies)
    int kmax;      // paired body: most copies an item has
};

// ND = 0: byte-parallel body; DK > 0: every image has exactly DK records per site.
template <int ND, int DK = 0>
__global__ __launch_bounds__(1024) void batch_sa_kernel(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cs[kMaxColours + 1];
    __shared__ int item_s;
    // ND = 0: byte-parallel path (x_bound <= 255 for every instance of the batch).
    using Lds = typename std::conditional<ND == 0, core::SwarLds, core::SaLds>::type;
    Lds L;
    const int e2q = a.qw > kBatchMaxItemQuads ? a.qw : kBatchMaxItemQuads;
    if constexpr (ND == 0)
        core::swar_layout(a.n_max, a.D_max, a.row_len, a.qw, &L, smem, e2q);
    else
        core::sa_layout(a.n_max, a.D_max, a.row_len, a.qw, &L, smem, e2q);
    int loaded = -1;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(a.counter, 1);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= a.n_items) break;
        const int b = a.items[3 * item];
        const BatchInst in = a.insts[b];
        core::SaItem it;
        it.image = a.images + in.image_off;
        it.tables = a.tables;
        it.init = nullptr;
        it.out = in.out;
        it.energies = in.energies;
        it.n = in.n;
        it.D = in.D;
        it.C = in.C;
        it.row_len = a.row_len;
        it.sweeps = a.sweeps;
        it.reads = in.reads;
        it.q0 = a.items[3 * item + 1];
        it.qw = a.items[3 * item + 2];
        it.sweep_offset = a.sweep_offset;
        it.k0 = (uint32_t)in.seed;
        it.k1 = (uint32_t)(in.seed >> 32);
        if constexpr (ND == 0) {
            if (b != loaded) {
                core::swar_load_instance(L, it, cs);
                loaded = b;
            }
            core::swar_run<DK, 1>(L, it, cs);
        } else {
            if (b != loaded) {
                core::sa_load_instance(L, it, cs);
                loaded = b;
            }
            core::sa_run<ND>(L, it, cs);
        }
    }
}

// Paired body: an item is (instance, first quad, copies); see swar_run_pairs.
template <int DK>
__global__ __launch_bounds__(1024) void batch_sa_paired_kernel(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cs[kMaxColours + 1];
    __shared__ int item_s;
    core::SwarLds L;
    core::swar_layout(a.n_max, DK, a.row_len, a.pairs_qw, &L, smem, 2 * a.kmax);
    int loaded = -1;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(a.counter, 1);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= a.n_items) break;
        const int b = a.items[3 * item];
        const BatchInst in = a.insts[b];
        core::SaItem it;
        it.image = a.images + in.image_off;
        it.tables = a.tables;
        it.init = nullptr;
        it.out = in.out;
        it.energies = in.energies;
        it.n = in.n;
        it.D = in.D;
        it.C = in.C;
        it.row_len = a.row_len;
        it.sweeps = a.sweeps;
        it.reads = in.reads;
        it.q0 = a.items[3 * item + 1];
        it.qw = 2;  // records address region 0: S [n][2], then ~S [n][2]
        it.sweep_offset = a.sweep_offset;
        it.k0 = (uint32_t)in.seed;
        it.k1 = (uint32_t)(in.seed >> 32);
        if (b != loaded) {
            core::swar_load_instance(L, it, cs);
            loaded = b;
        }
        core::swar_run_pairs<DK>(L, it, cs, a.items[3 * item + 2]);
    }
}

}  // namespace

hipError_t launch_batch_prep(const BatchInst *insts, int B, int n_max, int32_t *images, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_prep_order_kernel, dim3(B), dim3(1024), 0, s, insts, images);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_max <= 0) return e;
    hipLaunchKernelGGL(batch_prep_nbr_kernel, dim3((n_max + 255) / 256, B), dim3(256), 0, s, insts, images);
    return hipGetLastError();
}

size_t batch_paired_lds_bytes(int n_max, int D_max, int row_len, int pairs_qw, int kmax) {
    return core::swar_layout(n_max, D_max, row_len, pairs_qw, nullptr, nullptr, 2 * kmax);
}

size_t batch_lds_bytes(int n_max, int D_max, int row_len, int qw, int nd) {
    const int e2q = qw > kBatchMaxItemQuads ? qw : kBatchMaxItemQuads;
    if (sa_use_swar(nd, row_len)) return core::swar_layout(n_max, D_max, row_len, qw, nullptr, nullptr, e2q);
    return core::sa_layout(n_max, D_max, row_len, qw, nullptr, nullptr, e2q);
}

hipError_t launch_batch_sa(const BatchLaunch &L, hipStream_t s) {
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, L.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    BatchArgs a;
    a.insts = L.insts;
    a.items = L.items;
    a.n_items = L.n_items;
    a.counter = L.counter;
    a.images = L.images;
    a.tables = L.tables;
    a.row_len = L.row_len;
    a.sweeps = L.sweeps;
    a.qw = L.qw;
    a.n_max = L.n_max;
    a.D_max = L.D_max;
    a.sweep_offset = L.sweep_offset;
    a.pairs_qw = L.pairs_qw;
    a.kmax = L.kmax;
    if (L.paired) {
        const size_t plds = batch_paired_lds_bytes(L.n_max, L.dk, L.row_len, L.pairs_qw, L.kmax);
        if (L.dk == 6)
            hipLaunchKernelGGL((batch_sa_paired_kernel<6>), dim3(L.grid), dim3(L.threads), plds, s, a);
        else if (L.dk == 4)
            hipLaunchKernelGGL((batch_sa_paired_kernel<4>), dim3(L.grid), dim3(L.threads), plds, s, a);
        else if (L.dk == 8)
            hipLaunchKernelGGL((batch_sa_paired_kernel<8>), dim3(L.grid), dim3(L.threads), plds, s, a);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    const size_t lds = batch_lds_bytes(L.n_max, L.D_max, L.row_len, L.qw, L.nd);
    switch (sa_use_swar(L.nd, L.row_len) ? 0 : L.nd) {
        case 0:
            if (L.dk == 6)
                hipLaunchKernelGGL((batch_sa_kernel<0, 6>), dim3(L.grid), dim3(L.threads), lds, s, a);
            else if (L.dk == 4)
                hipLaunchKernelGGL((batch_sa_kernel<0, 4>), dim3(L.grid), dim3(L.threads), lds, s, a);
            else if (L.dk == 8)
                hipLaunchKernelGGL((batch_sa_kernel<0, 8>), dim3(L.grid), dim3(L.threads), lds, s, a);
            else
                hipLaunchKernelGGL(batch_sa_kernel<0>, dim3(L.grid), dim3(L.threads), lds, s, a);
            break;
        case 1:
            hipLaunchKernelGGL(batch_sa_kernel<1>, dim3(L.grid), dim3(L.threads), lds, s, a);
            break;
        case 2:
            hipLaunchKernelGGL(batch_sa_kernel<2>, dim3(L.grid), dim3(L.threads), lds, s, a);
            break;
        case 3:
            hipLaunchKernelGGL(batch_sa_kernel<3>, dim3(L.grid), dim3(L.threads), lds, s, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t shadow_stats_batch(unsigned long long *out, bool reset) { return shadow::read_stats(out, reset); }

}  // namespace spv
