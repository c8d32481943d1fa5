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
template <int ND, int DK = 0>
__global__ __launch_bounds__(1024) void sa_kernel(core::SaItem a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cs[kMaxColours + 1];
    a.q0 = blockIdx.x * a.qw;
    if constexpr (ND == 0) {
        core::SwarLds L;
        core::swar_layout(a.n, a.D, a.row_len, a.qw, &L, smem);
        core::swar_load_instance(L, a, cs);
        core::swar_run<DK>(L, a, cs);
    } else {
        core::SaLds L;
        core::sa_layout(a.n, a.D, a.row_len, a.qw, &L, smem);
        core::sa_load_instance(L, a, cs);
        core::sa_run<ND>(L, a, cs);
    }
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

hipError_t launch_prep(const spv_problem *P, int32_t *image, hipStream_t s) {
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

size_t sa_lds_bytes(int n, int D, int row_len, int qw) {
    if (sa_use_swar(1 + (row_len > kDigitSize ? 1 : 0), row_len))
        return core::swar_layout(n, D, row_len, qw, nullptr, nullptr);
    return core::sa_layout(n, D, row_len, qw, nullptr, nullptr);
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
    a.k0 = (uint32_t)L.seed;
    a.k1 = (uint32_t)(L.seed >> 32);
    const size_t lds = sa_lds_bytes(L.n, L.D, L.row_len, L.qw);
    if (lds > lds_limit) return hipErrorInvalidValue;
    const int quads = (L.reads + 3) / 4;
    const int grid = (quads + L.qw - 1) / L.qw;
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

hipError_t launch_energy(const int32_t *image, int n, int D, const int8_t *spins, int R,
                         int64_t *E, hipStream_t s) {
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL(energy_kernel, dim3(R), dim3(256), 0, s, image, n, D, spins, R,
                       reinterpret_cast<long long *>(E));
    return hipGetLastError();
}

}  // namespace spv
