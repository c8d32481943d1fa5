// Instance packing and the simulated-annealing sweep kernel.
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

// Sum of the four local fields of the quad at position p: f_b = h_p + sum_k J_k s_kb.
struct Fields {
    int32_t f[4];
};

__device__ __forceinline__ Fields local_fields(const uint32_t *__restrict__ nb,
                                               const uint32_t *__restrict__ S, int D, int qw,
                                               int q, int32_t hv) {
    Fields F;
#pragma unroll
    for (int b = 0; b < 4; ++b) F.f[b] = hv;
    for (int k = 0; k < D; ++k) {
        const uint32_t rec = nb[k];
        const int32_t Jv = (int32_t)(int16_t)(rec & 0xffffu);
        const uint32_t w = S[(rec >> 16) * qw + q];
#pragma unroll
        for (int b = 0; b < 4; ++b) F.f[b] += Jv * dev::spin_of(w, b);
    }
    return F;
}

template <int ND>
__device__ __forceinline__ uint32_t metropolis_mask(const int32_t x[4], const uint32_t *tab,
                                                    uint32_t i, uint32_t t, uint32_t quad,
                                                    uint32_t k0, uint32_t k1) {
    // Returns the xor mask (0xFE per accepted byte) that flips accepted replicas.
    bool pass[4];
    bool up[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        up[b] = x[b] > 0;
        pass[b] = true;
    }
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        uint32_t d[4];
        bool need = false;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            d[b] = up[b] ? (((uint32_t)x[b] >> (kDigitBits * j)) & (kDigitSize - 1)) : 0u;
            need |= pass[b] && d[b] != 0;
        }
        if (need) {
            const dev::Words4 w = dev::philox(i, t, quad, (2u << 24) | (uint32_t)j, k0, k1);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (d[b] != 0) pass[b] = pass[b] && (w.w[b] < tab[j * kDigitSize + d[b]]);
        }
    }
    uint32_t mask = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
        if (!up[b] || pass[b]) mask |= 0xFEu << (8 * b);
    return mask;
}

struct SaArgs {
    const int32_t *image;
    const uint32_t *tables;
    const int8_t *init;
    int8_t *out;
    int64_t *energies;
    int n, D, C, row_len, sweeps, reads, qw;
    uint32_t sweep_offset, k0, k1;
};

template <int ND>
__global__ __launch_bounds__(1024) void sa_kernel(SaArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = a.n, D = a.D, qw = a.qw, T = blockDim.x, tid = threadIdx.x;
    uint32_t *nbr = reinterpret_cast<uint32_t *>(smem);
    int32_t *hpos = reinterpret_cast<int32_t *>(nbr + (size_t)n * D);
    int32_t *ord = hpos + n;
    uint32_t *tab = reinterpret_cast<uint32_t *>(ord + n);       // [2][row_len]
    uint32_t *S = tab + 2 * a.row_len;                           // [n][qw]
    size_t e2_off = (reinterpret_cast<unsigned char *>(S + (size_t)n * qw) - smem + 7) & ~(size_t)7;
    unsigned long long *E2 = reinterpret_cast<unsigned long long *>(smem + e2_off);  // [4*qw]
    __shared__ int cs[kMaxColours + 1];

    const int32_t *img = a.image;
    const int q0 = blockIdx.x * qw;  // first quad of this workgroup
    // Each thread keeps one quad q for the whole launch and walks positions
    // slot, slot + nslots, ... of every class.
    const int q = tid % qw;
    const int slot = tid / qw;
    const int nslots = T / qw;
    const bool active = slot < nslots;
    if (tid <= a.C) cs[tid] = img[3 + tid];
    for (int k = tid; k < n * D; k += T) nbr[k] = reinterpret_cast<const uint32_t *>(img + kImgHeader + 3 * n)[k];
    for (int k = tid; k < n; k += T) {
        hpos[k] = img[kImgHeader + 2 * n + k];
        ord[k] = img[kImgHeader + k];
    }
    for (int k = tid; k < a.row_len; k += T) tab[k] = a.tables[k];
    for (int k = tid; k < 4 * qw; k += T) E2[k] = 0ull;
    __syncthreads();

    // Initial state.
    if (a.init == nullptr) {
        for (int p = slot; active && p < n; p += nslots) {
            const dev::Words4 w =
                dev::philox((uint32_t)ord[p], 0u, (uint32_t)(q0 + q), 1u << 24, a.k0, a.k1);
            uint32_t word = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) word |= ((w.w[b] >> 31) ? 0x01u : 0xFFu) << (8 * b);
            S[(size_t)p * qw + q] = word;
        }
    } else {
        const int32_t *pos_of = img + kImgHeader + n;
        unsigned char *Sb = reinterpret_cast<unsigned char *>(S);
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

    for (int ls = 0; ls < a.sweeps; ++ls) {
        const uint32_t t = a.sweep_offset + (uint32_t)ls;
        const uint32_t *tcur = tab + (ls & 1) * a.row_len;
        uint32_t *tnext = tab + ((ls + 1) & 1) * a.row_len;
        if (ls + 1 < a.sweeps)
            for (int k = tid; k < a.row_len; k += T)
                tnext[k] = a.tables[(size_t)(ls + 1) * a.row_len + k];
        for (int c = 0; c < a.C; ++c) {
            const int pe = cs[c + 1];
            for (int p = cs[c] + slot; active && p < pe; p += nslots) {
                const uint32_t self = S[(size_t)p * qw + q];
                const Fields F = local_fields(nbr + (size_t)p * D, S, D, qw, q, hpos[p]);
                int32_t x[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) x[b] = dev::spin_of(self, b) > 0 ? -F.f[b] : F.f[b];
                const uint32_t mask = metropolis_mask<ND>(x, tcur, (uint32_t)ord[p], t,
                                                          (uint32_t)(q0 + q), a.k0, a.k1);
                if (mask) S[(size_t)p * qw + q] = self ^ mask;
            }
            __syncthreads();
        }
    }

    // Energies: 2E = sum_p s_p (h_p + f_p) per replica.
    {
        long long e2[4] = {0, 0, 0, 0};
        for (int p = slot; active && p < n; p += nslots) {
            const uint32_t self = S[(size_t)p * qw + q];
            const Fields F = local_fields(nbr + (size_t)p * D, S, D, qw, q, hpos[p]);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                e2[b] += (long long)dev::spin_of(self, b) * ((long long)hpos[p] + F.f[b]);
        }
        if (active)
#pragma unroll
            for (int b = 0; b < 4; ++b) atomicAdd(&E2[q * 4 + b], (unsigned long long)e2[b]);
    }
    __syncthreads();
    for (int rl = tid; rl < 4 * qw; rl += T) {
        const int r = 4 * q0 + rl;
        if (r < a.reads) a.energies[r] = ((long long)E2[rl]) / 2;
    }
    // Spins, transposed back to [read][variable] in original variable order.
    const int32_t *pos_of = img + kImgHeader + n;
    const unsigned char *Sb = reinterpret_cast<const unsigned char *>(S);
    for (int idx = tid; idx < 4 * qw * n; idx += T) {
        const int rl = idx / n, i = idx - rl * n;
        const int r = 4 * q0 + rl;
        if (r < a.reads) {
            const int p = pos_of[i];
            a.out[(size_t)r * n + i] = (int8_t)Sb[((size_t)p * qw + (rl >> 2)) * 4 + (rl & 3)];
        }
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

size_t sa_lds_bytes(int n, int D, int row_len, int qw) {
    size_t b = (size_t)n * D * 4 + (size_t)n * 8 + (size_t)2 * row_len * 4 + (size_t)n * qw * 4;
    // dynamic LDS starts 16-aligned; E2 is placed at the next 8-byte boundary
    b = (b + 7) & ~(size_t)7;
    return b + (size_t)4 * qw * 8;
}

hipError_t launch_sa(const SaLaunch &L, hipStream_t s, size_t lds_limit) {
    SaArgs a;
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
    a.qw = L.qw;
    a.sweep_offset = L.sweep_offset;
    a.k0 = (uint32_t)L.seed;
    a.k1 = (uint32_t)(L.seed >> 32);
    const size_t lds = sa_lds_bytes(L.n, L.D, L.row_len, L.qw);
    if (lds > lds_limit) return hipErrorInvalidValue;
    const int quads = (L.reads + 3) / 4;
    const int grid = (quads + L.qw - 1) / L.qw;
    switch (L.nd) {
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
