// Colour classes for the parallel sweep (the sweep updates one independent set at
// a time): Jones-Plassmann rounds in one workgroup.  Vertex v has priority
// (word 0 of Philox(v, 0, 0, 5 << 24) under the seed, then v), higher first; in
// each round every uncoloured vertex whose priority exceeds that of all its
// uncoloured neighbours (every CSR entry counts as an edge) takes the smallest
// colour none of its coloured neighbours has.  Decisions of a round read only the
// colours at its start, so the result is unique: it equals first-fit greedy
// colouring in decreasing priority order.  The colours live in LDS (one byte per
// vertex, plus a byte for the round's decisions).
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "internal.hpp"

namespace spv {

namespace {

constexpr uint8_t kUncoloured = 0xFF;

__device__ __forceinline__ bool prio_gt(uint32_t pa, int a, uint32_t pb, int b) {
    return pa > pb || (pa == pb && a > b);
}

__global__ void colour_prio_kernel(int n, uint32_t k0, uint32_t k1, uint32_t *__restrict__ prio) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) prio[i] = dev::philox((uint32_t)i, 0u, 0u, 5u << 24, k0, k1).w[0];
}

// info[0]: colours used (max + 1); info[1]: rounds; info[2]: 1 when a colour reached
// kMaxColours.
__global__ __launch_bounds__(1024) void colour_jp_kernel(const int32_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ col, int n,
                                                         const uint32_t *__restrict__ prio,
                                                         uint8_t *__restrict__ colour_out, int *__restrict__ info) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint8_t *cl = smem;       // [n] colours (kUncoloured while open)
    uint8_t *nx = smem + n;   // [n] this round's decisions
    __shared__ int left_s, used_s;
    const int tid = threadIdx.x, T = blockDim.x;
    for (int i = tid; i < n; i += T) cl[i] = kUncoloured;
    if (tid == 0) {
        left_s = n;
        used_s = 0;
    }
    __syncthreads();
    int rounds = 0;
    while (__builtin_amdgcn_readfirstlane(left_s) > 0) {
        for (int i = tid; i < n; i += T) {
            uint8_t d = kUncoloured;
            if (cl[i] == kUncoloured) {
                const uint32_t pi = prio[i];
                bool top = true;
                unsigned long long seen = 0ull;  // colours 0..63 of coloured neighbours
                for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                    const int j = col[k];
                    const uint8_t cj = cl[j];
                    if (cj == kUncoloured) {
                        if (prio_gt(prio[j], j, pi, i)) {
                            top = false;
                            break;
                        }
                    } else if (cj < 64) {
                        seen |= 1ull << cj;
                    }
                }
                if (top) {
                    const int c = ~seen ? __builtin_ctzll(~seen) : 64;
                    d = (uint8_t)(c < kMaxColours ? c : kMaxColours);
                }
            }
            nx[i] = d;
        }
        __syncthreads();
        int done = 0, used = 0;
        for (int i = tid; i < n; i += T)
            if (nx[i] != kUncoloured) {
                cl[i] = nx[i];
                ++done;
                used = max(used, (int)nx[i] + 1);
            }
        if (done) atomicSub(&left_s, done);
        if (used) atomicMax(&used_s, used);
        ++rounds;
        __syncthreads();
    }
    for (int i = tid; i < n; i += T) colour_out[i] = cl[i];
    if (tid == 0) {
        info[0] = used_s > 0 ? used_s : 1;
        info[1] = rounds;
        info[2] = used_s > kMaxColours ? 1 : 0;
    }
}

}  // namespace

size_t colour_lds_bytes(int n) { return (size_t)2 * (size_t)(n > 0 ? n : 1) + 16; }

hipError_t launch_colour(const Inst *P, uint64_t seed, uint8_t *colour, uint32_t *prio, int *info,
                         hipStream_t s) {
    const int n = P->n;
    hipLaunchKernelGGL(colour_prio_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, (uint32_t)seed,
                       (uint32_t)(seed >> 32), prio);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colour_jp_kernel, dim3(1), dim3(1024), colour_lds_bytes(n), s, P->row_ptr, P->col, n, prio,
                       colour, info);
    return hipGetLastError();
}

}  // namespace spv
