// Device probes behind the roofline figures.
//
// LDS read-bandwidth probe: the measured denominator of the LDS roofline of the
// LDS-resident sweeps.  Two 1024-thread workgroups per CU read a 64 KiB LDS array
// 16 bytes per lane per instruction; consecutive lanes read consecutive 16-byte
// words, so every read is free of bank conflicts, and four reads per iteration use
// immediate offsets (no address arithmetic).  One three-input xor per 16 bytes
// keeps the data live; a compiler-only memory barrier per iteration keeps the
// reads in the loop.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "internal.hpp"

namespace spv {

namespace {

constexpr int kProbeWords = 4096;  // uint4 words: 64 KiB

__global__ __launch_bounds__(1024) void lds_probe_kernel(int iters, uint32_t *out) {
    __shared__ uint4 buf[kProbeWords];
    const int tid = threadIdx.x;
    for (int i = tid; i < kProbeWords; i += blockDim.x) buf[i] = make_uint4(i, 3u * i, 5u * i, 7u * i);
    __syncthreads();
    uint32_t a = 0, b = 0;
    const int base = tid & (kProbeWords / 4 - 1);  // 1024 lanes cover a quarter
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint4 v = buf[base + u * (kProbeWords / 4)];
            a = __builtin_amdgcn_bitop3_b32(a, v.x, v.y, 0x96);
            b = __builtin_amdgcn_bitop3_b32(b, v.z, v.w, 0x96);
        }
        __asm__ __volatile__("" ::: "memory");
    }
    if ((a ^ b) == 0x9E3779B9u) out[blockIdx.x] = a;  // practically never: keeps the reads
}

// Philox throughput probe: every lane chains Philox4x32-10 blocks (each block's
// output is the next counter) at 16 waves per CU, so the VALU pipes stay full; the
// issue slots per block follow from blocks per second and the chip's lane-slot rate.
__global__ __launch_bounds__(256) void philox_probe_kernel(int iters, uint32_t k0, uint32_t k1, uint32_t *out) {
    uint32_t c0 = blockIdx.x * blockDim.x + threadIdx.x, c1 = 7u, c2 = 11u, c3 = 13u;
    for (int it = 0; it < iters; ++it) {
        const dev::Words4 w = dev::philox(c0, c1, c2, c3, k0, k1);
        c0 = w.w[0];
        c1 = w.w[1];
        c2 = w.w[2];
        c3 = w.w[3];
    }
    if ((c0 ^ c1 ^ c2 ^ c3) == 0x9E3779B9u) out[blockIdx.x] = c0;  // practically never: keeps the chain
}

}  // namespace

hipError_t run_philox_probe(int iters, int num_cus, uint32_t *out, double *blocks_per_s, hipStream_t s) {
    const int blocks = 16 * num_cus, threads = 256;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    hipLaunchKernelGGL(philox_probe_kernel, dim3(blocks), dim3(threads), 0, s, iters, 1u, 2u, out);  // warm-up
    e = hipEventRecord(e0, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(philox_probe_kernel, dim3(blocks), dim3(threads), 0, s, iters, 1u, 2u, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    *blocks_per_s = (double)blocks * threads * (double)iters / ((double)ms * 1e-3);
    return hipSuccess;
}

hipError_t run_lds_probe(int iters, int num_cus, uint32_t *out, double *bytes_per_s, hipStream_t s) {
    const int blocks = 2 * num_cus, threads = 1024;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    hipLaunchKernelGGL(lds_probe_kernel, dim3(blocks), dim3(threads), 0, s, iters, out);  // warm-up
    e = hipEventRecord(e0, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(lds_probe_kernel, dim3(blocks), dim3(threads), 0, s, iters, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    *bytes_per_s = (double)blocks * threads * (double)iters * 4.0 * 16.0 / ((double)ms * 1e-3);
    return hipSuccess;
}

}  // namespace spv
