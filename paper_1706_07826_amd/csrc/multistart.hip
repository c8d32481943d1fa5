// Device helpers of the multi-start driver (Algorithm 2): recorded solving
// energies in full-problem units, the first minimum of the recorded energies,
// and the completion of the best state with its start's fixed values.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "internal.hpp"

namespace spv {

namespace {

// solving_E[s][r] = E'_s[r] + offset_s (E' = 0 when start s fixed everything).
__global__ void ms_offset_kernel(const long long *__restrict__ Ered, const long long *__restrict__ info,
                                 int info_stride, int S, int Rs, long long *__restrict__ solving_E) {
    const size_t total = (size_t)S * Rs;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < total; x += (size_t)gridDim.x * blockDim.x) {
        const int s = (int)(x / Rs);
        const long long *in = info + (size_t)s * info_stride;
        solving_E[x] = (in[0] > 0 ? Ered[x] : 0ll) + in[2];
    }
}

// First minimum of the recorded energies in the order: start 0's fixing rows,
// start 0's solving rows, start 1's fixing rows, ...  out[0] = energy,
// out[1] = position in that order.
__global__ __launch_bounds__(1024) void ms_argmin_kernel(const long long *__restrict__ fixE,
                                                         const long long *__restrict__ solE, int S, int F, int Rs,
                                                         long long *__restrict__ out) {
    __shared__ long long be[16], bi[16];
    const int tid = threadIdx.x, lane = dev::lane_id(), wid = tid >> 6, per = F + Rs;
    long long e = 0x7FFFFFFFFFFFFFFFll, idx = 0x7FFFFFFFFFFFFFFFll;
    const long long total = (long long)S * per;
    for (long long x = tid; x < total; x += blockDim.x) {
        const int s = (int)(x / per), k = (int)(x - (long long)s * per);
        const long long v = k < F ? fixE[(size_t)s * F + k] : solE[(size_t)s * Rs + (k - F)];
        if (v < e || (v == e && x < idx)) {
            e = v;
            idx = x;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const long long oe = __shfl_xor(e, d, 64), oi = __shfl_xor(idx, d, 64);
        if (oe < e || (oe == e && oi < idx)) {
            e = oe;
            idx = oi;
        }
    }
    if (lane == 0) {
        be[wid] = e;
        bi[wid] = idx;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            if (be[w] < e || (be[w] == e && bi[w] < idx)) {
                e = be[w];
                idx = bi[w];
            }
        out[0] = e;
        out[1] = idx;
    }
}

// best[i]: the fixing row itself, or the solving row completed with the start's
// fixed values (free variable u of start s is original variable orig_s[u]).
__global__ __launch_bounds__(1024) void ms_expand_kernel(const long long *__restrict__ best, int S, int F, int Rs,
                                                         int n, const int8_t *__restrict__ fix_spins,
                                                         const int8_t *__restrict__ sol_spins, size_t sol_stride,
                                                         const uint8_t *__restrict__ fmask,
                                                         const int8_t *__restrict__ fval,
                                                         const int32_t *__restrict__ orig, size_t orig_stride,
                                                         const long long *__restrict__ info, int info_stride,
                                                         int8_t *__restrict__ out) {
    const int tid = threadIdx.x, T = blockDim.x, per = F + Rs;
    const long long x = best[1];
    const int s = (int)(x / per), k = (int)(x - (long long)s * per);
    if (k < F) {
        for (int i = tid; i < n; i += T) out[i] = fix_spins[((size_t)s * F + k) * n + i];
        return;
    }
    const int r = k - F, nf = (int)info[(size_t)s * info_stride];
    for (int i = tid; i < n; i += T) out[i] = fmask[(size_t)s * n + i] ? fval[(size_t)s * n + i] : (int8_t)0;
    __syncthreads();
    const int8_t *row = sol_spins + (size_t)s * sol_stride + (size_t)r * nf;
    const int32_t *og = orig + (size_t)s * orig_stride;
    for (int u = tid; u < nf; u += T) out[og[u]] = row[u];
}

}  // namespace

hipError_t launch_ms_offset(const int64_t *Ered, const int64_t *info, int info_stride, int S, int Rs,
                            int64_t *solving_E, hipStream_t s) {
    const size_t total = (size_t)S * Rs;
    if (!total) return hipSuccess;
    hipLaunchKernelGGL(ms_offset_kernel, dim3((unsigned)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096)),
                       dim3(256), 0, s, reinterpret_cast<const long long *>(Ered),
                       reinterpret_cast<const long long *>(info), info_stride, S, Rs,
                       reinterpret_cast<long long *>(solving_E));
    return hipGetLastError();
}

hipError_t launch_ms_best(const int64_t *fixE, const int64_t *solE, int S, int F, int Rs, int n,
                          const int8_t *fix_spins, const int8_t *sol_spins, size_t sol_stride, const uint8_t *fmask,
                          const int8_t *fval, const int32_t *orig, size_t orig_stride, const int64_t *info,
                          int info_stride, int64_t *best, int8_t *best_spins, hipStream_t s) {
    hipLaunchKernelGGL(ms_argmin_kernel, dim3(1), dim3(1024), 0, s, reinterpret_cast<const long long *>(fixE),
                       reinterpret_cast<const long long *>(solE), S, F, Rs, reinterpret_cast<long long *>(best));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !best_spins || n <= 0) return e;
    hipLaunchKernelGGL(ms_expand_kernel, dim3(1), dim3(1024), 0, s, reinterpret_cast<const long long *>(best), S, F,
                       Rs, n, fix_spins, sol_spins, sol_stride, fmask, fval, orig, orig_stride,
                       reinterpret_cast<const long long *>(info), info_stride, best_spins);
    return hipGetLastError();
}

}  // namespace spv
