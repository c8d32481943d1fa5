// Device helpers of the multi-start driver (Algorithm 2): recorded energies in
// full-problem units, fixes composed into original indices, the per-start and
// overall first minimum of the recorded energies, and the lift of the best row
// through a start's reductions back to the full problem.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "internal.hpp"

namespace spv {

namespace {

// rec[s][r] = (start s's problem is empty ? 0 : rec[s][r]) + off[s].
__global__ void ms_record_kernel(long long *__restrict__ rec, int S, int R, MsStageParams prm) {
    const size_t total = (size_t)S * R;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < total; x += (size_t)gridDim.x * blockDim.x) {
        const int s = (int)(x / R);
        rec[x] = (prm.ncur[s] > 0 ? rec[x] : 0ll) + prm.off[s];
    }
}

// One reduction level of every start (blockIdx.y = start): its fixed variables
// into the start's original-index mask and values, and the map of the level's
// free variables to original indices, map_next[u] = map_cur[orig[u]].
__global__ __launch_bounds__(256) void ms_compose_kernel(MsStageParams prm,
                                                         const unsigned char *__restrict__ lvl, size_t lvl_stride,
                                                         MsLevelOffsets lo, int with_fixes,
                                                         const int32_t *__restrict__ map_cur,
                                                         int32_t *__restrict__ map_next, int n,
                                                         uint8_t *__restrict__ fm, int8_t *__restrict__ fv) {
    const int s = blockIdx.y;
    const unsigned char *L = lvl + (size_t)s * lvl_stride;
    const int n_prev = prm.n_prev[s], n_next = prm.n_next[s];
    const int32_t *mc = map_cur + (size_t)s * n;
    int32_t *mn = map_next + (size_t)s * n;
    const int32_t *orig = reinterpret_cast<const int32_t *>(L + lo.orig);
    const int stride = (int)(gridDim.x * blockDim.x);
    const int t0 = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (with_fixes) {
        const uint8_t *mask = L + lo.mask;
        const int8_t *val = reinterpret_cast<const int8_t *>(L + lo.val);
        for (int i = t0; i < n_prev; i += stride)
            if (mask[i]) {
                fm[(size_t)s * n + mc[i]] = 1;
                fv[(size_t)s * n + mc[i]] = val[i];
            }
    }
    for (int u = t0; u < n_next; u += stride) mn[u] = mc[orig[u]];
}

// Start maps before the loop: identity, or the pre-processing's free variables.
__global__ void ms_map_init_kernel(int32_t *__restrict__ map, int S, int n, int n_base,
                                   const int32_t *__restrict__ pre_orig, uint8_t *__restrict__ fm,
                                   int8_t *__restrict__ fv) {
    const size_t total = (size_t)S * n;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < total; x += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(x % n);
        if (i < n_base) map[x] = pre_orig ? pre_orig[i] : i;
        fm[x] = 0;
        fv[x] = 0;
    }
}

// Per start: the lowest recorded energy and its first position in the start's
// stage order (stage j's rows follow stage j-1's).
__global__ __launch_bounds__(256) void ms_start_best_kernel(MsRecords rc, int S, long long *__restrict__ sb_E,
                                                            long long *__restrict__ sb_pos) {
    __shared__ long long be[4], bi[4];
    const int s = blockIdx.x, tid = threadIdx.x, lane = dev::lane_id(), wid = tid >> 6;
    long long e = 0x7FFFFFFFFFFFFFFFll, idx = 0x7FFFFFFFFFFFFFFFll, base = 0;
    for (int j = 0; j < rc.nst; ++j) {
        const long long *E = rc.E[j] + (size_t)s * rc.R[j];
        for (int r = tid; r < rc.R[j]; r += blockDim.x) {
            const long long v = E[r], x = base + r;
            if (v < e || (v == e && x < idx)) {
                e = v;
                idx = x;
            }
        }
        base += rc.R[j];
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
        sb_E[s] = e;
        sb_pos[s] = idx;
    }
}

// The overall first minimum over starts in start order: out[0] = energy,
// out[1] = start, out[2] = position inside the start.
__global__ void ms_best_kernel(const long long *__restrict__ sb_E, const long long *__restrict__ sb_pos, int S,
                               long long *__restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    long long e = sb_E[0];
    int bs = 0;
    for (int s = 1; s < S; ++s)
        if (sb_E[s] < e) {
            e = sb_E[s];
            bs = s;
        }
    out[0] = e;
    out[1] = bs;
    out[2] = sb_pos[bs];
}

// One persistence level in reverse: prev[i] = the fixed value of i (free
// variables are written only by the scatter, so the two never meet), then
// prev[orig[u]] = cur[u].
__global__ void ms_lift_kernel(const int8_t *__restrict__ cur, int n_next, const int32_t *__restrict__ orig,
                               const int8_t *__restrict__ val, int n_prev, int8_t *__restrict__ prev) {
    const int stride = (int)(gridDim.x * blockDim.x);
    const int t0 = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    for (int i = t0; i < n_prev; i += stride)
        if (val[i]) prev[i] = val[i];
    for (int u = t0; u < n_next; u += stride) prev[orig[u]] = cur[u];
}

}  // namespace

hipError_t launch_ms_record(int64_t *rec, int S, int R, const MsStageParams &prm, hipStream_t s) {
    const size_t total = (size_t)S * R;
    if (!total) return hipSuccess;
    const unsigned g = (unsigned)std::min<size_t>(4096, (total + 255) / 256);
    hipLaunchKernelGGL(ms_record_kernel, dim3(g), dim3(256), 0, s, reinterpret_cast<long long *>(rec), S, R, prm);
    return hipGetLastError();
}

hipError_t launch_ms_compose(const MsStageParams &prm, int S, int n, const unsigned char *lvl, size_t lvl_stride,
                             MsLevelOffsets lo, bool with_fixes, const int32_t *map_cur, int32_t *map_next,
                             uint8_t *fm, int8_t *fv, hipStream_t s) {
    if (S <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(ms_compose_kernel, dim3((unsigned)std::min(64, (n + 255) / 256), (unsigned)S), dim3(256), 0, s,
                       prm, lvl, lvl_stride, lo, with_fixes ? 1 : 0, map_cur, map_next, n, fm, fv);
    return hipGetLastError();
}

hipError_t launch_ms_map_init(int32_t *map, int S, int n, int n_base, const int32_t *pre_orig, uint8_t *fm,
                              int8_t *fv, hipStream_t s) {
    const size_t total = (size_t)S * n;
    if (!total) return hipSuccess;
    const unsigned g = (unsigned)std::min<size_t>(4096, (total + 255) / 256);
    hipLaunchKernelGGL(ms_map_init_kernel, dim3(g), dim3(256), 0, s, map, S, n, n_base, pre_orig, fm, fv);
    return hipGetLastError();
}

hipError_t launch_ms_best(const MsRecords &rc, int S, int64_t *sb_E, int64_t *sb_pos, int64_t *best, hipStream_t s) {
    hipLaunchKernelGGL(ms_start_best_kernel, dim3((unsigned)S), dim3(256), 0, s, rc, S,
                       reinterpret_cast<long long *>(sb_E), reinterpret_cast<long long *>(sb_pos));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ms_best_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<const long long *>(sb_E),
                       reinterpret_cast<const long long *>(sb_pos), S, reinterpret_cast<long long *>(best));
    return hipGetLastError();
}

hipError_t launch_ms_lift(const int8_t *cur, int n_next, const int32_t *orig, const int8_t *val, int n_prev,
                          int8_t *prev, hipStream_t s) {
    const int m = std::max(n_prev, n_next);
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(ms_lift_kernel, dim3((unsigned)std::min(64, (m + 255) / 256)), dim3(256), 0, s, cur, n_next,
                       orig, val, n_prev, prev);
    return hipGetLastError();
}

}  // namespace spv
