// Instance ingest (Sec. I problem statement: an Ising instance J, h): every
// sampling call validates its CSR on the device and derives the two bounds the
// host sizes tables, digits and layouts by, so no caller-supplied bound is
// trusted.  One thread per row; a problem per grid row (blockIdx.y).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.hpp"

namespace spv {

namespace {

__device__ __forceinline__ unsigned long long umin(unsigned long long a, unsigned long long b) { return a < b ? a : b; }
__device__ __forceinline__ unsigned long long umax(unsigned long long a, unsigned long long b) { return a > b ? a : b; }

// Each row is examined in the order of the checks; a row whose row_ptr entries
// are out of order or out of range is not read further, so every access stays
// inside [0, n] of row_ptr and [0, nnz) of col and J.
__global__ __launch_bounds__(256) void ingest_kernel(const IngestDesc *__restrict__ descs,
                                                     IngestResult *__restrict__ res) {
    const IngestDesc P = descs[blockIdx.y];
    __shared__ int cnt[kMaxColours];
    if (threadIdx.x < kMaxColours) cnt[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long bad = ~0ull, xmax = 0ull;
    int dmax = 0;
    const int stride = (int)(gridDim.x * blockDim.x);
    for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < P.n; i += stride) {
        const unsigned long long row = (unsigned long long)(i + 1) << 8;
        if (i == 0 && (P.row_ptr[0] != 0 || P.row_ptr[P.n] != P.nnz)) bad = umin(bad, kChkRowPtrEnds);
        const int a = P.row_ptr[i], b = P.row_ptr[i + 1];
        if (a < 0 || b < a || b > P.nnz) {
            bad = umin(bad, row | kChkRowPtrOrder);
            continue;
        }
        const int deg = b - a;
        dmax = deg > dmax ? deg : dmax;
        if (deg > kMaxDegree) bad = umin(bad, row | kChkDegree);
        int ci = 0;
        if (P.check_colours) {
            ci = P.colour[i];
            if (ci >= P.n_colours) bad = umin(bad, row | kChkColourRange);
            else atomicAdd(&cnt[ci], 1);
        }
        const int hv = P.h ? P.h[i] : 0;  // structure-only ingest reads neither h nor J
        unsigned long long x = (unsigned long long)(hv < 0 ? -(long long)hv : (long long)hv);
        int prev = -1;
        for (int k = a; k < b; ++k) {
            const int j = P.col[k];
            if (j < 0 || j >= P.n) {
                bad = umin(bad, row | kChkColRange);
                break;
            }
            if (j == i) bad = umin(bad, row | kChkSelfLoop);
            if (j <= prev) bad = umin(bad, row | kChkUnsorted);
            prev = j;
            const int Jk = P.J ? P.J[k] : 0;
            if (Jk > 32767 || Jk < -32767) bad = umin(bad, row | kChkJRange);
            x += (unsigned long long)(Jk < 0 ? -(long long)Jk : (long long)Jk);
            if (P.check_colours == 1 && P.colour[j] == ci) bad = umin(bad, row | kChkColourEdge);
            // the transposed entry, by bisection over row j (an out-of-order row j is
            // that row's own failure)
            const int ja = P.row_ptr[j], jb = P.row_ptr[j + 1];
            if (ja < 0 || jb < ja || jb > P.nnz) continue;
            int lo = ja, hi = jb;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (P.col[mid] < i) lo = mid + 1;
                else hi = mid;
            }
            if (lo == jb || P.col[lo] != i || (P.J && P.J[lo] != Jk)) bad = umin(bad, row | kChkNoTranspose);
        }
        xmax = umax(xmax, x);
    }
    for (int d = 32; d >= 1; d >>= 1) {
        bad = umin(bad, __shfl_xor(bad, d, 64));
        xmax = umax(xmax, __shfl_xor(xmax, d, 64));
        const int od = __shfl_xor(dmax, d, 64);
        dmax = od > dmax ? od : dmax;
    }
    IngestResult *R = res + blockIdx.y;
    if ((threadIdx.x & 63) == 0) {
        if (bad != ~0ull) atomicMin(&R->first_bad, bad);
        if (xmax) atomicMax(&R->x_max, xmax);
        if (dmax) atomicMax(&R->max_degree, dmax);
    }
    __syncthreads();
    if (threadIdx.x < kMaxColours && cnt[threadIdx.x]) atomicAdd(&R->class_n[threadIdx.x], cnt[threadIdx.x]);
}

}  // namespace

hipError_t launch_ingest(const IngestDesc *d, IngestResult *r, int B, int n_max, hipStream_t s) {
    if (B <= 0 || n_max <= 0) return hipSuccess;
    const int gx = std::min(256, (n_max + 255) / 256);
    hipLaunchKernelGGL(ingest_kernel, dim3(gx, B), dim3(256), 0, s, d, r);
    return hipGetLastError();
}

}  // namespace spv
