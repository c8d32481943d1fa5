// Tree / degree-1 pre-processing (Sec. II.C) and the completion of reduced
// states.
//
// One workgroup removes, round by round, every remaining variable with at most
// one remaining J != 0 neighbour (of two variables joined only to each other,
// the larger index first): a variable whose coupler cannot outweigh its bias
// is fixed to -sign(h), otherwise its value follows its neighbour's, and its
// effect is folded into the neighbour's bias and the offset.  Degrees are
// kept incrementally and each round only visits the neighbours whose degree
// fell to one or zero in the previous round, so the work is O(n + nnz).  Each
// variable also keeps the XOR of its remaining neighbours' indices and of
// their couplers: once one neighbour is left, the two words are that
// neighbour and its coupler, so a round reads no adjacency at all.
// Within a round the removals are independent (a variable being removed never
// receives a fold in the same round), so the result does not depend on the
// order inside a round.  The remaining variables form the reduced problem.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "internal.hpp"

namespace spv {

namespace {

struct TreeArgs {
    const int32_t *row_ptr, *col, *J, *h;
    const uint8_t *colour;
    int n, nnz;
    // outputs
    uint8_t *kind;
    int8_t *value;
    int32_t *parent, *round, *order;
    int32_t *row_ptr_o, *col_o, *J_o, *h_o;
    uint8_t *colour_o;
    int32_t *orig_o;
    long long *info;
    unsigned char *scratch;  // working state when it does not fit in LDS
};

// Working state, byte offsets from one base (LDS or the scratch buffer):
//   hw    int32 [n]        biases as folds arrive
//   nx    int32 [n]        XOR of the remaining J != 0 neighbours' indices; afterwards the new index
//   jx    uint32 [n]       XOR of their couplers
//   deg   uint16 [n]       remaining J != 0 neighbours, two to a 32-bit word (updated by word atomics)
//   lst   uint32 [n / 32]  bit set: already listed for the next round
//   listA, listB uint16 [n]  candidates of this round / the next
//   kind  uint8 [n]        0 remaining, 1 fixed, 2 inferred, 3 removed in the current round
struct TreeLayout {
    size_t hw, nx, jx, deg, lst, la, lb, kind, bytes;
};

__host__ __device__ inline TreeLayout tree_layout(int n) {
    const size_t N = (size_t)(n > 0 ? n : 1), N2 = (N + 1) & ~(size_t)1;
    TreeLayout L;
    L.hw = 0;
    L.nx = L.hw + 4 * N;
    L.jx = L.nx + 4 * N;
    L.deg = L.jx + 4 * N;
    L.lst = L.deg + 2 * N2;
    L.la = L.lst + 4 * ((N + 31) / 32);
    L.lb = L.la + 2 * N2;
    L.kind = L.lb + 2 * N2;
    L.bytes = (L.kind + N + 15) & ~(size_t)15;
    return L;
}

__device__ inline int deg_of(const uint32_t *deg, int i) { return (int)((deg[i >> 1] >> (16 * (i & 1))) & 0xFFFFu); }

// kLds: the working state lives in LDS (n small enough), else in the scratch buffer.
template <bool kLds>
__global__ __launch_bounds__(1024) void tree_kernel(TreeArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int scan_tmp[1024 / 64 + 1];
    __shared__ int n_cur, n_next, n_removed, n_fix, n_inf, base_s, base_z;
    __shared__ long long offset;
    const int tid = threadIdx.x, T = blockDim.x, n = a.n;
    const TreeLayout Ly = tree_layout(n);
    unsigned char *base;
    if constexpr (kLds)
        base = smem;
    else
        base = a.scratch;
    int32_t *hw = reinterpret_cast<int32_t *>(base + Ly.hw);
    int32_t *nx = reinterpret_cast<int32_t *>(base + Ly.nx);
    uint32_t *jx = reinterpret_cast<uint32_t *>(base + Ly.jx);
    uint32_t *deg = reinterpret_cast<uint32_t *>(base + Ly.deg);
    uint32_t *lst = reinterpret_cast<uint32_t *>(base + Ly.lst);
    uint16_t *cur = reinterpret_cast<uint16_t *>(base + Ly.la);
    uint16_t *next = reinterpret_cast<uint16_t *>(base + Ly.lb);
    uint8_t *kind = base + Ly.kind;
    if (tid == 0) {
        n_cur = 0;
        n_next = 0;
        n_removed = 0;
        n_fix = 0;
        n_inf = 0;
        offset = 0;
    }
    for (int w = tid; w < (n + 31) / 32; w += T) lst[w] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += T) {
        kind[i] = 0;
        a.kind[i] = 0;
        a.value[i] = 0;
        a.parent[i] = -1;
        a.round[i] = -1;
        hw[i] = a.h[i];
        int d = 0, x = 0;
        uint32_t y = 0;
        for (int k = a.row_ptr[i]; k < a.row_ptr[i + 1]; ++k) {
            const int32_t v = a.J[k];
            if (v != 0) {
                ++d;
                x ^= a.col[k];
                y ^= (uint32_t)v;
            }
        }
        nx[i] = x;
        jx[i] = y;
        reinterpret_cast<uint16_t *>(deg)[i] = (uint16_t)d;
        if (d <= 1) cur[atomicAdd(&n_cur, 1)] = (uint16_t)i;  // the first round's candidates
    }
    __syncthreads();
    int rounds = 0;
    for (;;) {
        const int nc = n_cur, removed_before = n_removed;
        if (nc == 0) break;
        // decide: a candidate of degree <= 1 goes; of an isolated pair, the larger index first
        for (int x = tid; x < nc; x += T) {
            const int i = cur[x];
            const int d = deg_of(deg, i);
            if (d <= 1) {
                const int j = d == 1 ? nx[i] : -1;
                if (!(j >= 0 && deg_of(deg, j) == 1 && j > i)) kind[i] = 3;
            }
            if (rounds > 0) atomicAnd(&lst[i >> 5], ~(1u << (i & 31)));
        }
        __syncthreads();
        // apply (the neighbour of a removed variable stays this round, so its words are stable)
        for (int x = tid; x < nc; x += T) {
            const int i = cur[x];
            if (kind[i] != 3) continue;
            const long long hi = hw[i];
            a.round[i] = rounds;
            a.order[atomicAdd(&n_removed, 1)] = i;
            if (deg_of(deg, i) == 0) {
                const int8_t s = hi > 0 ? -1 : 1;
                kind[i] = 1;
                a.kind[i] = 1;
                a.value[i] = s;
                atomicAdd(reinterpret_cast<unsigned long long *>(&offset), (unsigned long long)(hi * s));
                atomicAdd(&n_fix, 1);
                continue;
            }
            const int j = nx[i];
            const int32_t Jw = (int32_t)jx[i];
            const long long Jv = Jw, aJ = Jv < 0 ? -Jv : Jv, ah = hi < 0 ? -hi : hi;
            a.parent[i] = j;
            if (aJ <= ah) {
                const int8_t s = hi > 0 ? -1 : 1;
                kind[i] = 1;
                a.kind[i] = 1;
                a.value[i] = s;
                atomicAdd(&hw[j], (int32_t)(Jv * s));
                atomicAdd(reinterpret_cast<unsigned long long *>(&offset), (unsigned long long)(hi * s));
                atomicAdd(&n_fix, 1);
            } else {
                const int8_t f = Jv > 0 ? -1 : 1;
                kind[i] = 2;
                a.kind[i] = 2;
                a.value[i] = f;
                atomicAdd(&hw[j], (int32_t)(f * hi));
                atomicAdd(reinterpret_cast<unsigned long long *>(&offset), (unsigned long long)(-aJ));
                atomicAdd(&n_inf, 1);
            }
            // Take the edge out of the neighbour's words.  Its count is >= 1, so the half-word never
            // borrows; it is listed once for the next round when at most one neighbour is left.
            atomicXor(&nx[j], i);
            atomicXor(&jx[j], (uint32_t)Jw);
            const int sh = 16 * (j & 1);
            const int nd = (int)((atomicSub(&deg[j >> 1], 1u << sh) >> sh) & 0xFFFFu) - 1;
            if (nd <= 1) {
                const uint32_t bit = 1u << (j & 31);
                if (!(atomicOr(&lst[j >> 5], bit) & bit)) next[atomicAdd(&n_next, 1)] = (uint16_t)j;
            }
        }
        __syncthreads();
        const bool progressed = n_removed > removed_before;  // a round counts when it removes something
        if (tid == 0) {
            n_cur = n_next;
            n_next = 0;
        }
        uint16_t *t = cur;
        cur = next;
        next = t;
        if (progressed) ++rounds;
        __syncthreads();
        if (!progressed) break;
    }
    // the reduced problem: remaining variables in index order (nx now holds the new index)
    int32_t *newidx = nx;
    if (tid == 0) {
        base_s = 0;
        base_z = 0;
    }
    __syncthreads();
    for (int i0 = 0; i0 < n; i0 += T) {
        const int i = i0 + tid;
        const int keep = (i < n && kind[i] == 0) ? 1 : 0;
        int tot;
        const int ex = dev::block_exclusive_scan(keep, scan_tmp, &tot);
        if (keep) {
            newidx[i] = base_s + ex;
            a.orig_o[base_s + ex] = i;
        } else if (i < n) {
            newidx[i] = -1;
        }
        __syncthreads();
        if (tid == 0) base_s += tot;
        __syncthreads();
    }
    const int nf = base_s;
    if (tid == 0) a.row_ptr_o[0] = 0;
    for (int u0 = 0; u0 < nf; u0 += T) {
        const int u = u0 + tid;
        int cnt = 0, i = -1;
        if (u < nf) {
            i = a.orig_o[u];
            for (int k = a.row_ptr[i]; k < a.row_ptr[i + 1]; ++k) cnt += kind[a.col[k]] == 0;
        }
        int tot;
        const int ex = dev::block_exclusive_scan(cnt, scan_tmp, &tot);
        if (u < nf) {
            int z = base_z + ex;
            for (int k = a.row_ptr[i]; k < a.row_ptr[i + 1]; ++k)
                if (kind[a.col[k]] == 0) {
                    a.col_o[z] = newidx[a.col[k]];
                    a.J_o[z] = a.J[k];
                    ++z;
                }
            a.row_ptr_o[u + 1] = base_z + ex + cnt;
            a.h_o[u] = hw[i];
            a.colour_o[u] = a.colour[i];
        }
        __syncthreads();
        if (tid == 0) base_z += tot;
        __syncthreads();
    }
    if (tid == 0) {
        a.info[0] = nf;
        a.info[1] = base_z;
        a.info[2] = offset;
        a.info[3] = n_fix;
        a.info[4] = n_inf;
        a.info[5] = rounds;
        a.info[6] = 0;
        a.info[7] = n_removed;
    }
}

// Completion: one thread per row; the removed variables in reverse removal
// order (a followed neighbour is removed in a later round or remains).
__global__ void tree_complete_kernel(int n, const uint8_t *__restrict__ kind, const int8_t *__restrict__ value,
                                     const int32_t *__restrict__ parent, const int32_t *__restrict__ order,
                                     int n_removed, const int32_t *__restrict__ orig, int n_free,
                                     const int8_t *__restrict__ reduced, int R, int8_t *__restrict__ full) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    int8_t *s = full + (size_t)r * n;
    const int8_t *red = reduced + (size_t)r * n_free;
    for (int u = 0; u < n_free; ++u) s[orig[u]] = red[u];
    for (int x = n_removed - 1; x >= 0; --x) {
        const int v = order[x];
        s[v] = kind[v] == 1 ? value[v] : (int8_t)(value[v] * s[parent[v]]);
    }
}

}  // namespace

size_t tree_scratch_bytes(int n) { return tree_layout(n).bytes; }

bool tree_state_in_lds(int n, size_t lds_max) { return tree_layout(n).bytes + 256 <= lds_max; }

hipError_t launch_tree_reduce(const spv_problem *P, const spv_tree_out *out, void *scratch, size_t lds_max,
                              hipStream_t s) {
    TreeArgs a;
    a.row_ptr = P->row_ptr;
    a.col = P->col;
    a.J = P->J;
    a.h = P->h;
    a.colour = P->colour;
    a.n = P->n;
    a.nnz = P->nnz;
    a.kind = out->kind;
    a.value = out->value;
    a.parent = out->parent;
    a.round = out->round;
    a.order = out->order;
    a.row_ptr_o = out->row_ptr;
    a.col_o = out->col;
    a.J_o = out->J;
    a.h_o = out->h;
    a.colour_o = out->colour;
    a.orig_o = out->orig_index;
    a.info = reinterpret_cast<long long *>(out->info);
    a.scratch = static_cast<unsigned char *>(scratch);
    if (tree_state_in_lds(P->n, lds_max))
        hipLaunchKernelGGL(tree_kernel<true>, dim3(1), dim3(1024), tree_layout(P->n).bytes, s, a);
    else
        hipLaunchKernelGGL(tree_kernel<false>, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tree_complete(int n, const spv_tree_out *t, int n_free, int n_removed, const int8_t *reduced, int R,
                                int8_t *full, hipStream_t s) {
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL(tree_complete_kernel, dim3((R + 255) / 256), dim3(256), 0, s, n, t->kind, t->value, t->parent,
                       t->order, n_removed, t->orig_index, n_free, reduced, R, full);
    return hipGetLastError();
}

}  // namespace spv
