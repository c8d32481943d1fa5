// C ABI of libspvar: argument validation, context scratch, acceptance tables,
// launch-shape selection and the iterated-SPVAR host loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "internal.hpp"


namespace spv {

spv_status set_err(Ctx *c, spv_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

spv_status hip_check(Ctx *c, hipError_t e, const char *what) {
    if (e == hipSuccess) return SPV_OK;
    return set_err(c, SPV_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

spv_status ensure(Ctx *c, DevBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (b.bytes >= bytes) return SPV_OK;
    // Growing scratch that earlier work may still read: drain the device (or,
    // for a stream-private context, its own stream) first.
    hipError_t e = c->stream_private ? hipStreamSynchronize(c->own_stream) : hipDeviceSynchronize();
    if (e != hipSuccess) return hip_check(c, e, "hipDeviceSynchronize");
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    size_t want = bytes + bytes / 4;
    e = hipMalloc(&b.p, want);
    if (e != hipSuccess) return set_err(c, SPV_ENOMEM, "hipMalloc(%zu): %s", want, hipGetErrorString(e));
    b.bytes = want;
    return SPV_OK;
}

int digits_for(int64_t x_bound) {
    int nd = 1;
    while (nd < 7 && (x_bound >> (kDigitBits * nd)) != 0) ++nd;
    return nd;
}

// T_j[d] = min(2^32-1, floor(2^32 exp(-(beta * (unit d 512^j)) / 2^scale))), evaluated as
// one double multiply, an exact power-of-two scaling, exp and an exact 2^32 scaling.
uint32_t threshold_word(double beta, int64_t unit, int scale_log2, int digit, uint32_t d) {
    const int64_t steps = unit * (int64_t)d * ((int64_t)1 << (kDigitBits * digit));
    const double energy_units = (double)steps;
    const double arg = std::ldexp(beta * energy_units, -scale_log2);
    const double v = std::exp(-arg) * 4294967296.0;
    if (v >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)std::floor(v);
}

// Words of one Metropolis table row: full base-512 digits below the top one,
// and the top digit only up to the largest value x_bound can take there.
int table_row_len(int64_t x_bound) {
    const int nd = digits_for(x_bound);
    return kDigitSize * (nd - 1) + (int)(x_bound >> (kDigitBits * (nd - 1))) + 1;
}

int swap_digits(double dbeta, int scale_log2) {
    for (int nd = 1; nd < 7; ++nd)
        if (threshold_word(dbeta, 1, scale_log2, nd, 1) == 0u) return nd;
    return 7;
}

}  // namespace spv

using namespace spv;

namespace spv {

spv_status check_problem_host(Ctx *c, const spv_problem *P) {
    if (!P) return set_err(c, SPV_EINVAL, "problem is NULL");
    if (P->n < 0 || P->n > kMaxN) return set_err(c, SPV_ECAPACITY, "n=%d outside [0, %d]", P->n, kMaxN);
    if (P->nnz < 0) return set_err(c, SPV_EINVAL, "nnz=%d < 0", P->nnz);
    if (P->n_colours < 1 || P->n_colours > kMaxColours)
        return set_err(c, SPV_EINVAL, "n_colours=%d outside [1, %d]", P->n_colours, kMaxColours);
    if (P->scale_log2 < 0 || P->scale_log2 > 30)
        return set_err(c, SPV_EINVAL, "scale_log2=%d outside [0, 30]", P->scale_log2);
    if (P->n > 0) {
        if (!P->row_ptr || !P->h || !P->colour || (P->nnz > 0 && (!P->col || !P->J)))
            return set_err(c, SPV_EINVAL, "problem array pointer is NULL");
    } else if (P->nnz != 0) {
        return set_err(c, SPV_EASYM, "n=0 with nnz=%d", P->nnz);
    }
    return SPV_OK;
}

spv_status ingest(Ctx *c, const spv_problem *P, int B, int flags, hipStream_t s, Inst *out) {
    if (B < 0 || (B > 0 && (!P || !out))) return set_err(c, SPV_EINVAL, "ingest: B=%d or NULL problem", B);
    int n_max = 0;
    const bool structure = (flags & kIngestStructure) != 0;
    for (int b = 0; b < B; ++b) {
        spv_status st = SPV_OK;
        if (!structure) {
            st = check_problem_host(c, &P[b]);
        } else if (P[b].n < 0 || P[b].n > kMaxN) {
            st = set_err(c, SPV_ECAPACITY, "n=%d outside [0, %d]", P[b].n, kMaxN);
        } else if (P[b].nnz < 0 || (P[b].n == 0 && P[b].nnz != 0)) {
            st = set_err(c, SPV_EASYM, "n=%d with nnz=%d", P[b].n, P[b].nnz);
        } else if (P[b].n > 0 && (!P[b].row_ptr || (P[b].nnz > 0 && !P[b].col))) {
            st = set_err(c, SPV_EINVAL, "problem array pointer is NULL");
        }
        if (st) return B > 1 ? set_err(c, st, "instance %d: %s", b, std::string(c->err).c_str()) : st;
        static_cast<spv_problem &>(out[b]) = P[b];
        out[b].max_degree = 1;
        out[b].x_bound = 0;
        n_max = std::max(n_max, P[b].n);
    }
    if (n_max == 0) return SPV_OK;
    const size_t b_desc = ((size_t)B * sizeof(IngestDesc) + 255) & ~(size_t)255;
    const size_t bytes = b_desc + (size_t)B * sizeof(IngestResult);
    if (c->ingest_host_bytes < bytes) {
        if (c->ingest_host) (void)hipHostFree(c->ingest_host);
        c->ingest_host = nullptr;
        c->ingest_host_bytes = 0;
        if (hipHostMalloc(&c->ingest_host, bytes, hipHostMallocDefault) != hipSuccess)
            return set_err(c, SPV_ENOMEM, "hipHostMalloc(%zu)", bytes);
        c->ingest_host_bytes = bytes;
    }
    spv_status st = ensure(c, c->ingest, bytes);
    if (st) return st;
    unsigned char *hb = static_cast<unsigned char *>(c->ingest_host);
    IngestDesc *hd = reinterpret_cast<IngestDesc *>(hb);
    IngestResult *hr = reinterpret_cast<IngestResult *>(hb + b_desc);
    for (int b = 0; b < B; ++b) {
        hd[b].row_ptr = P[b].row_ptr;
        hd[b].col = P[b].col;
        hd[b].J = structure ? nullptr : P[b].J;
        hd[b].h = structure ? nullptr : P[b].h;
        hd[b].colour = P[b].colour;
        hd[b].n = P[b].n;
        hd[b].nnz = P[b].nnz;
        hd[b].n_colours = P[b].n_colours;
        hd[b].check_colours = (!structure && (flags & kIngestColours)) ? 1 : 0;
        // race-detection build only: colourings with an edge inside a class may be let
        // through, so that the detector can be shown to see the races they cause
        if (kLdsShadow && hd[b].check_colours && std::getenv("SPVAR_SHADOW_ALLOW_COLOUR_EDGES"))
            hd[b].check_colours = 2;
        std::memset(&hr[b], 0, sizeof hr[b]);
        hr[b].first_bad = ~0ull;
    }
    unsigned char *db = static_cast<unsigned char *>(c->ingest.p);
    hipError_t e = hipMemcpyAsync(db, hb, bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_ingest(reinterpret_cast<const IngestDesc *>(db), reinterpret_cast<IngestResult *>(db + b_desc), B,
                          n_max, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hr, db + b_desc, (size_t)B * sizeof(IngestResult), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_check(c, e, "ingest");
    for (int b = 0; b < B; ++b) {
        char where[32] = "";
        if (B > 1) snprintf(where, sizeof where, "instance %d: ", b);
        const unsigned long long f = hr[b].first_bad;
        if (f != ~0ull) {
            const long long row = (long long)(f >> 8) - 1;
            switch ((unsigned)(f & 0xff)) {
            case kChkRowPtrEnds:
                return set_err(c, SPV_EASYM, "%srow_ptr[0] != 0 or row_ptr[n] != nnz=%d", where, P[b].nnz);
            case kChkRowPtrOrder:
                return set_err(c, SPV_EASYM, "%srow_ptr decreases or leaves [0, nnz] at row %lld", where, row);
            case kChkDegree:
                return set_err(c, SPV_ECAPACITY, "%srow %lld has more than %d entries", where, row, kMaxDegree);
            case kChkColourRange:
                return set_err(c, SPV_ECOLOUR, "%scolour of %lld >= n_colours=%d", where, row, P[b].n_colours);
            case kChkColRange: return set_err(c, SPV_EASYM, "%srow %lld has a column outside [0, n)", where, row);
            case kChkSelfLoop: return set_err(c, SPV_EASYM, "%sself loop at %lld", where, row);
            case kChkUnsorted: return set_err(c, SPV_EASYM, "%srow %lld not strictly increasing", where, row);
            case kChkJRange: return set_err(c, SPV_ERANGE, "%srow %lld has |J| > 32767", where, row);
            case kChkColourEdge: return set_err(c, SPV_ECOLOUR, "%srow %lld has an edge inside its colour", where, row);
            case kChkNoTranspose:
                return set_err(c, SPV_EASYM, "%srow %lld has an entry with no equal transpose", where, row);
            default: return set_err(c, SPV_EINTERNAL, "%singest code %llu", where, f);
            }
        }
        if (hr[b].x_max >= (1ull << 26))
            return set_err(c, SPV_ERANGE, "%smax_i |h_i| + sum_j |J_ij| = %llu, not below 2^26", where, hr[b].x_max);
        out[b].max_degree = std::max(1, hr[b].max_degree);
        out[b].x_bound = (int32_t)hr[b].x_max;
        for (int k = 0; k < kMaxColours; ++k) out[b].class_n[k] = (flags & kIngestColours) ? hr[b].class_n[k] : 0;
    }
    return SPV_OK;
}

spv_status check_betas(Ctx *c, const double *b, int count) {
    if (count > 0 && !b) return set_err(c, SPV_EINVAL, "betas is NULL");
    for (int k = 0; k < count; ++k)
        if (!(b[k] >= 0.0) || std::isinf(b[k]))
            return set_err(c, SPV_EINVAL, "beta[%d]=%g is not a finite non-negative number", k, b[k]);
    return SPV_OK;
}

// Tables for a list of betas, one row per beta (row_len words).  Cached on the context.
spv_status upload_tables(Ctx *c, DevBuf &dst, const double *betas, int count, int unit, int scale,
                         int nd, int row_len, hipStream_t s) {
    TableCache &tc = c->tcache;
    const bool hit = &dst == &c->tables && tc.scale == scale && tc.nd == nd && tc.row_len == row_len &&
                     tc.unit == unit && (int)tc.betas.size() == count &&
                     (count == 0 || std::memcmp(tc.betas.data(), betas, sizeof(double) * count) == 0);
    if (hit) return SPV_OK;
    const size_t words = (size_t)count * row_len;
    spv_status st = ensure(c, dst, words * 4);
    if (st) return st;
    c->host_tables.assign(words, 0u);
    for (int k = 0; k < count; ++k) {
        uint32_t *row = c->host_tables.data() + (size_t)k * row_len;
        for (int j = 0; j < nd; ++j)
            for (int d = 0; d < kDigitSize && j * kDigitSize + d < row_len; ++d)
                row[j * kDigitSize + d] = threshold_word(betas[k], unit, scale, j, (uint32_t)d);
    }
    if ((st = upload(c, dst, 0, c->host_tables.data(), words * 4, s))) return st;
    if (&dst == &c->tables) {
        tc.betas.assign(betas, betas + count);
        tc.scale = scale;
        tc.nd = nd;
        tc.row_len = row_len;
        tc.unit = unit;
    }
    return SPV_OK;
}

spv_status upload(Ctx *c, DevBuf &dst, size_t dst_off, const void *src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return SPV_OK;
    spv_status st = ensure(c, dst, dst_off + bytes);
    if (st) return st;
    hipError_t e;
    if (!c->stream_private) {
        // Earlier work on any stream may still read this buffer.
        e = hipDeviceSynchronize();
        if (e == hipSuccess)
            e = hipMemcpy(static_cast<unsigned char *>(dst.p) + dst_off, src, bytes, hipMemcpyHostToDevice);
        return hip_check(c, e, "upload");
    }
    // Stream-private: the previous staged copy must have left the staging buffer;
    // earlier kernels on the same stream are ordered before this copy.
    if (c->stage_done && (e = hipEventSynchronize(c->stage_done)) != hipSuccess)
        return hip_check(c, e, "staging event");
    if (c->stage_bytes < bytes) {
        if (c->stage) (void)hipHostFree(c->stage);
        c->stage = nullptr;
        c->stage_bytes = 0;
        if ((e = hipHostMalloc(&c->stage, bytes, hipHostMallocDefault)) != hipSuccess)
            return set_err(c, SPV_ENOMEM, "hipHostMalloc(%zu)", bytes);
        c->stage_bytes = bytes;
    }
    if (!c->stage_done && (e = hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming)) != hipSuccess)
        return hip_check(c, e, "event create");
    std::memcpy(c->stage, src, bytes);
    e = hipMemcpyAsync(static_cast<unsigned char *>(dst.p) + dst_off, c->stage, bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(c->stage_done, s);
    return hip_check(c, e, "upload");
}

// Ladder split of a tempering job (see the split kernel): whether to use it,
// the group count G and size m, the workgroup shape and whether the instance
// stays in LDS.  Groups hold a multiple of 4 slots; with cluster moves on, and
// more workgroups available than quads, groups of 2 slots (half a quad each) or,
// beyond K / 2 groups, of 1 slot: every group's cluster-move work shrinks with
// its slot count.  SPVAR_PT_SPLIT=0 disables the
// split, =1 forces it (K % 4 == 0); SPVAR_PT_GROUPS fixes G; SPVAR_PT_BIG=1
// reads the instance from global memory even when it would fit in LDS;
// SPVAR_PT_ESUM=0 keeps a group with one slot pair on the separate cluster
// energy pass.
static int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

unsigned pt_spin_limit() { return (unsigned)env_int("SPVAR_PT_SPIN", 1 << 24); }

spv_status plan_pt_split(Ctx *c, int n, int D, int K, int runs, int chains, int row_len, int nd, int icm_lo,
                         int icm_hi, bool single_fits, PtSplit *sp) {
    sp->use = false;
    const int mode = env_int("SPVAR_PT_SPLIT", -1);
    if (mode == 0 || K % 4 != 0 || n < 1) return SPV_OK;
    const int quads = K / 4, maxg = icm_hi > icm_lo ? K : quads;
    int G = env_int("SPVAR_PT_GROUPS", 0);
    if (G <= 0) G = std::max(1, std::min(maxg, c->num_cus / std::max(runs, 1)));
    G = std::min(G, maxg);
    if (mode != 1 && single_fits && G == 1) return SPV_OK;
    for (;; ++G) {
        if (G > maxg)
            return set_err(c, SPV_ECAPACITY, "PT run does not fit even split into %d groups (n=%d)", maxg, n);
        const int m = G > K / 2 ? 1 : G > quads ? 2 : 4 * ((quads + G - 1) / G);
        const int Gr = (K + m - 1) / m;
        const int nq = chains * ((m + 3) / 4);  // (one word per site when packed: fewer tasks)
        const long long tasks = (long long)n * nq;
        int threads = env_int("SPVAR_PT_THREADS", tasks >= 1536 ? 1024 : tasks >= 768 ? 512 : 256);
        while (threads < nq) threads *= 2;
        if (threads > 1024) continue;
        const int icm_slots = icm_hi > icm_lo ? std::min(m, icm_hi - icm_lo) : 0;
        for (int big = env_int("SPVAR_PT_BIG", 0) ? 1 : 0; big < 2; ++big) {
            for (int nw = std::min(icm_slots, 4); nw >= (icm_slots ? 1 : 0); --nw)
            for (int esum = nw == 1 && env_int("SPVAR_PT_ESUM", 1) ? 1 : 0; esum >= 0; --esum) {
                const size_t lds = ptx_lds_bytes(n, D, m, chains, row_len, nw, big != 0, esum != 0) + 256;
                if (lds > c->lds_max) continue;
                int bpc = 0;
                hipError_t e = ptx_max_groups_resident(nd, big != 0, D, threads, lds, &bpc);
                if (e != hipSuccess) return hip_check(c, e, "occupancy query");
                if ((long long)bpc * c->num_cus < (long long)runs * Gr)
                    return set_err(c, SPV_ECAPACITY, "split PT grid %d x %d exceeds %d resident workgroups", runs,
                                   Gr, bpc * c->num_cus);
                sp->use = true;
                sp->G = Gr;
                sp->m = m;
                sp->threads = threads;
                sp->nw_icm = nw;
                sp->esum = esum != 0;
                sp->big = big != 0;
                return SPV_OK;
            }
        }
    }
}

spv_status pt_lds_footprint(Ctx *c, const Inst *P, int K, int runs, int chains, int icm_lo, int icm_hi,
                            int64_t *lds_total) {
    const int n = P->n, D = P->max_degree > 0 ? P->max_degree : 1;
    const int nd = digits_for(P->x_bound), row_len = table_row_len(P->x_bound);
    const bool icm = icm_hi > icm_lo;
    const int cK = chains * K, nqa = (cK % 4 == 0) ? cK / 4 : cK / 4 + 2;
    const int threads = (n * nqa >= 4096) ? 1024 : 256;
    const int nw_icm = icm ? std::min(threads / 64, icm_hi - icm_lo) : 0;
    const size_t lds = pt_lds_bytes(n, D, K, chains, row_len, nqa, nw_icm) + 256;
    PtSplit sp;
    spv_status st = plan_pt_split(c, n, D, K, runs, chains, row_len, nd, icm ? icm_lo : 0, icm ? icm_hi : 0,
                                  lds <= c->lds_max, &sp);
    if (st) return st;
    if (sp.use)
        *lds_total = (int64_t)runs * sp.G * (int64_t)(ptx_lds_bytes(n, D, sp.m, chains, row_len, sp.nw_icm, sp.big, sp.esum) + 256);
    else
        *lds_total = (int64_t)runs * (int64_t)lds;
    return SPV_OK;
}

int sa_threads_env() {
    const char *v = getenv("SPVAR_SA_THREADS");
    return v ? atoi(v) : 0;
}
int sa_qw_env() {
    const char *v = getenv("SPVAR_SA_QW");
    return v ? atoi(v) : 0;
}
int sa_spin_env() {
    const char *v = getenv("SPVAR_SA_SPIN");
    const int k = v ? atoi(v) : 0;
    return k > 0 ? k : (1 << 22);
}
// SPVAR_SA_STREAM=0: never stream; =<grid>: always stream on that many workgroups.
bool sa_stream_env_off() {
    const char *v = getenv("SPVAR_SA_STREAM");
    return v && v[0] == '0';
}
int sa_stream_env_grid() {
    const char *v = getenv("SPVAR_SA_STREAM");
    const int g = v ? atoi(v) : 0;
    return g > 0 ? g : 0;
}
bool sa_big_env() {  // SPVAR_SA_BIG=1: the global-memory instance even when the LDS would hold it
    const char *v = getenv("SPVAR_SA_BIG");
    return v && v[0] == '1';
}
int sa_wpl_env() {
    const char *v = getenv("SPVAR_SA_WPL");
    return v ? atoi(v) : 0;
}

}  // namespace spv

extern "C" {

const char *spv_version(void) { return kLdsShadow ? "spvar-mi355x 0.1 (LDS race detection)" : "spvar-mi355x 0.1"; }

spv_status spv_debug_lds_shadow(spv_ctx *ctx, uint64_t counts[4], int32_t reset) {
    if (!ctx || !counts) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    if (!kLdsShadow) return set_err(c, SPV_EINVAL, "library built without LDS race detection (SPV_LDS_SHADOW=1)");
    DeviceGuard g(c->device);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_check(c, e, "synchronize before reading the race counts");
    unsigned long long v[4] = {0, 0, 0, 0};
    if ((e = shadow_stats_sa(v, reset != 0)) != hipSuccess) return hip_check(c, e, "race counts (SA)");
    if ((e = shadow_stats_batch(v, reset != 0)) != hipSuccess) return hip_check(c, e, "race counts (batch)");
    if ((e = shadow_stats_pt(v, reset != 0)) != hipSuccess) return hip_check(c, e, "race counts (tempering)");
    if ((e = shadow_stats_ptx(v, reset != 0)) != hipSuccess) return hip_check(c, e, "race counts (split tempering)");
    if ((e = shadow_stats_sqa(v, reset != 0)) != hipSuccess) return hip_check(c, e, "race counts (SQA)");
    for (int k = 0; k < 4; ++k) counts[k] = (uint64_t)v[k];
    return SPV_OK;
}

spv_status spv_ctx_create(int32_t device, spv_ctx **out) {
    if (!out) return SPV_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return SPV_EDEVICE;
    spv_ctx *x = new (std::nothrow) spv_ctx();
    if (!x) return SPV_ENOMEM;
    x->c.device = device;
    DeviceGuard g(device);
    int cus = 0, lds = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) {
        delete x;
        return SPV_EDEVICE;
    }
    x->c.num_cus = cus;
    x->c.lds_max = (size_t)lds - kShadowLdsBytes;
    // Set-up of the allocation-free persistence: this device's scratch address.
    void *na = nullptr;
    if (noalloc_scratch(device, &na) != hipSuccess) {
        delete x;
        return SPV_EDEVICE;
    }
    *out = x;
    return SPV_OK;
}

void spv_ctx_destroy(spv_ctx *ctx) {
    if (!ctx) return;
    DeviceGuard g(ctx->c.device);
    (void)hipDeviceSynchronize();
    batch_release(&ctx->c);
    if (ctx->c.stage) (void)hipHostFree(ctx->c.stage);
    if (ctx->c.ingest_host) (void)hipHostFree(ctx->c.ingest_host);
    if (ctx->c.stage_done) (void)hipEventDestroy(ctx->c.stage_done);
    for (DevBuf *b : {&ctx->c.image, &ctx->c.tables, &ctx->c.tables2, &ctx->c.scratch, &ctx->c.scratch2,
                      &ctx->c.rounds, &ctx->c.pt, &ctx->c.pt_tab, &ctx->c.top, &ctx->c.serve, &ctx->c.merge, &ctx->c.ms, &ctx->c.tree, &ctx->c.sa_stream, &ctx->c.sa_big, &ctx->c.sqa, &ctx->c.ingest})
        if (b->p) (void)hipFree(b->p);
    delete ctx;
}

const char *spv_last_error(const spv_ctx *ctx) { return ctx ? ctx->c.err.c_str() : "no context"; }

spv_status spv_problem_check(spv_ctx *ctx, const spv_problem *P, int32_t *max_degree, int32_t *x_bound) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    // Synchronous: the problem arrays may come from work on any stream.
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_check(c, e, "hipDeviceSynchronize");
    Inst Q;
    const spv_status st = ingest(c, P, 1, kIngestColours, nullptr, &Q);
    if (st) return st;
    if (max_degree) *max_degree = Q.max_degree;
    if (x_bound) *x_bound = Q.x_bound;
    return SPV_OK;
}

spv_status spv_energy(spv_ctx *ctx, const spv_problem *P0, const int8_t *spins, int32_t R,
                      int64_t *energies, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    if (R < 0) return set_err(c, SPV_EINVAL, "R=%d < 0", R);
    Inst Q;
    spv_status st = ingest(c, P0, 1, kIngestColours, stream, &Q);
    if (st) return st;
    const Inst *P = &Q;
    if (R == 0) return SPV_OK;
    if (!energies || (P->n > 0 && !spins)) return set_err(c, SPV_EINVAL, "NULL spins/energies");
    if (P->n == 0) return hip_check(c, hipMemsetAsync(energies, 0, 8ull * R, stream), "memset");
    st = ensure(c, c->image, image_words(P->n, P->max_degree) * 4);
    if (st) return st;
    hipError_t e = launch_prep(P, static_cast<int32_t *>(c->image.p), stream);
    if (e == hipSuccess)
        e = launch_energy(static_cast<int32_t *>(c->image.p), P->n, P->max_degree, spins, R, energies, stream);
    return hip_check(c, e, "energy launch");
}

}  // extern "C"

namespace spv {

spv_status sample_inst(spv_ctx *ctx, const Inst *P, const double *betas, int32_t sweeps, int32_t reads,
                       uint64_t seed, uint32_t sweep_offset, const int8_t *init_spins, int8_t *spins,
                       int64_t *energies, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    spv_status st = SPV_OK;
    if (sweeps < 0 || reads < 0) return set_err(c, SPV_EINVAL, "sweeps=%d reads=%d", sweeps, reads);
    if ((st = check_betas(c, betas, sweeps))) return st;
    if (reads == 0) return SPV_OK;
    if (!energies || (P->n > 0 && !spins)) return set_err(c, SPV_EINVAL, "NULL spins/energies");
    if (P->n == 0) return hip_check(c, hipMemsetAsync(energies, 0, 8ull * reads, stream), "memset");
    const int n = P->n, D = P->max_degree;
    const int nd = digits_for(P->x_bound);
    if (nd > 3) return set_err(c, SPV_ERANGE, "x_bound=%d needs %d digits (max 3)", P->x_bound, nd);
    const int row_len = table_row_len(P->x_bound);
    st = ensure(c, c->image, image_words(n, D) * 4);
    if (st) return st;
    hipError_t e = launch_prep(P, static_cast<int32_t *>(c->image.p), stream);
    if (e != hipSuccess) return hip_check(c, e, "prep launch");
    if (sweeps > 0) {
        st = upload_tables(c, c->tables, betas, sweeps, 2, P->scale_log2, nd, row_len, stream);
        if (st) return st;
    }
    SaLaunch L;
    L.image = static_cast<const int32_t *>(c->image.p);
    L.n = n;
    L.D = D;
    L.C = P->n_colours;
    L.tables = static_cast<const uint32_t *>(c->tables.p);
    L.row_len = row_len;
    L.nd = nd;
    L.sweeps = sweeps;
    L.sweep_offset = sweep_offset;
    L.seed = seed;
    L.reads = reads;
    L.init = init_spins;
    L.out = spins;
    L.energies = energies;
    // Launch shape: small workgroups with few quads each, so that several
    // workgroups share a CU and hide each other's barriers.  Measured: when the
    // workgroups outnumber the CUs (Chimera 8x8, 10,000 reads) the byte-parallel
    // path is fastest with 2 quads per 256-thread workgroup, each lane holding both
    // words of its site (fewer instructions per update); when they do not fill the
    // device (residual problems, 1,000 reads) two lanes per site (2 quads per
    // 512-thread workgroup) finish sooner.  The general path: 1 quad per workgroup,
    // 512 threads when the workgroups outnumber the CUs, else 1024 (measured on the
    // L = 10 and L = 20 Gaussian cubes: more sites in flight per CU when few
    // workgroups share it), and no more threads than sites.
    const bool swar = sa_use_swar(nd, row_len);
    const bool saturated = ((reads + 3) / 4 + 1) / 2 > c->num_cus;
    int qw = sa_qw_env();
    if (qw <= 0) qw = swar ? 2 : 1;
    int threads = sa_threads_env();
    if (threads <= 0) {
        if (swar)
            threads = saturated ? 256 : 512;
        else
            threads = std::min((reads + 3) / 4 > c->num_cus ? 512 : 1024, std::max(64, (n + 63) / 64 * 64));
    }
    threads = std::max(64, std::min(1024, threads / qw * qw));
    // An instance that does not fit the LDS beside its replicas stays in global
    // memory: LDS then holds the tables and the spins only.
    const int qw0 = qw;
    bool big = sa_big_env();
    if (!big) {
        while (qw > 1 && sa_lds_bytes(n, D, row_len, qw) + 256 > c->lds_max) --qw;
        if (sa_lds_bytes(n, D, row_len, qw) + 256 > c->lds_max) {
            big = true;
            qw = qw0;
        }
    }
    if (big) {
        while (qw > 1 && sa_lds_bytes(n, D, row_len, qw, true) + 256 > c->lds_max) --qw;
        if (sa_lds_bytes(n, D, row_len, qw, true) + 256 > c->lds_max)
            return set_err(c, SPV_ECAPACITY, "spins of one quad need %zu B of LDS > %zu",
                           sa_lds_bytes(n, D, row_len, qw, true), c->lds_max);
        L.global_instance = true;
        if (swar) {
            st = ensure(c, c->sa_big, sa_big_bytes(n, D));
            if (st) return st;
            L.big = static_cast<unsigned char *>(c->sa_big.p);
        }
    }
    int wpl = sa_wpl_env();
    if (wpl <= 0) wpl = saturated ? 2 : 1;
    L.qw = qw;
    L.wpl = (swar && wpl == 2 && qw == 2) ? 2 : 1;
    const int lanes_per_site = qw / L.wpl;
    L.threads = std::max(lanes_per_site, threads / lanes_per_site * lanes_per_site);
    L.spin_limit = sa_spin_env();
    const int plan = sa_stream_env_off() ? 1 : sa_stream_plan(L, c->num_cus, sa_stream_env_grid());
    c->last_sa_shape[0] = L.threads;
    c->last_sa_shape[1] = L.qw;
    c->last_sa_shape[2] = L.wpl;
    c->last_sa_shape[3] = plan == 1 ? 1 : sa_stream_chunks_of(L, plan);
    c->last_sa_shape[4] = L.global_instance ? 1 : 0;
    if (plan != 1) {
        st = ensure(c, c->sa_stream, sa_stream_bytes(n, reads, qw));
        if (st) return st;
        e = launch_sa_stream(L, plan, c->sa_stream.p, stream);
        return hip_check(c, e, "sa stream launch");
    }
    e = launch_sa(L, stream, c->lds_max);
    return hip_check(c, e, "sa launch");
}

}  // namespace spv

extern "C" {

spv_status spv_sample(spv_ctx *ctx, const spv_problem *P, const double *betas, int32_t sweeps,
                      int32_t reads, uint64_t seed, uint32_t sweep_offset, const int8_t *init_spins,
                      int8_t *spins, int64_t *energies, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    Inst Q;
    const spv_status st = ingest(c, P, 1, kIngestColours, stream, &Q);
    if (st) return st;
    return sample_inst(ctx, &Q, betas, sweeps, reads, seed, sweep_offset, init_spins, spins, energies, stream);
}

}  // extern "C"

namespace spv {

spv_status sqa_inst(spv_ctx *ctx, const Inst *P, const double *betas, const double *gammas, int32_t sweeps,
                    int32_t trotter, int32_t reads, uint64_t seed, int8_t *spins, int64_t *energies,
                    hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    spv_status st = SPV_OK;
    if (sweeps < 0 || reads < 0) return set_err(c, SPV_EINVAL, "sweeps=%d reads=%d", sweeps, reads);
    if (trotter < 8 || trotter > 256 || trotter % 8 != 0)
        return set_err(c, SPV_EINVAL, "trotter=%d: a multiple of 8 in [8, 256]", trotter);
    if (sweeps > 0 && (!betas || !gammas)) return set_err(c, SPV_EINVAL, "NULL betas/gammas");
    // Inter-slice coupling per sweep, Jp = round(P Jperp 2^scale) with
    // Jperp = -ln(tanh(beta Gamma / P)) / (2 beta), in double in this order.
    std::vector<int32_t> jp((size_t)std::max(sweeps, 1), 0);
    std::vector<double> bp((size_t)std::max(sweeps, 1), 0.0);
    int64_t jmax = 0;
    for (int t = 0; t < sweeps; ++t) {
        const double beta = betas[t], gamma = gammas[t];
        if (!(beta > 0.0) || !(gamma > 0.0) || std::isinf(beta) || std::isinf(gamma))
            return set_err(c, SPV_EINVAL, "sweep %d: beta=%g gamma=%g (both > 0 and finite)", t, beta, gamma);
        const double arg = beta * gamma / (double)trotter;
        const double jperp = -0.5 * std::log(std::tanh(arg)) / beta;
        const double v = jperp * (double)trotter * std::ldexp(1.0, P->scale_log2);
        if (!(v >= 0.0) || !(v < 16777216.0))
            return set_err(c, SPV_ERANGE, "sweep %d: slice coupling %g units outside [0, 2^24)", t, v);
        jp[t] = (int32_t)std::floor(v + 0.5);
        jmax = std::max<int64_t>(jmax, jp[t]);
        bp[t] = beta / (double)trotter;
    }
    if (reads == 0) return SPV_OK;
    if (!energies || (P->n > 0 && !spins)) return set_err(c, SPV_EINVAL, "NULL spins/energies");
    if (P->n == 0) return hip_check(c, hipMemsetAsync(energies, 0, 8ull * reads, stream), "memset");
    const int64_t xeff = (int64_t)P->x_bound + 2 * jmax;
    if (xeff >= (int64_t)1 << 26) return set_err(c, SPV_ERANGE, "x_bound + 2 Jp = %lld beyond 2^26", (long long)xeff);
    const int nd = digits_for(xeff);
    if (nd > 3) return set_err(c, SPV_ERANGE, "x_bound + 2 Jp = %lld needs %d digits (max 3)", (long long)xeff, nd);
    const int row_len = table_row_len(xeff);
    const int n = P->n, D = P->max_degree;
    // The instance moves to global memory when it does not fit beside the slices.
    bool big = getenv("SPVAR_SQA_BIG") && getenv("SPVAR_SQA_BIG")[0] == '1';
    if (!big && sqa_lds_bytes(n, D, row_len, trotter) + 256 > c->lds_max) big = true;
    if (sqa_lds_bytes(n, D, row_len, trotter, true) + 256 > c->lds_max)
        return set_err(c, SPV_ECAPACITY, "SQA: %d slices of %d variables need %zu B of LDS > %zu", trotter, n,
                       sqa_lds_bytes(n, D, row_len, trotter, true), c->lds_max);
    st = ensure(c, c->image, image_words(n, D) * 4);
    if (st) return st;
    hipError_t e = launch_prep(P, static_cast<int32_t *>(c->image.p), stream);
    if (e != hipSuccess) return hip_check(c, e, "prep launch");
    if (sweeps > 0) {
        if ((st = upload_tables(c, c->tables, bp.data(), sweeps, 2, P->scale_log2, nd, row_len, stream))) return st;
        if ((st = upload(c, c->sqa, 0, jp.data(), sizeof(int32_t) * (size_t)sweeps, stream))) return st;
    }
    SqaLaunch L;
    L.image = static_cast<const int32_t *>(c->image.p);
    L.tables = static_cast<const uint32_t *>(c->tables.p);
    L.jp = static_cast<const int32_t *>(c->sqa.p);
    L.out = spins;
    L.energies = energies;
    L.n = n;
    L.D = D;
    L.C = P->n_colours;
    L.row_len = row_len;
    L.nd = nd;
    L.sweeps = sweeps;
    L.reads = reads;
    L.P = trotter;
    L.x_bound = P->x_bound;
    L.global_instance = big;
    L.seed = seed;
    // one lane per (site, word of one parity) of the largest colour class
    const int tasks = (n + P->n_colours - 1) / P->n_colours * (trotter / 8);
    L.threads = std::max(64, std::min(1024, (tasks + 63) / 64 * 64));
    if (const char *v = getenv("SPVAR_SQA_THREADS"))  // tuning: workgroup size (results do not depend on it)
        if (atoi(v) >= 64 && atoi(v) <= 1024) L.threads = atoi(v);
    L.threads -= L.threads % (trotter / 8);
    e = launch_sqa(L, stream);
    return hip_check(c, e, "sqa launch");
}

}  // namespace spv

extern "C" {

spv_status spv_sqa_sample(spv_ctx *ctx, const spv_problem *P, const double *betas, const double *gammas,
                          int32_t sweeps, int32_t trotter, int32_t reads, uint64_t seed, int8_t *spins,
                          int64_t *energies, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    Inst Q;
    const spv_status st = ingest(c, P, 1, kIngestColours, stream, &Q);
    if (st) return st;
    return sqa_inst(ctx, &Q, betas, gammas, sweeps, trotter, reads, seed, spins, energies, stream);
}

spv_status spv_sample_last_shape(const spv_ctx *ctx, int32_t *threads, int32_t *quads_per_wg,
                                 int32_t *words_per_lane, int32_t *chunks, int32_t *global_instance) {
    if (!ctx) return SPV_EINVAL;
    if (threads) *threads = ctx->c.last_sa_shape[0];
    if (quads_per_wg) *quads_per_wg = ctx->c.last_sa_shape[1];
    if (words_per_lane) *words_per_lane = ctx->c.last_sa_shape[2];
    if (chunks) *chunks = ctx->c.last_sa_shape[3];
    if (global_instance) *global_instance = ctx->c.last_sa_shape[4];
    return SPV_OK;
}

}  // extern "C"

namespace spv {

// Argument checks and launch parameters shared by both persistence entry points;
// *scratch_bytes receives the scratch the launch needs.
spv_status persist_prepare(Ctx *c, const spv_problem *P, const int8_t *samples, const int64_t *energies, int32_t R,
                           double elite_frac, double threshold, int32_t gauge, const spv_fix_out *out, FixLaunch *L,
                           size_t *scratch_bytes) {
    spv_status st = check_problem_host(c, P);
    if (st) return st;
    if (R < 1) return set_err(c, SPV_EINVAL, "R=%d < 1", R);
    if (!(elite_frac > 0.0 && elite_frac <= 1.0)) return set_err(c, SPV_EINVAL, "elite_frac=%g outside (0,1]", elite_frac);
    if (!(threshold > 0.0 && threshold <= 1.0)) return set_err(c, SPV_EINVAL, "threshold=%g outside (0,1]", threshold);
    if (gauge < 0 || gauge > 2) return set_err(c, SPV_EINVAL, "gauge=%d", gauge);
    if (!out || !out->info || !out->fixed_mask || !out->fixed_val || !out->row_ptr || !out->h ||
        !out->colour || !out->orig_index || (P->nnz > 0 && (!out->col || !out->J)))
        return set_err(c, SPV_EINVAL, "NULL output buffer");
    if (!energies || (P->n > 0 && !samples)) return set_err(c, SPV_EINVAL, "NULL samples/energies");
    const double mm = std::ceil(elite_frac * (double)R);
    int m = (int)mm;
    m = std::max(1, std::min(m, R));
    const double kk = std::ceil(threshold * (double)m);
    const int kmin = (int)kk;
    if (kmin < 1) return set_err(c, SPV_EINVAL, "k_min < 1");
    L->P = P;
    L->image = nullptr;
    L->samples = samples;
    L->energies = energies;
    L->R = R;
    L->m = m;
    L->kmin = kmin;
    L->gauge_mode = gauge;
    L->out = out;
    L->scratch = nullptr;
    L->scratch_bytes = 0;
    *scratch_bytes = fix_scratch_bytes(P->n, R, m);
    return SPV_OK;
}

}  // namespace spv

extern "C" {

spv_status spv_persist_fix(spv_ctx *ctx, const spv_problem *P, const int8_t *samples,
                           const int64_t *energies, int32_t R, double elite_frac, double threshold,
                           int32_t gauge, const spv_fix_out *out, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    FixLaunch L;
    size_t bytes = 0;
    spv_status st = persist_prepare(c, P, samples, energies, R, elite_frac, threshold, gauge, out, &L, &bytes);
    if (st) return st;
    if ((st = ensure(c, c->scratch, bytes))) return st;
    L.scratch = c->scratch.p;
    L.scratch_bytes = c->scratch.bytes;
    return hip_check(c, launch_persist_fix(L, stream), "persist launch");
}

spv_status spv_persist_fix_noalloc(spv_ctx *ctx, const spv_problem *P, const int8_t *samples,
                                   const int64_t *energies, int32_t R, double elite_frac, double threshold,
                                   int32_t gauge, const spv_fix_out *out, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    FixLaunch L;
    size_t bytes = 0;
    spv_status st = persist_prepare(c, P, samples, energies, R, elite_frac, threshold, gauge, out, &L, &bytes);
    if (st) return st;
    if (bytes > kNoAllocScratchBytes)
        return set_err(c, SPV_ECAPACITY, "spv_persist_fix_noalloc: n=%d, R=%d, m=%d need %zu B of scratch > %zu",
                       P->n, R, L.m, bytes, kNoAllocScratchBytes);
    void *p = nullptr;
    const hipError_t e = noalloc_scratch(c->device, &p);
    if (e != hipSuccess) return hip_check(c, e, "spv_persist_fix_noalloc scratch");
    L.scratch = p;
    L.scratch_bytes = kNoAllocScratchBytes;
    return hip_check(c, launch_persist_fix(L, stream), "persist launch");
}

spv_status spv_ispvar(spv_ctx *ctx, const spv_problem *P0, const double *betas, int32_t sweeps,
                      int32_t reads, uint64_t seed, int32_t rounds, double elite_frac,
                      double threshold, int32_t gauge, uint8_t *fixed_mask, int8_t *fixed_val,
                      int64_t *round_info, int32_t *rounds_run, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    Inst Q;
    spv_status st = ingest(c, P0, 1, kIngestColours, stream, &Q);
    if (st) return st;
    const Inst *P = &Q;
    if (rounds < 0 || reads < 1) return set_err(c, SPV_EINVAL, "rounds=%d reads=%d", rounds, reads);
    if (!rounds_run || (rounds > 0 && !round_info) || (P->n > 0 && (!fixed_mask || !fixed_val)))
        return set_err(c, SPV_EINVAL, "NULL output");
    *rounds_run = 0;
    const int n = P->n, nnz = P->nnz;
    // Working set: two problem buffers, three index maps, one sample, one round output.
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t sz_prob = al(4ull * (n + 1)) + 2 * al(4ull * std::max(nnz, 1)) + al(4ull * std::max(n, 1)) +
                           al(std::max(n, 1));
    const size_t sz_map = al(4ull * std::max(n, 1));
    const size_t total = 2 * sz_prob + 3 * sz_map + al((size_t)reads * std::max(n, 1)) + al(8ull * reads) +
                         2 * al(std::max(n, 1)) + al(64);
    st = ensure(c, c->rounds, total);
    if (st) return st;
    unsigned char *base = static_cast<unsigned char *>(c->rounds.p);
    struct ProbBuf {
        int32_t *rp, *col, *J, *h;
        uint8_t *co;
    } pb[2];
    for (int b = 0; b < 2; ++b) {
        unsigned char *p = base + b * sz_prob;
        pb[b].rp = reinterpret_cast<int32_t *>(p);
        p += al(4ull * (n + 1));
        pb[b].col = reinterpret_cast<int32_t *>(p);
        p += al(4ull * std::max(nnz, 1));
        pb[b].J = reinterpret_cast<int32_t *>(p);
        p += al(4ull * std::max(nnz, 1));
        pb[b].h = reinterpret_cast<int32_t *>(p);
        p += al(4ull * std::max(n, 1));
        pb[b].co = p;
    }
    unsigned char *p = base + 2 * sz_prob;
    int32_t *orig_cur = reinterpret_cast<int32_t *>(p);
    p += sz_map;
    int32_t *orig_new = reinterpret_cast<int32_t *>(p);
    p += sz_map;
    int32_t *orig_out = reinterpret_cast<int32_t *>(p);
    p += sz_map;
    int8_t *spins = reinterpret_cast<int8_t *>(p);
    p += al((size_t)reads * std::max(n, 1));
    int64_t *E = reinterpret_cast<int64_t *>(p);
    p += al(8ull * reads);
    uint8_t *fm = p;
    p += al(std::max(n, 1));
    int8_t *fv = reinterpret_cast<int8_t *>(p);
    p += al(std::max(n, 1));
    int64_t *info = reinterpret_cast<int64_t *>(p);

    hipError_t e = hipSuccess;
    if (n > 0) {
        e = hipMemcpyAsync(pb[0].rp, P->row_ptr, 4ull * (n + 1), hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess && nnz)
            e = hipMemcpyAsync(pb[0].col, P->col, 4ull * nnz, hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess && nnz)
            e = hipMemcpyAsync(pb[0].J, P->J, 4ull * nnz, hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(pb[0].h, P->h, 4ull * n, hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(pb[0].co, P->colour, n, hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess) e = launch_iota(n, orig_cur, fixed_mask, fixed_val, stream);
    }
    if (e != hipSuccess) return hip_check(c, e, "ispvar setup");
    Inst cur = *P;  // reduced problems keep the parent's bounds
    for (int k = 0; k < kMaxColours; ++k) cur.class_n[k] = 0;
    int b = 0;
    int64_t offset_total = 0;
    std::vector<int64_t> hE(reads);
    for (int rd = 0; rd < rounds; ++rd) {
        cur.row_ptr = pb[b].rp;
        cur.col = pb[b].col;
        cur.J = pb[b].J;
        cur.h = pb[b].h;
        cur.colour = pb[b].co;
        if (cur.n == 0) break;
        st = sample_inst(ctx, &cur, betas, sweeps, reads, seed + (uint64_t)rd, 0, nullptr, spins, E, stream);
        if (st) return st;
        spv_fix_out out;
        out.fixed_mask = fm;
        out.fixed_val = fv;
        out.row_ptr = pb[1 - b].rp;
        out.col = pb[1 - b].col;
        out.J = pb[1 - b].J;
        out.h = pb[1 - b].h;
        out.colour = pb[1 - b].co;
        out.orig_index = orig_out;
        out.info = info;
        st = spv_persist_fix(ctx, &cur, spins, E, reads, elite_frac, threshold, gauge, &out, stream);
        if (st) return st;
        e = launch_compose(cur.n, fm, fv, orig_cur, fixed_mask, fixed_val, info, orig_out, orig_new, stream);
        int64_t hinfo[8];
        if (e == hipSuccess) e = hipMemcpyAsync(hinfo, info, sizeof hinfo, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(hE.data(), E, 8ull * reads, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_check(c, e, "ispvar round");
        if (hinfo[7] != 0) return set_err(c, (spv_status)hinfo[7], "persist_fix device status %lld in round %d",
                                          (long long)hinfo[7], rd);
        const int64_t best = *std::min_element(hE.begin(), hE.end());
        round_info[rd * 4 + 0] = hinfo[0];
        round_info[rd * 4 + 2] = best + offset_total;
        offset_total += hinfo[2];
        round_info[rd * 4 + 1] = offset_total;
        round_info[rd * 4 + 3] = hinfo[3];
        std::swap(orig_cur, orig_new);
        cur.n = (int32_t)hinfo[0];
        cur.nnz = (int32_t)hinfo[1];
        b = 1 - b;
        *rounds_run = rd + 1;
    }
    return SPV_OK;
}

}  // extern "C"

namespace spv {

spv_status pt_inst(spv_ctx *ctx, const Inst *P, const spv_pt_params *prm, const spv_pt_out *out,
                   hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    spv_status st = SPV_OK;
    if (!prm || !out) return set_err(c, SPV_EINVAL, "NULL params/out");
    const int K = prm->K, runs = prm->runs, chains = prm->chains;
    if (K < 1 || runs < 1 || chains < 1 || chains > 64 || prm->sweeps < 0)
        return set_err(c, SPV_EINVAL, "K=%d runs=%d chains=%d sweeps=%d", K, runs, chains, prm->sweeps);
    if ((st = check_betas(c, prm->betas, K))) return st;
    for (int k = 1; k < K; ++k)
        if (prm->betas[k] < prm->betas[k - 1]) return set_err(c, SPV_EINVAL, "betas not ascending at %d", k);
    const bool icm = prm->icm_hi > prm->icm_lo;
    if (icm && (chains != 2 || prm->icm_lo < 0 || prm->icm_hi > K))
        return set_err(c, SPV_EINVAL, "cluster moves need chains == 2 and 0 <= icm_lo < icm_hi <= K");
    if ((long long)runs * chains * K >= (1ll << 31)) return set_err(c, SPV_ERANGE, "too many replicas");
    const bool rs_top = prm->resume_top_count != nullptr;
    if (rs_top != (prm->resume_top_E != nullptr) || (P->n > 0 && rs_top != (prm->resume_top_spins != nullptr)))
        return set_err(c, SPV_EINVAL, "resume_top_spins, resume_top_E and resume_top_count: all three or none");
    PtResume rs;
    rs.spins = prm->resume_spins;
    rs.top_spins = prm->resume_top_spins;
    rs.top_E = prm->resume_top_E;
    rs.top_count = prm->resume_top_count;
    const int n = P->n, D = P->max_degree > 0 ? P->max_degree : 1;
    const int nd = digits_for(P->x_bound);
    if (nd > 3) return set_err(c, SPV_ERANGE, "x_bound=%d needs %d digits (max 3)", P->x_bound, nd);
    const int row_len = table_row_len(P->x_bound);
    const int cK = chains * K, half = K / 2, Ls = chains * half;
    const int nqa = (cK % 4 == 0) ? cK / 4 : cK / 4 + 2;
    int threads = (n * nqa >= 4096) ? 1024 : 256;
    const int nw_icm = icm ? std::min(threads / 64, prm->icm_hi - prm->icm_lo) : 0;
    const size_t lds = pt_lds_bytes(n, D, K, chains, row_len, nqa, nw_icm) + 256;
    PtSplit sp;
    if ((st = plan_pt_split(c, n, D, K, runs, chains, row_len, nd, icm ? prm->icm_lo : 0, icm ? prm->icm_hi : 0,
                            lds <= c->lds_max, &sp)))
        return st;
    if (!sp.use && lds > c->lds_max)
        return set_err(c, SPV_ECAPACITY, "PT run needs %zu B of LDS > %zu (n=%d, %d replicas)", lds, c->lds_max, n, cK);
    // Device tables: Metropolis rows per slot, swap rows per pair, swap digit counts
    // (cached on the context with the ladder they were built for).
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_mt = al((size_t)K * row_len * 4), b_st = al((size_t)std::max(K - 1, 1) * 7 * kDigitSize * 4),
                 b_snd = al((size_t)std::max(K - 1, 1) * 4);
    PtTableCache &ptc = c->pt_cache;
    const bool hit = ptc.dev == c->pt_tab.p && c->pt_tab.p && ptc.scale == P->scale_log2 && ptc.nd == nd &&
                     ptc.row_len == row_len && (int)ptc.betas.size() == K &&
                     std::memcmp(ptc.betas.data(), prm->betas, sizeof(double) * K) == 0;
    if (!hit) {
        std::vector<unsigned char> blob(b_mt + b_st + b_snd, 0);
        uint32_t *mt = reinterpret_cast<uint32_t *>(blob.data());
        uint32_t *stt = reinterpret_cast<uint32_t *>(blob.data() + b_mt);
        int32_t *snd = reinterpret_cast<int32_t *>(blob.data() + b_mt + b_st);
        snd[0] = 1;
        for (int k = 0; k < K; ++k)
            for (int j = 0; j < nd; ++j)
                for (int d = 0; d < kDigitSize && j * kDigitSize + d < row_len; ++d)
                    mt[(size_t)k * row_len + j * kDigitSize + d] =
                        threshold_word(prm->betas[k], 2, P->scale_log2, j, (uint32_t)d);
        for (int k = 0; k + 1 < K; ++k) {
            const double db = prm->betas[k + 1] - prm->betas[k];
            snd[k] = swap_digits(db, P->scale_log2);
            for (int j = 0; j < snd[k]; ++j)
                for (int d = 0; d < kDigitSize; ++d)
                    stt[((size_t)k * 7 + j) * kDigitSize + d] = threshold_word(db, 1, P->scale_log2, j, (uint32_t)d);
        }
        ptc.dev = nullptr;
        if ((st = upload(c, c->pt_tab, 0, blob.data(), blob.size(), stream))) return st;
        ptc.dev = c->pt_tab.p;
        ptc.betas.assign(prm->betas, prm->betas + K);
        ptc.scale = P->scale_log2;
        ptc.nd = nd;
        ptc.row_len = row_len;
    }
    const size_t b_top = al((size_t)runs * std::max(Ls, 1) * 10 * std::max(n, 1));
    const size_t n_grp = sp.use ? (size_t)runs * sp.G : 0;
    const size_t b_xw = al(n_grp * 4 * chains * (size_t)ptx_msg_words(std::max(n, 1)) * 4);
    st = ensure(c, c->pt, b_top + b_xw);
    if (st) return st;
    st = ensure(c, c->image, image_words(std::max(n, 1), D) * 4);
    if (st) return st;
    unsigned char *base = static_cast<unsigned char *>(c->pt_tab.p);
    unsigned char *sbase = static_cast<unsigned char *>(c->pt.p);
    hipError_t e = hipSuccess;
    Inst Pp = *P;
    Pp.max_degree = D;
    e = launch_prep(&Pp, static_cast<int32_t *>(c->image.p), stream);
    if (e != hipSuccess) return hip_check(c, e, "prep launch");
    if (sp.use) {
        PtxLaunch X;
        X.image = static_cast<const int32_t *>(c->image.p);
        X.n = n;
        X.D = D;
        X.C = P->n_colours;
        X.K = K;
        X.runs = runs;
        X.chains = chains;
        X.sweeps = prm->sweeps;
        X.sweep_offset = prm->sweep_offset;
        X.seed = prm->seed;
        X.icm_lo = icm ? prm->icm_lo : 0;
        X.icm_hi = icm ? prm->icm_hi : 0;
        X.nw_icm = sp.nw_icm;
        X.esum = sp.esum;
        X.mtab = reinterpret_cast<const uint32_t *>(base);
        X.row_len = row_len;
        X.nd = nd;
        X.stab = reinterpret_cast<const uint32_t *>(base + b_mt);
        X.snd = reinterpret_cast<const int32_t *>(base + b_mt + b_st);
        X.out = out;
        unsigned char *sc = sbase;
        X.tops = reinterpret_cast<int8_t *>(sc);
        X.xw = reinterpret_cast<uint32_t *>(sc + b_top);
        X.G = sp.G;
        X.m = sp.m;
        X.threads = sp.threads;
        X.big = sp.big;
        X.spin_limit = pt_spin_limit();
        X.resume = rs;
        return hip_check(c, launch_ptx(X, stream), "split pt launch");
    }
    PtLaunch L;
    L.image = static_cast<const int32_t *>(c->image.p);
    L.n = n;
    L.D = D;
    L.C = P->n_colours;
    L.K = K;
    L.runs = runs;
    L.chains = chains;
    L.sweeps = prm->sweeps;
    L.sweep_offset = prm->sweep_offset;
    L.seed = prm->seed;
    L.icm_lo = icm ? prm->icm_lo : 0;
    L.icm_hi = icm ? prm->icm_hi : 0;
    L.nw_icm = nw_icm;
    L.mtab = reinterpret_cast<const uint32_t *>(base);
    L.row_len = row_len;
    L.nd = nd;
    L.stab = reinterpret_cast<const uint32_t *>(base + b_mt);
    L.snd = reinterpret_cast<const int32_t *>(base + b_mt + b_st);
    L.out = out;
    L.scratch = sbase;
    L.nqa = nqa;
    L.threads = threads;
    L.resume = rs;
    return hip_check(c, launch_pt(L, stream), "pt launch");
}

}  // namespace spv

extern "C" {

spv_status spv_pt_sample(spv_ctx *ctx, const spv_problem *P, const spv_pt_params *prm,
                         const spv_pt_out *out, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    Inst Q;
    const spv_status st = ingest(c, P, 1, kIngestColours, stream, &Q);
    if (st) return st;
    return pt_inst(ctx, &Q, prm, out, stream);
}

spv_status spv_top_sample(spv_ctx *ctx, const int8_t *top_spins, const int64_t *top_E,
                          const int32_t *top_count, int32_t lists, int32_t n, int8_t *spins,
                          int64_t *energies, int32_t *rows, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    if (!rows || lists < 0 || n < 0) return set_err(c, SPV_EINVAL, "spv_top_sample: lists=%d n=%d", lists, n);
    *rows = 0;
    if (lists == 0) return SPV_OK;
    if (!top_E || !top_count || !energies || (n > 0 && (!top_spins || !spins)))
        return set_err(c, SPV_EINVAL, "spv_top_sample: null buffer");
    std::vector<int32_t> cnt(lists), off(lists);
    hipError_t e = hipMemcpyAsync(cnt.data(), top_count, 4ull * lists, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_check(c, e, "top_count read");
    int32_t total = 0;
    for (int l = 0; l < lists; ++l) {
        if (cnt[l] < 0 || cnt[l] > kTopK) return set_err(c, SPV_EINVAL, "top_count[%d] = %d", l, cnt[l]);
        off[l] = total;
        total += cnt[l];
    }
    spv_status st = upload(c, c->top, 0, off.data(), 4ull * lists, stream);
    if (st) return st;
    e = launch_top_gather(top_spins, top_E, top_count, static_cast<const int32_t *>(c->top.p), lists, n,
                          spins, energies, stream);
    if (e != hipSuccess) return hip_check(c, e, "top gather launch");
    *rows = total;
    return SPV_OK;
}

spv_status spv_components(spv_ctx *ctx, const spv_problem *P, int32_t *comp, int32_t *n_comp,
                          hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    spv_status st = check_problem_host(c, P);
    if (st) return st;
    if (!n_comp || (P->n > 0 && !comp)) return set_err(c, SPV_EINVAL, "spv_components: NULL output");
    *n_comp = 0;
    if (P->n == 0) return SPV_OK;
    if (components_lds_bytes(P->n) + 256 > c->lds_max)
        return set_err(c, SPV_ECAPACITY, "spv_components: n=%d exceeds one workgroup's LDS", P->n);
    if ((st = ensure(c, c->merge, 256))) return st;
    int32_t *dcount = static_cast<int32_t *>(c->merge.p);
    hipError_t e = launch_components(P, comp, dcount, stream);
    int32_t hcount = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hcount, dcount, 4, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_check(c, e, "components");
    *n_comp = hcount;
    return SPV_OK;
}

spv_status spv_merge_components(spv_ctx *ctx, const spv_problem *P, const int32_t *comp, int32_t n_comp,
                                const int8_t *samples, int32_t R, int8_t *merged, int64_t *merged_E,
                                int64_t *part_E, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    spv_status st = check_problem_host(c, P);
    if (st) return st;
    if (R < 0) return set_err(c, SPV_EINVAL, "spv_merge_components: R=%d", R);
    if (R == 0) return SPV_OK;
    if (P->n == 0) {
        if (!merged_E) return set_err(c, SPV_EINVAL, "spv_merge_components: NULL merged_E");
        return hip_check(c, hipMemsetAsync(merged_E, 0, 8ull * R, stream), "memset");
    }
    if (n_comp < 1 || n_comp > P->n) return set_err(c, SPV_EINVAL, "spv_merge_components: n_comp=%d", n_comp);
    if (!comp || !samples || !merged || !merged_E)
        return set_err(c, SPV_EINVAL, "spv_merge_components: NULL buffer");
    if ((size_t)n_comp * (size_t)R > (size_t)1 << 31)
        return set_err(c, SPV_ECAPACITY, "spv_merge_components: n_comp x R too large");
    if ((st = ensure(c, c->merge, 256 + merge_scratch_bytes(n_comp, R)))) return st;
    void *scratch = static_cast<unsigned char *>(c->merge.p) + 256;
    return hip_check(c, launch_merge(P, comp, n_comp, samples, R, merged, merged_E, part_E, scratch, stream),
                     "merge launch");
}

spv_status spv_colour(spv_ctx *ctx, const spv_problem *P0, uint64_t seed, uint8_t *colour, int32_t *n_colours,
                      hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    if (!P0 || !n_colours) return set_err(c, SPV_EINVAL, "spv_colour: NULL argument");
    if (P0->n > 0 && !colour) return set_err(c, SPV_EINVAL, "spv_colour: NULL colour output");
    // The colouring is the output here, and only the graph structure is read.
    Inst Q;
    spv_status st0 = ingest(c, P0, 1, kIngestStructure, stream, &Q);
    if (st0) return st0;
    const Inst *P = &Q;
    if (P->n == 0) {
        *n_colours = 1;
        return SPV_OK;
    }
    if (colour_lds_bytes(P->n) + 256 > c->lds_max)
        return set_err(c, SPV_ECAPACITY, "spv_colour: n=%d needs %zu B of LDS", P->n, colour_lds_bytes(P->n));
    spv_status st = ensure(c, c->scratch2, (size_t)P->n * 4 + 64);
    if (st) return st;
    uint32_t *prio = static_cast<uint32_t *>(c->scratch2.p);
    int *info = reinterpret_cast<int *>(static_cast<unsigned char *>(c->scratch2.p) + (((size_t)P->n * 4 + 15) & ~(size_t)15));
    hipError_t e = launch_colour(P, seed, colour, prio, info, stream);
    int h[4] = {0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(h, info, 3 * sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_check(c, e, "colour");
    *n_colours = h[0];
    if (h[2]) return set_err(c, SPV_ERANGE, "spv_colour: more than %d colours needed", kMaxColours);
    return SPV_OK;
}

spv_status spv_lds_probe(spv_ctx *ctx, int32_t iters, double *bytes_per_s, hipStream_t stream) {
    if (!ctx || !bytes_per_s) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    if (iters < 1 || iters > (1 << 24)) return set_err(c, SPV_EINVAL, "spv_lds_probe: iters=%d", iters);
    spv_status st = ensure(c, c->scratch2, (size_t)2 * c->num_cus * 4);
    if (st) return st;
    return hip_check(c, run_lds_probe(iters, c->num_cus, static_cast<uint32_t *>(c->scratch2.p), bytes_per_s, stream),
                     "lds probe");
}

spv_status spv_philox_probe(spv_ctx *ctx, int32_t iters, double *blocks_per_s, hipStream_t stream) {
    if (!ctx || !blocks_per_s) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    if (iters < 1 || iters > (1 << 24)) return set_err(c, SPV_EINVAL, "spv_philox_probe: iters=%d", iters);
    spv_status st = ensure(c, c->scratch2, (size_t)16 * c->num_cus * 4);
    if (st) return st;
    return hip_check(c,
                     run_philox_probe(iters, c->num_cus, static_cast<uint32_t *>(c->scratch2.p), blocks_per_s, stream),
                     "philox probe");
}

spv_status spv_tree_reduce(spv_ctx *ctx, const spv_problem *P, const spv_tree_out *out, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    spv_status st = check_problem_host(c, P);
    if (st) return st;
    if (!out || !out->info || !out->row_ptr)
        return set_err(c, SPV_EINVAL, "spv_tree_reduce: NULL output");
    if (P->n > 0 && (!out->kind || !out->value || !out->parent || !out->round || !out->order || !out->h ||
                     !out->colour || !out->orig_index || (P->nnz > 0 && (!out->col || !out->J))))
        return set_err(c, SPV_EINVAL, "spv_tree_reduce: NULL output");
    if (P->n == 0) {
        const int64_t zero[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        hipError_t e = hipMemsetAsync(out->row_ptr, 0, 4, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(out->info, zero, sizeof zero, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        return hip_check(c, e, "tree reduce (empty)");
    }
    if (!tree_state_in_lds(P->n, c->lds_max) && (st = ensure(c, c->tree, tree_scratch_bytes(P->n)))) return st;
    return hip_check(c, launch_tree_reduce(P, out, c->tree.p, c->lds_max, stream), "tree reduce launch");
}

spv_status spv_tree_complete(spv_ctx *ctx, int32_t n, const spv_tree_out *t, int32_t n_free, int32_t n_removed,
                             const int8_t *reduced, int32_t R, int8_t *full, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    if (!t || n < 0 || R < 0 || n_free < 0 || n_removed < 0 || n_free + n_removed != n)
        return set_err(c, SPV_EINVAL, "spv_tree_complete: n=%d n_free=%d n_removed=%d R=%d", n, n_free, n_removed, R);
    if (R == 0 || n == 0) return SPV_OK;
    if (!full || (n_free > 0 && (!reduced || !t->orig_index)) ||
        (n_removed > 0 && (!t->kind || !t->value || !t->parent || !t->order)))
        return set_err(c, SPV_EINVAL, "spv_tree_complete: NULL buffer");
    return hip_check(c, launch_tree_complete(n, t, n_free, n_removed, reduced, R, full, stream), "tree complete");
}

}  // extern "C"
