// Multi-start SPVAR (Algorithm 2) on the device.  [Optional] tree
// pre-processing of the problem before the loop; then the starts run their
// stages side by side: every sampling stage is one launch over all starts (the
// first samples the shared problem as one job; later stages sample each start's
// own modified problem: SA in one batched launch, SQA a launch per start), and
// every reduction stage (the correlation step, the SPVAR step of Algorithm 1,
// the optional tree step) runs per start on the device.  The host reads back
// the per-start sizes after each reduction; the best recorded state is found
// and lifted to the full problem on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

using namespace spv;

namespace {

constexpr int kMaxStarts = 4096;
constexpr int kStageCorr = 0, kStageFix = 1, kStageTree = 2, kStageSolve = 3;

inline size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

// One reduction level slot with capacity n variables and nnz entries.
MsLevelOffsets level_offsets(size_t n, size_t nnz, size_t *bytes) {
    const size_t z = std::max<size_t>(nnz, 1), nn = std::max<size_t>(n, 1);
    MsLevelOffsets o;
    size_t p = 0;
    o.rp = p;
    p += al(4 * (nn + 1));
    o.col = p;
    p += al(4 * z);
    o.J = p;
    p += al(4 * z);
    o.h = p;
    p += al(4 * nn);
    o.co = p;
    p += al(nn);
    o.orig = p;
    p += al(4 * nn);
    o.val = p;
    p += al(nn);
    o.mask = p;
    p += al(nn);
    o.kind = p;
    p += al(nn);
    o.parent = p;
    p += al(4 * nn);
    o.round = p;
    p += al(4 * nn);
    o.order = p;
    p += al(4 * nn);
    o.info = p;
    p += al(64);
    *bytes = p;
    return o;
}

spv_fix_out fix_out_of(unsigned char *L, const MsLevelOffsets &o) {
    spv_fix_out f;
    f.fixed_mask = L + o.mask;
    f.fixed_val = reinterpret_cast<int8_t *>(L + o.val);
    f.row_ptr = reinterpret_cast<int32_t *>(L + o.rp);
    f.col = reinterpret_cast<int32_t *>(L + o.col);
    f.J = reinterpret_cast<int32_t *>(L + o.J);
    f.h = reinterpret_cast<int32_t *>(L + o.h);
    f.colour = L + o.co;
    f.orig_index = reinterpret_cast<int32_t *>(L + o.orig);
    f.info = reinterpret_cast<int64_t *>(L + o.info);
    return f;
}

spv_tree_out tree_out_of(unsigned char *L, const MsLevelOffsets &o) {
    spv_tree_out t;
    t.kind = L + o.kind;
    t.value = reinterpret_cast<int8_t *>(L + o.val);
    t.parent = reinterpret_cast<int32_t *>(L + o.parent);
    t.round = reinterpret_cast<int32_t *>(L + o.round);
    t.order = reinterpret_cast<int32_t *>(L + o.order);
    t.row_ptr = reinterpret_cast<int32_t *>(L + o.rp);
    t.col = reinterpret_cast<int32_t *>(L + o.col);
    t.J = reinterpret_cast<int32_t *>(L + o.J);
    t.h = reinterpret_cast<int32_t *>(L + o.h);
    t.colour = L + o.co;
    t.orig_index = reinterpret_cast<int32_t *>(L + o.orig);
    t.info = reinterpret_cast<int64_t *>(L + o.info);
    return t;
}

// The problem a level leaves (it keeps the parent's bounds).
Inst level_problem(const Inst &parent, unsigned char *L, const MsLevelOffsets &o, int n, int nnz) {
    Inst q = parent;
    q.n = n;
    q.nnz = nnz;
    for (int k = 0; k < kMaxColours; ++k) q.class_n[k] = 0;  // not counted for the reduced problem
    q.row_ptr = reinterpret_cast<const int32_t *>(L + o.rp);
    q.col = reinterpret_cast<const int32_t *>(L + o.col);
    q.J = reinterpret_cast<const int32_t *>(L + o.J);
    q.h = reinterpret_cast<const int32_t *>(L + o.h);
    q.colour = L + o.co;
    return q;
}

struct Level {
    int type = 0;  // 1 persistence, 2 tree
    int n_prev = 0, n_next = 0;
    unsigned char *slot = nullptr;
};

}  // namespace

extern "C" {

void spv_multistart_split(int32_t total, int32_t zero_bias, int32_t *corr, int32_t *fix, int32_t *solve) {
    const int32_t t = std::max(total, 0);
    const int32_t c = zero_bias ? (int32_t)(((int64_t)2 * t) / 5) : 0, rest = t - c;
    if (corr) *corr = c;
    if (fix) *fix = (rest + 1) / 2;
    if (solve) *solve = rest - (rest + 1) / 2;
}

double spv_r99(const int64_t *start_best, int32_t starts, int64_t e_target, double per_start, double *p) {
    int32_t hit = 0;
    for (int32_t s = 0; s < starts; ++s) hit += start_best[s] <= e_target;
    const double q = starts > 0 ? (double)hit / (double)starts : 0.0;
    if (p) *p = q;
    if (hit == 0) return -1.0;
    const double n99 = hit == starts ? 1.0 : std::log(0.01) / std::log(1.0 - q);
    return std::max(1.0, n99) * per_start;
}

spv_status spv_multistart(spv_ctx *ctx, const spv_problem *P0, const spv_multistart_params *prm,
                          const spv_multistart_out *out, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    if (!prm || !out) return set_err(c, SPV_EINVAL, "spv_multistart: NULL params/out");
    const int S = prm->starts, Rc = prm->corr_reads, F = prm->fixing_reads, Rs = prm->solving_reads;
    const int Rmax = std::max(std::max(Rc, F), Rs);
    if (S < 1 || S > kMaxStarts || F < 1 || Rc < 0 || Rs < 0 || (long long)S * Rmax > (1ll << 30))
        return set_err(c, SPV_EINVAL, "spv_multistart: starts=%d corr_reads=%d fixing_reads=%d solving_reads=%d", S,
                       Rc, F, Rs);
    if (Rc > 0 && (!(prm->corr_elite_frac > 0.0 && prm->corr_elite_frac <= 1.0) ||
                   !(prm->corr_threshold > 0.0 && prm->corr_threshold <= 1.0)))
        return set_err(c, SPV_EINVAL, "spv_multistart: corr_elite_frac=%g corr_threshold=%g", prm->corr_elite_frac,
                       prm->corr_threshold);
    if (prm->corr_after < 0 || prm->corr_after > 1 || prm->preprocess < 0 || prm->preprocess > 3)
        return set_err(c, SPV_EINVAL, "spv_multistart: corr_after=%d preprocess=%d", prm->corr_after, prm->preprocess);
    if (!out->fixing_E || (Rs > 0 && !out->solving_E) || (Rc > 0 && !out->corr_E))
        return set_err(c, SPV_EINVAL, "spv_multistart: NULL energy output");
    if (prm->sweeps < 0) return set_err(c, SPV_EINVAL, "spv_multistart: sweeps=%d", prm->sweeps);
    spv_status st = check_betas(c, prm->betas, prm->sweeps);
    if (st) return st;
    const bool sqa = prm->sampler == 1;
    if (prm->sampler != 0 && !sqa) return set_err(c, SPV_EINVAL, "spv_multistart: sampler=%d", prm->sampler);
    Inst Q;
    if ((st = ingest(c, P0, 1, kIngestColours, stream, &Q))) return st;
    const Inst *P = &Q;
    const int n = P->n, nnz = P->nnz;
    if (n < 1) return set_err(c, SPV_EINVAL, "spv_multistart: empty problem");

    // Stages of every start, in order.
    int kinds[5], nst = 0;
    if (Rc > 0 && prm->corr_after == 0) kinds[nst++] = kStageCorr;
    kinds[nst++] = kStageFix;
    if (prm->preprocess & 2) kinds[nst++] = kStageTree;
    if (Rc > 0 && prm->corr_after == 1) kinds[nst++] = kStageCorr;
    if (Rs > 0) kinds[nst++] = kStageSolve;
    int n_levels = 0, n_samples = 0;
    for (int j = 0; j < nst; ++j) {
        if (kinds[j] != kStageSolve) ++n_levels;
        if (kinds[j] != kStageTree) ++n_samples;
    }

    // Working set: per-start values, two index maps, fixes, the pre-processing
    // level, a level slot per (reduction, start), a sample per sampling stage,
    // the recombined rows, per-start bests, two lift buffers.
    size_t slot_bytes = 0;
    const MsLevelOffsets lo = level_offsets((size_t)n, (size_t)nnz, &slot_bytes);
    const size_t nn = (size_t)n;
    const size_t par_bytes = al(8ull * S) + 3 * al(4ull * S);
    std::vector<size_t> smp_off(n_samples);
    size_t p = 0;
    const size_t o_par = p;
    p += par_bytes;
    const size_t o_mapA = p;
    p += al(4 * nn * S);
    const size_t o_mapB = p;
    p += al(4 * nn * S);
    const size_t o_fm = p;
    p += al(nn * S);
    const size_t o_fv = p;
    p += al(nn * S);
    const size_t o_pre = p;
    if (prm->preprocess & 1) p += slot_bytes;
    const size_t o_lvl = p;
    p += (size_t)n_levels * S * slot_bytes;
    for (int j = 0, k = 0; j < nst; ++j) {
        if (kinds[j] == kStageTree) continue;
        const int R = kinds[j] == kStageCorr ? Rc : kinds[j] == kStageFix ? F : Rs;
        smp_off[k++] = p;
        p += al((size_t)S * R * nn);
    }
    const bool merge = prm->merge != 0 && Rs > 0;
    const size_t o_merge = p;
    if (merge) p += al((size_t)S * Rs * nn);
    const size_t o_comp = p;
    p += al(4 * nn);
    const size_t o_sb = p;
    p += 2 * al(8ull * S) + al(64);
    const size_t o_lift = p;
    p += 2 * al(nn);
    if ((st = ensure(c, c->ms, p))) return st;
    // Pinned staging: per-start values (off, ncur, n_prev, n_next), level infos,
    // start bests, the best position, pivots.  The values are rewritten only
    // after a stream synchronisation, so no copy from them is still in flight.
    const size_t hb = par_bytes + al(64ull * S) + al(8ull * S) + al(64) + al(4ull * S);
    if (c->ms_host_bytes < hb) {
        if (c->ms_host) (void)hipHostFree(c->ms_host);
        c->ms_host = nullptr;
        c->ms_host_bytes = 0;
        if (hipHostMalloc(&c->ms_host, hb, hipHostMallocDefault) != hipSuccess)
            return set_err(c, SPV_ENOMEM, "hipHostMalloc(%zu)", hb);
        c->ms_host_bytes = hb;
    }
    unsigned char *base = static_cast<unsigned char *>(c->ms.p);
    unsigned char *hbase = static_cast<unsigned char *>(c->ms_host);
    long long *h_off = reinterpret_cast<long long *>(hbase);
    int *h_ncur = reinterpret_cast<int *>(hbase + al(8ull * S));
    int *h_nprev = reinterpret_cast<int *>(hbase + al(8ull * S) + al(4ull * S));
    int *h_nnext = reinterpret_cast<int *>(hbase + al(8ull * S) + 2 * al(4ull * S));
    int64_t *h_info = reinterpret_cast<int64_t *>(hbase + par_bytes);
    int64_t *h_sb = reinterpret_cast<int64_t *>(hbase + par_bytes + al(64ull * S));
    int64_t *h_best = reinterpret_cast<int64_t *>(hbase + par_bytes + al(64ull * S) + al(8ull * S));
    int32_t *h_piv = reinterpret_cast<int32_t *>(hbase + par_bytes + al(64ull * S) + al(8ull * S) + al(64));
    MsStageParams dprm;
    dprm.off = reinterpret_cast<const long long *>(base + o_par);
    dprm.ncur = reinterpret_cast<const int *>(base + o_par + al(8ull * S));
    dprm.n_prev = reinterpret_cast<const int *>(base + o_par + al(8ull * S) + al(4ull * S));
    dprm.n_next = reinterpret_cast<const int *>(base + o_par + al(8ull * S) + 2 * al(4ull * S));
    int32_t *mapA = reinterpret_cast<int32_t *>(base + o_mapA), *mapB = reinterpret_cast<int32_t *>(base + o_mapB);
    uint8_t *fm = out->fixed_mask ? out->fixed_mask : base + o_fm;
    int8_t *fv = out->fixed_val ? out->fixed_val : reinterpret_cast<int8_t *>(base + o_fv);
    auto lvl_slot = [&](int k, int s) { return base + o_lvl + ((size_t)k * S + s) * slot_bytes; };
    auto upload_params = [&]() -> hipError_t {
        return hipMemcpyAsync(base + o_par, hbase, par_bytes, hipMemcpyHostToDevice, stream);
    };
    std::vector<Inst> cur(S);
    std::vector<std::vector<Level>> lv(S);
    std::vector<int64_t> info((size_t)S * 8, 0);
    int64_t info_pre[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = 0; s < S; ++s) info[(size_t)s * 8 + 6] = -1;
    hipError_t e = hipSuccess;

    // [Optional] pre-processing of the problem before the loop.
    Inst basep = *P;
    int64_t off_pre = 0;
    spv_tree_out pre_t{};
    if (prm->preprocess & 1) {
        pre_t = tree_out_of(base + o_pre, lo);
        if ((st = spv_tree_reduce(ctx, P, &pre_t, stream))) return st;
        e = hipMemcpyAsync(h_info, pre_t.info, 64, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_check(c, e, "multistart pre-processing");
        std::memcpy(info_pre, h_info, 64);
        basep = level_problem(*P, base + o_pre, lo, (int)info_pre[0], (int)info_pre[1]);
        off_pre = info_pre[2];
    } else {
        info_pre[0] = n;
        info_pre[1] = nnz;
    }
    for (int s = 0; s < S; ++s) {
        cur[s] = basep;
        h_off[s] = off_pre;
        h_ncur[s] = basep.n;
        h_nprev[s] = h_nnext[s] = 0;
    }
    if ((e = launch_ms_map_init(mapA, S, n, basep.n, (prm->preprocess & 1) ? pre_t.orig_index : nullptr, fm, fv,
                                stream)) != hipSuccess)
        return hip_check(c, e, "multistart init");

    // Stages.  Rows of sampling stage k for start s start at its sample + s*R*n
    // (row length: the start's problem size then), except the shared first
    // stage, one job whose rows are packed at the shared problem's size.
    MsRecords recs{};
    std::vector<std::vector<int>> n_at(n_samples, std::vector<int>(S, 0));
    std::vector<std::vector<int>> depth_at(n_samples, std::vector<int>(S, 0));
    std::vector<const int8_t *> rows_of(n_samples, nullptr);
    std::vector<int> R_of(n_samples, 0), packed(n_samples, 0);
    auto start_rows = [&](int k, int s) {
        return packed[k] ? rows_of[k] + (size_t)s * R_of[k] * (size_t)basep.n : rows_of[k] + (size_t)s * R_of[k] * nn;
    };
    int ks = 0, nl = 0;
    for (int j = 0; j < nst; ++j) {
        const int kind = kinds[j];
        if (kind != kStageTree) {
            const int R = kind == kStageCorr ? Rc : kind == kStageFix ? F : Rs;
            int64_t *rec = kind == kStageCorr ? out->corr_E : kind == kStageFix ? out->fixing_E : out->solving_E;
            int8_t *sp = reinterpret_cast<int8_t *>(base + smp_off[ks]);
            const bool shared = ks == 0;
            if (shared) {
                // the problem every start shares: one job, start s owns reads [s*R, (s+1)*R)
                if (basep.n > 0) {
                    st = sqa ? sqa_inst(ctx, &basep, prm->betas, prm->gammas, prm->sweeps, prm->trotter, S * R,
                                        prm->seed, sp, rec, stream)
                             : sample_inst(ctx, &basep, prm->betas, prm->sweeps, S * R, prm->seed, 0, nullptr, sp,
                                           rec, stream);
                    if (st) return st;
                }
            } else {
                std::vector<Inst> probs;
                std::vector<int32_t> reads;
                std::vector<uint64_t> seeds;
                std::vector<int8_t *> sps;
                std::vector<int64_t *> ens;
                for (int s = 0; s < S; ++s) {
                    if (cur[s].n == 0) continue;
                    probs.push_back(cur[s]);
                    reads.push_back(R);
                    seeds.push_back(prm->seed + 1 + (uint64_t)(ks - 1) * (uint64_t)S + (uint64_t)s);
                    sps.push_back(sp + (size_t)s * R * nn);
                    ens.push_back(rec + (size_t)s * R);
                }
                if (sqa) {
                    for (size_t b = 0; b < probs.size(); ++b)
                        if ((st = sqa_inst(ctx, &probs[b], prm->betas, prm->gammas, prm->sweeps, prm->trotter, R,
                                           seeds[b], sps[b], ens[b], stream)))
                            return st;
                } else if (!probs.empty()) {
                    // Modified problems are small: a workgroup just wide enough for one colour
                    // class x 2 quad words, so each item's barriers stay cheap and many items share a CU.
                    int cls = 1;
                    for (const Inst &q2 : probs) cls = std::max(cls, (q2.n + q2.n_colours - 1) / q2.n_colours);
                    spv_batch_opts bo;
                    bo.threads = std::min(256, (2 * cls + 63) / 64 * 64);
                    bo.quads_per_item = 2;
                    bo.wgs_per_cu = std::min(16, 1024 / bo.threads);
                    bo.flags = 0;
                    if ((st = sample_batch_inst(ctx, (int32_t)probs.size(), probs.data(), prm->betas, prm->sweeps,
                                                reads.data(), seeds.data(), sps.data(), ens.data(), &bo, stream)))
                        return st;
                }
            }
            rows_of[ks] = sp;
            R_of[ks] = R;
            packed[ks] = shared ? 1 : 0;
            if (kind == kStageSolve && merge) {
                // recombination over each modified problem's components (Sec. II.C)
                int8_t *msp = reinterpret_cast<int8_t *>(base + o_merge);
                int32_t *comp = reinterpret_cast<int32_t *>(base + o_comp);
                for (int s = 0; s < S; ++s) {
                    if (cur[s].n == 0) continue;
                    int32_t nc = 0;
                    if ((st = spv_components(ctx, &cur[s], comp, &nc, stream))) return st;
                    if ((st = spv_merge_components(ctx, &cur[s], comp, nc, start_rows(ks, s), R,
                                                   msp + (size_t)s * R * nn, rec + (size_t)s * R, nullptr, stream)))
                        return st;
                    info[(size_t)s * 8 + 5] = nc;
                }
                rows_of[ks] = msp;
                packed[ks] = 0;
            }
            if ((e = upload_params()) != hipSuccess || (e = launch_ms_record(rec, S, R, dprm, stream)) != hipSuccess)
                return hip_check(c, e, "multistart record");
            for (int s = 0; s < S; ++s) {
                n_at[ks][s] = cur[s].n;
                depth_at[ks][s] = (int)lv[s].size();
            }
            recs.E[ks] = reinterpret_cast<const long long *>(rec);
            recs.R[ks] = R;
            ++ks;
            if (kind == kStageSolve) break;
        }
        // The reduction of this stage, per start (a start whose problem is empty skips it).
        bool any = false;
        for (int s = 0; s < S; ++s) {
            if (cur[s].n == 0) continue;
            any = true;
            unsigned char *L = lvl_slot(nl, s);
            if (kind == kStageTree) {
                const spv_tree_out t = tree_out_of(L, lo);
                if ((st = spv_tree_reduce(ctx, &cur[s], &t, stream))) return st;
            } else {
                const bool corr = kind == kStageCorr;
                const int64_t *E = (corr ? out->corr_E : out->fixing_E) + (size_t)s * R_of[ks - 1];
                const spv_fix_out fo = fix_out_of(L, lo);
                if ((st = spv_persist_fix(ctx, &cur[s], start_rows(ks - 1, s), E, R_of[ks - 1],
                                          corr ? prm->corr_elite_frac : prm->elite_frac,
                                          corr ? prm->corr_threshold : prm->threshold, corr ? 1 : prm->gauge, &fo,
                                          stream)))
                    return st;
            }
            e = hipMemcpyAsync(h_info + (size_t)s * 8, L + lo.info, 64, hipMemcpyDeviceToHost, stream);
            if (e != hipSuccess) return hip_check(c, e, "multistart level info");
        }
        if (!any) {
            ++nl;
            continue;
        }
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_check(c, e, "multistart sizes");
        for (int s = 0; s < S; ++s) {
            h_nprev[s] = 0;
            h_nnext[s] = 0;
            h_piv[s] = -1;
            if (cur[s].n == 0) continue;
            const int64_t *hi = h_info + (size_t)s * 8;
            if (kind != kStageTree && hi[7] != 0)
                return set_err(c, (spv_status)hi[7], "persist_fix device status %lld in start %d", (long long)hi[7], s);
            h_nprev[s] = cur[s].n;
            h_nnext[s] = (int)hi[0];
            if (kind == kStageCorr && hi[4] >= 0) h_piv[s] = (int32_t)hi[4];
        }
        // the correlation pivots in original indices (read from the current maps)
        if (kind == kStageCorr) {
            bool read = false;
            for (int s = 0; s < S; ++s)
                if (h_piv[s] >= 0) {
                    e = hipMemcpyAsync(h_piv + s, mapA + (size_t)s * n + h_piv[s], 4, hipMemcpyDeviceToHost, stream);
                    if (e != hipSuccess) return hip_check(c, e, "multistart pivot");
                    read = true;
                }
            if (read && (e = hipStreamSynchronize(stream)) != hipSuccess) return hip_check(c, e, "multistart pivot");
        }
        for (int s = 0; s < S; ++s) {
            if (h_nprev[s] == 0) continue;
            const int64_t *hi = h_info + (size_t)s * 8;
            int64_t *oi = &info[(size_t)s * 8];
            if (kind == kStageTree) {
                oi[2] += hi[7];
            } else {
                oi[kind == kStageCorr ? 0 : 1] += hi[3];
                if (kind == kStageCorr) oi[6] = h_piv[s];
            }
            h_off[s] += hi[2];
            Level l;
            l.type = kind == kStageTree ? 2 : 1;
            l.n_prev = h_nprev[s];
            l.n_next = h_nnext[s];
            l.slot = lvl_slot(nl, s);
            lv[s].push_back(l);
            cur[s] = level_problem(cur[s], l.slot, lo, (int)hi[0], (int)hi[1]);
            h_ncur[s] = cur[s].n;
        }
        if ((e = upload_params()) != hipSuccess ||
            (e = launch_ms_compose(dprm, S, n, lvl_slot(nl, 0), slot_bytes, lo, kind != kStageTree, mapA, mapB, fm,
                                   fv, stream)) != hipSuccess)
            return hip_check(c, e, "multistart compose");
        std::swap(mapA, mapB);
        ++nl;
    }
    for (int s = 0; s < S; ++s) {
        info[(size_t)s * 8 + 3] = cur[s].n;
        info[(size_t)s * 8 + 4] = h_off[s];
    }

    // The best recorded state: per-start and overall first minima on the device.
    recs.nst = ks;
    int64_t *sb_E = reinterpret_cast<int64_t *>(base + o_sb);
    int64_t *sb_pos = reinterpret_cast<int64_t *>(base + o_sb + al(8ull * S));
    int64_t *dbest = reinterpret_cast<int64_t *>(base + o_sb + 2 * al(8ull * S));
    if ((e = launch_ms_best(recs, S, sb_E, sb_pos, dbest, stream)) != hipSuccess)
        return hip_check(c, e, "multistart best");
    e = hipMemcpyAsync(h_sb, sb_E, 8ull * S, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h_best, dbest, 24, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_check(c, e, "multistart best read-back");
    if (out->best_spins) {
        // the best row, lifted through its start's levels in reverse, then the pre-processing
        const int s = (int)h_best[1];
        long long pos = h_best[2];
        int k = 0;
        while (k + 1 < ks && pos >= R_of[k]) pos -= R_of[k++];
        const int8_t *src = start_rows(k, s) + (size_t)pos * (size_t)n_at[k][s];
        int n_src = n_at[k][s];
        int8_t *bufA = reinterpret_cast<int8_t *>(base + o_lift), *bufB = bufA + al(nn), *dst = bufA;
        for (int d = depth_at[k][s] - 1; d >= 0; --d) {
            const Level &l = lv[s][d];
            if (l.type == 2) {
                const spv_tree_out t = tree_out_of(l.slot, lo);
                e = launch_tree_complete(l.n_prev, &t, n_src, l.n_prev - n_src, src, 1, dst, stream);
            } else {
                e = launch_ms_lift(src, n_src, reinterpret_cast<const int32_t *>(l.slot + lo.orig),
                                   reinterpret_cast<const int8_t *>(l.slot + lo.val), l.n_prev, dst, stream);
            }
            if (e != hipSuccess) return hip_check(c, e, "multistart lift");
            src = dst;
            n_src = l.n_prev;
            dst = dst == bufA ? bufB : bufA;
        }
        if (prm->preprocess & 1) {
            e = launch_tree_complete(n, &pre_t, basep.n, n - basep.n, src, 1, dst, stream);
            if (e != hipSuccess) return hip_check(c, e, "multistart lift");
            src = dst;
        }
        e = hipMemcpyAsync(out->best_spins, src, nn, hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) return hip_check(c, e, "multistart best state");
    }
    if (out->best_E) *out->best_E = h_best[0];
    if (out->start_best) std::memcpy(out->start_best, h_sb, 8ull * S);
    if (out->info) std::memcpy(out->info, info.data(), 64ull * S);
    if (out->info_pre) std::memcpy(out->info_pre, info_pre, 64);
    return SPV_OK;
}

}  // extern "C"
