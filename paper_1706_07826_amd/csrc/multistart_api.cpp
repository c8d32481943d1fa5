// Multi-start SPVAR (Algorithm 2) on the device: one sampler launch for the
// fixing samples of every start, the persistence step per start, the starts'
// modified problems sampled (SA: one batched launch; SQA: a launch per start),
// optional recombination over components, and the best recorded state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.hpp"

using namespace spv;

extern "C" {

spv_status spv_multistart(spv_ctx *ctx, const spv_problem *P0, const spv_multistart_params *prm,
                          const spv_multistart_out *out, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    Inst Q;
    spv_status st = ingest(c, P0, 1, kIngestColours, stream, &Q);
    if (st) return st;
    const Inst *P = &Q;
    if (!prm || !out) return set_err(c, SPV_EINVAL, "spv_multistart: NULL params/out");
    const int S = prm->starts, F = prm->fixing_reads, Rs = prm->solving_reads, n = P->n, nnz = P->nnz;
    if (S < 1 || F < 1 || Rs < 0 || (long long)S * F > (1ll << 30) || (long long)S * Rs > (1ll << 30))
        return set_err(c, SPV_EINVAL, "spv_multistart: starts=%d fixing_reads=%d solving_reads=%d", S, F, Rs);
    if (n < 1) return set_err(c, SPV_EINVAL, "spv_multistart: empty problem");
    if (!out->fixing_E || (Rs > 0 && !out->solving_E))
        return set_err(c, SPV_EINVAL, "spv_multistart: NULL energy output");
    if ((st = check_betas(c, prm->betas, prm->sweeps))) return st;
    const bool sqa = prm->sampler == 1;
    if (prm->sampler != 0 && !sqa) return set_err(c, SPV_EINVAL, "spv_multistart: sampler=%d", prm->sampler);

    // Working set.
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t nn = (size_t)n, z = (size_t)std::max(nnz, 1);
    const size_t o_rp = 0, o_col = o_rp + al(4 * (nn + 1)), o_J = o_col + al(4 * z), o_h = o_J + al(4 * z),
                 o_co = o_h + al(4 * nn), o_orig = o_co + al(nn), o_info = o_orig + al(4 * nn),
                 pstride = o_info + al(64);
    const size_t sz_fs = al((size_t)S * F * nn), sz_starts = (size_t)S * pstride, sz_fm = al((size_t)S * nn),
                 sz_E = al(8 * (size_t)S * std::max(Rs, 1)), sz_sp = al((size_t)S * std::max(Rs, 1) * nn),
                 sz_comp = al(4 * nn);
    const bool merge = prm->merge != 0 && Rs > 0;
    size_t total = sz_fs + sz_starts + 2 * sz_fm + sz_E + sz_sp + sz_comp + al(64);
    if (merge) total += sz_E + sz_sp;
    if ((st = ensure(c, c->ms, total))) return st;
    unsigned char *base = static_cast<unsigned char *>(c->ms.p), *q = base;
    int8_t *fs = reinterpret_cast<int8_t *>(q);
    q += sz_fs;
    unsigned char *starts = q;
    q += sz_starts;
    uint8_t *fm = out->fixed_mask ? out->fixed_mask : q;
    q += sz_fm;
    int8_t *fv = out->fixed_val ? out->fixed_val : reinterpret_cast<int8_t *>(q);
    q += sz_fm;
    int64_t *Ered = reinterpret_cast<int64_t *>(q);
    q += sz_E;
    int8_t *sol = reinterpret_cast<int8_t *>(q);
    q += sz_sp;
    int32_t *comp = reinterpret_cast<int32_t *>(q);
    q += sz_comp;
    int64_t *best = reinterpret_cast<int64_t *>(q);
    q += al(64);
    int64_t *mE = nullptr;
    int8_t *msp = nullptr;
    if (merge) {
        mE = reinterpret_cast<int64_t *>(q);
        q += sz_E;
        msp = reinterpret_cast<int8_t *>(q);
    }
    auto blk = [&](int s, size_t off) { return starts + (size_t)s * pstride + off; };

    // 1. Fixing samples of every start: one sampler job, start s owns reads [s*F, (s+1)*F).
    st = sqa ? sqa_inst(ctx, P, prm->betas, prm->gammas, prm->sweeps, prm->trotter, S * F, prm->seed, fs,
                              out->fixing_E, stream)
             : sample_inst(ctx, P, prm->betas, prm->sweeps, S * F, prm->seed, 0, nullptr, fs, out->fixing_E, stream);
    if (st) return st;
    // 2. SPVAR per start.
    for (int s = 0; s < S; ++s) {
        spv_fix_out fo;
        fo.fixed_mask = fm + (size_t)s * nn;
        fo.fixed_val = fv + (size_t)s * nn;
        fo.row_ptr = reinterpret_cast<int32_t *>(blk(s, o_rp));
        fo.col = reinterpret_cast<int32_t *>(blk(s, o_col));
        fo.J = reinterpret_cast<int32_t *>(blk(s, o_J));
        fo.h = reinterpret_cast<int32_t *>(blk(s, o_h));
        fo.colour = blk(s, o_co);
        fo.orig_index = reinterpret_cast<int32_t *>(blk(s, o_orig));
        fo.info = reinterpret_cast<int64_t *>(blk(s, o_info));
        if ((st = spv_persist_fix(ctx, P, fs + (size_t)s * F * nn, out->fixing_E + (size_t)s * F, F, prm->elite_frac,
                                  prm->threshold, prm->gauge, &fo, stream)))
            return st;
    }
    std::vector<int64_t> hinfo((size_t)S * 8);
    hipError_t e = hipSuccess;
    for (int s = 0; s < S && e == hipSuccess; ++s)
        e = hipMemcpyAsync(&hinfo[(size_t)s * 8], blk(s, o_info), 64, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_check(c, e, "multistart sizes");
    for (int s = 0; s < S; ++s)
        if (hinfo[(size_t)s * 8 + 7] != 0)
            return set_err(c, (spv_status)hinfo[(size_t)s * 8 + 7], "persist_fix device status %lld in start %d",
                           (long long)hinfo[(size_t)s * 8 + 7], s);
    std::vector<int32_t> ncomp(S, 0);
    const int8_t *sol_used = sol;
    const int64_t *E_used = Ered;
    if (Rs > 0) {
        // 3. Solving samples of the starts' modified problems in one batched launch.
        std::vector<Inst> probs;
        std::vector<int32_t> reads;
        std::vector<uint64_t> seeds;
        std::vector<int8_t *> sp;
        std::vector<int64_t *> en;
        std::vector<int> who;
        for (int s = 0; s < S; ++s) {
            const int nf = (int)hinfo[(size_t)s * 8 + 0];
            if (nf == 0) continue;
            Inst q2 = *P;  // keeps the parent's bounds
            q2.n = nf;
            q2.nnz = (int32_t)hinfo[(size_t)s * 8 + 1];
            q2.row_ptr = reinterpret_cast<const int32_t *>(blk(s, o_rp));
            q2.col = reinterpret_cast<const int32_t *>(blk(s, o_col));
            q2.J = reinterpret_cast<const int32_t *>(blk(s, o_J));
            q2.h = reinterpret_cast<const int32_t *>(blk(s, o_h));
            q2.colour = blk(s, o_co);
            probs.push_back(q2);
            reads.push_back(Rs);
            seeds.push_back(prm->seed + 1 + (uint64_t)s);
            sp.push_back(sol + (size_t)s * Rs * nn);
            en.push_back(Ered + (size_t)s * Rs);
            who.push_back(s);
        }
        if (sqa) {
            for (size_t b = 0; b < probs.size(); ++b)
                if ((st = sqa_inst(ctx, &probs[b], prm->betas, prm->gammas, prm->sweeps, prm->trotter, Rs,
                                         seeds[b], sp[b], en[b], stream)))
                    return st;
        } else if (!probs.empty()) {
            // Residuals after fixing are small: a workgroup just wide enough for one
            // colour class x 2 quad words (one wavefront for ~60 free variables), so each
            // item's barriers stay cheap and many items share a CU.
            int cls = 1;
            for (const Inst &q2 : probs) cls = std::max(cls, (q2.n + q2.n_colours - 1) / q2.n_colours);
            spv_batch_opts bo;
            bo.threads = std::min(256, (2 * cls + 63) / 64 * 64);
            bo.quads_per_item = 2;
            bo.wgs_per_cu = std::min(16, 1024 / bo.threads);
            bo.flags = 0;
            if ((st = sample_batch_inst(ctx, (int32_t)probs.size(), probs.data(), prm->betas, prm->sweeps, reads.data(),
                                       seeds.data(), sp.data(), en.data(), &bo, stream)))
                return st;
        }
        // 4. Optional recombination over each modified problem's components (Sec. II.C).
        if (merge) {
            for (size_t b = 0; b < probs.size(); ++b) {
                const int s = who[b];
                int32_t nc = 0;
                if ((st = spv_components(ctx, &probs[b], comp, &nc, stream))) return st;
                if ((st = spv_merge_components(ctx, &probs[b], comp, nc, sp[b], Rs, msp + (size_t)s * Rs * nn,
                                               mE + (size_t)s * Rs, nullptr, stream)))
                    return st;
                ncomp[s] = nc;
            }
            sol_used = msp;
            E_used = mE;
        }
        e = launch_ms_offset(E_used, reinterpret_cast<const int64_t *>(blk(0, o_info)), (int)(pstride / 8), S, Rs,
                             out->solving_E, stream);
        if (e != hipSuccess) return hip_check(c, e, "multistart offsets");
    }
    // 5. The best recorded state.
    e = launch_ms_best(out->fixing_E, Rs > 0 ? out->solving_E : out->fixing_E, S, F, Rs, n, fs, sol_used,
                       (size_t)Rs * nn, fm, fv, reinterpret_cast<const int32_t *>(blk(0, o_orig)), pstride / 4,
                       reinterpret_cast<const int64_t *>(blk(0, o_info)), (int)(pstride / 8), best, out->best_spins,
                       stream);
    if (e != hipSuccess) return hip_check(c, e, "multistart best");
    if (out->best_E) {
        e = hipMemcpyAsync(out->best_E, best, 8, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_check(c, e, "multistart best read-back");
    }
    if (out->info)
        for (int s = 0; s < S; ++s) {
            out->info[s * 4 + 0] = hinfo[(size_t)s * 8 + 3];
            out->info[s * 4 + 1] = hinfo[(size_t)s * 8 + 0];
            out->info[s * 4 + 2] = hinfo[(size_t)s * 8 + 2];
            out->info[s * 4 + 3] = ncomp[s];
        }
    return SPV_OK;
}

}  // extern "C"
