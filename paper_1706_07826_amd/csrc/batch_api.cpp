// Host side of the batched launch: descriptors, largest-first work list,
// hipGraph capture and replay per batch shape, and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.hpp"


namespace spv {

void batch_release(Ctx *c) {
    for (auto &g : c->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    if (c->batch_host) (void)hipHostFree(c->batch_host);
    c->batch_host = nullptr;
    c->batch_host_bytes = 0;
    if (c->batch_done) (void)hipEventDestroy(c->batch_done);
    c->batch_done = nullptr;
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    c->capture_stream = nullptr;
    if (c->batch.p) (void)hipFree(c->batch.p);
    c->batch.p = nullptr;
    c->batch.bytes = 0;
}

namespace {

struct Shape {
    int threads, qw, wgs_per_cu;
    bool paired = false;  // the paired body (copies of 2 quads per item, chosen per instance)
};

struct Plan {
    int B = 0, n_max = 0, D_max = 1, nd = 1, row_len = 1, scale = 0, dk = 0;
    long long image_words = 0, total_quads = 0;
    std::vector<BatchInst> insts;
    std::vector<std::vector<int>> classes;  // class sizes per instance (empty: not counted)
};

constexpr int kMaxPairCopies = 64;

// The paired body's item list and LDS: per instance, the copy count k that fills the
// most lanes of a class pass (k x class size over whole multiples of the workgroup,
// class size estimated as ceil(n / C)), within the spin area the LDS leaves after the
// records and site constants (lds_wg bytes per workgroup).  Returns false when even one
// copy of the largest instance does not fit.
struct PairPlan {
    std::vector<int32_t> items;
    int pairs_qw = 0, kmax = 1;
    size_t lds = 0;
};

bool make_pair_items(const Plan &pl, int threads, size_t lds_wg, PairPlan *pp) {
    // the spin area is allocated in granules of 2 n_max words: keep one granule of margin
    const size_t fixed = batch_paired_lds_bytes(pl.n_max, pl.dk, pl.row_len, 0, kMaxPairCopies) + 512 +
                         8 * (size_t)std::max(pl.n_max, 1);
    if (fixed >= lds_wg) return false;
    const size_t s_budget = lds_wg - fixed;
    std::vector<int> order(pl.B);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return pl.insts[a].n > pl.insts[b].n; });
    pp->items.clear();
    pp->kmax = 1;
    long long s_words = 0;
    for (int b : order) {
        const BatchInst &in = pl.insts[b];
        const int quads = (in.reads + 3) / 4;
        if (quads == 0 || in.n <= 0) continue;
        const int pairs = (quads + 1) / 2;
        const long long per_copy = 16ll * in.n;  // bytes of one pair's region
        if (per_copy > (long long)s_budget) return false;
        const int kcap = (int)std::min<long long>({(long long)kMaxPairCopies, (long long)pairs,
                                                    (long long)s_budget / per_copy});
        std::vector<int> cls = pl.classes[b];
        if (cls.empty()) cls.assign(in.C, std::max(1, (in.n + in.C - 1) / in.C));  // estimate
        int best_k = 1;
        double best_u = -1.0;
        for (int k = 1; k <= kcap; ++k) {
            long long tasks = 0, slots = 0;
            for (int c : cls) {
                const long long t = (long long)k * c;
                tasks += t;
                slots += (t + threads - 1) / threads * threads;
            }
            const double u = slots ? (double)tasks / (double)slots : 0.0;
            if (u >= best_u - 1e-9) {
                best_u = u;
                best_k = k;
            }
        }
        // the instance's pairs in items of as equal a size as best_k allows
        const int n_it = (pairs + best_k - 1) / best_k, base_k = pairs / n_it, extra = pairs % n_it;
        for (int j = 0, first = 0; j < n_it; ++j) {
            const int k = base_k + (j < extra ? 1 : 0);
            pp->items.push_back(b);
            pp->items.push_back(2 * first);
            pp->items.push_back(k);
            pp->kmax = std::max(pp->kmax, k);
            s_words = std::max<long long>(s_words, 4ll * in.n * k);
            first += k;
        }
    }
    const int nm = std::max(pl.n_max, 1);
    pp->pairs_qw = (int)((s_words + 2ll * nm - 1) / (2ll * nm));
    pp->lds = batch_paired_lds_bytes(pl.n_max, pl.dk, pl.row_len, pp->pairs_qw, pp->kmax);
    return pp->lds + 256 <= lds_wg;
}

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Quads per item of instance b: at least the base shape, more for small
// instances so that (class size x quads) fills the workgroup, within the LDS
// spin capacity of the base shape (n_max x qw words).
int item_quads(const Plan &pl, int b, int qw, int threads) {
    const BatchInst &in = pl.insts[b];
    if (in.n <= 0) return qw;
    const int cls = std::max(1, (in.n + in.C - 1) / in.C);
    const int want = std::max(qw, threads / cls);
    const int cap = std::max(qw, (int)((long long)pl.n_max * qw / in.n));
    return std::max(1, std::min(std::min(want, cap), std::max(qw, kBatchMaxItemQuads)));
}

// Largest-instance-first list of (instance, first quad, quads) items.
std::vector<int32_t> make_items(const Plan &pl, int qw, int threads) {
    std::vector<int> order(pl.B);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return pl.insts[a].n > pl.insts[b].n; });
    std::vector<int32_t> items;
    for (int b : order) {
        const int quads = (pl.insts[b].reads + 3) / 4;
        const int qb = item_quads(pl, b, qw, threads);
        for (int q0 = 0; q0 < quads; q0 += qb) {
            items.push_back(b);
            items.push_back(q0);
            items.push_back(qb);
        }
    }
    return items;
}

// Device layout: [insts][items][counter][images]; host staging mirrors [insts][items].
struct Layout {
    size_t insts, items, counter, images, total, host;
};

Layout layout_for(const Plan &pl, size_t n_items) {
    Layout l;
    l.insts = 0;
    l.items = al256(sizeof(BatchInst) * std::max(pl.B, 1));
    l.counter = l.items + al256(12 * std::max<size_t>(n_items, 1));
    l.images = l.counter + 256;
    l.total = l.images + al256(4 * std::max<long long>(pl.image_words, 1));
    l.host = l.counter;
    return l;
}

spv_status enqueue(Ctx *c, const Plan &pl, const Layout &ly, size_t n_items, const Shape &sh,
                   int sweeps, uint32_t sweep_offset, hipStream_t s, const PairPlan *pp = nullptr) {
    unsigned char *dev = static_cast<unsigned char *>(c->batch.p);
    hipError_t e = hipMemcpyAsync(dev, c->batch_host, ly.host, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_check(c, e, "batch descriptor upload");
    const BatchInst *insts = reinterpret_cast<const BatchInst *>(dev + ly.insts);
    int32_t *images = reinterpret_cast<int32_t *>(dev + ly.images);
    e = launch_batch_prep(insts, pl.B, pl.n_max, images, s);
    if (e != hipSuccess) return hip_check(c, e, "batch prep");
    BatchLaunch L;
    L.insts = insts;
    L.items = reinterpret_cast<const int32_t *>(dev + ly.items);
    L.n_items = (int)n_items;
    L.counter = reinterpret_cast<int *>(dev + ly.counter);
    L.images = images;
    L.tables = static_cast<const uint32_t *>(c->tables.p);
    L.row_len = pl.row_len;
    L.nd = pl.nd;
    L.sweeps = sweeps;
    L.qw = sh.qw;
    L.n_max = pl.n_max;
    L.D_max = pl.D_max;
    L.dk = pl.dk;
    L.threads = sh.threads;
    L.grid = (int)std::max<size_t>(1, std::min<size_t>(n_items, (size_t)c->num_cus * sh.wgs_per_cu));
    L.sweep_offset = sweep_offset;
    if (sh.paired && pp) {
        L.paired = true;
        L.pairs_qw = pp->pairs_qw;
        L.kmax = pp->kmax;
        L.qw = 2;
    }
    return hip_check(c, launch_batch_sa(L, s), "batch launch");
}

spv_status stage(Ctx *c, const Plan &pl, const std::vector<int32_t> &items, const Layout &ly) {
    if (c->batch_done) {
        hipError_t e = hipEventSynchronize(c->batch_done);  // previous launch read the staging
        if (e != hipSuccess) return hip_check(c, e, "batch event");
    }
    if (c->batch_host_bytes < ly.host) {
        if (c->batch_host) (void)hipHostFree(c->batch_host);
        c->batch_host = nullptr;
        c->batch_host_bytes = 0;
        for (auto &g : c->graphs)
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
        c->graphs.clear();  // graphs captured the old staging address
        const size_t want = ly.host + ly.host / 2 + 4096;
        hipError_t e = hipHostMalloc(&c->batch_host, want, hipHostMallocDefault);
        if (e != hipSuccess) return set_err(c, SPV_ENOMEM, "hipHostMalloc(%zu)", want);
        c->batch_host_bytes = want;
    }
    unsigned char *h = static_cast<unsigned char *>(c->batch_host);
    std::memcpy(h + ly.insts, pl.insts.data(), sizeof(BatchInst) * pl.B);
    std::memcpy(h + ly.items, items.data(), 4 * items.size());
    return SPV_OK;
}

spv_status ensure_batch_buf(Ctx *c, size_t bytes) {
    if (c->batch.bytes >= bytes) return SPV_OK;
    for (auto &g : c->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();  // graphs captured the old device address
    return ensure(c, c->batch, bytes);
}

}  // namespace
}  // namespace spv

using namespace spv;

namespace spv {

spv_status sample_batch_inst(spv_ctx *ctx, int32_t B, const Inst *problems, const double *betas, int32_t sweeps,
                             const int32_t *reads, const uint64_t *seeds, int8_t *const *spins,
                             int64_t *const *energies, const spv_batch_opts *opts, hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    if (B < 0 || (B > 0 && (!problems || !reads || !seeds || !spins || !energies)))
        return set_err(c, SPV_EINVAL, "B=%d or NULL batch array", B);
    if (sweeps < 0) return set_err(c, SPV_EINVAL, "sweeps=%d", sweeps);
    spv_status st = check_betas(c, betas, sweeps);
    if (st) return st;
    if (B == 0) return SPV_OK;
    Plan pl;
    pl.B = B;
    pl.insts.resize(B);
    pl.classes.resize(B);
    int x_max = 0;
    for (int b = 0; b < B; ++b) {
        const Inst *P = &problems[b];
        {
            long long counted = 0;
            for (int c = 0; c < P->n_colours && c < kMaxColours; ++c) counted += P->class_n[c];
            if (counted == P->n && P->n > 0) pl.classes[b].assign(P->class_n, P->class_n + P->n_colours);
        }
        if (reads[b] < 0) return set_err(c, SPV_EINVAL, "reads[%d]=%d", b, reads[b]);
        if (reads[b] > 0 && (!energies[b] || (P->n > 0 && !spins[b])))
            return set_err(c, SPV_EINVAL, "instance %d: NULL output", b);
        if (b > 0 && P->scale_log2 != problems[0].scale_log2)
            return set_err(c, SPV_EINVAL, "instance %d: scale_log2 differs within the batch", b);
        BatchInst &in = pl.insts[b];
        std::memset(&in, 0, sizeof in);
        in.row_ptr = P->row_ptr;
        in.col = P->col;
        in.J = P->J;
        in.h = P->h;
        in.colour = P->colour;
        in.out = spins[b];
        in.energies = energies[b];
        in.seed = seeds[b];
        in.n = P->n;
        in.nnz = P->nnz;
        in.D = std::max(1, P->max_degree);
        in.C = P->n_colours;
        in.reads = reads[b];
        in.image_off = pl.image_words;
        pl.image_words += ((long long)image_words(P->n, in.D) + 3) & ~3ll;
        pl.n_max = std::max(pl.n_max, P->n);
        pl.D_max = std::max(pl.D_max, in.D);
        pl.total_quads += (reads[b] + 3) / 4;
        x_max = std::max(x_max, P->x_bound);
    }
    pl.scale = problems[0].scale_log2;
    pl.nd = digits_for(x_max);
    if (pl.nd > 3) return set_err(c, SPV_ERANGE, "x_bound=%d needs %d digits (max 3)", x_max, pl.nd);
    pl.row_len = table_row_len(x_max);
    // The byte-parallel body has straight-line variants for 4, 6 and 8 records per
    // site: pad every image of the batch to the largest degree (zero-coupling records).
    if (sa_use_swar(pl.nd, pl.row_len) && (pl.D_max == 4 || pl.D_max == 6 || pl.D_max == 8)) {
        pl.dk = pl.D_max;
        pl.image_words = 0;
        for (int b = 0; b < B; ++b) {
            BatchInst &in = pl.insts[b];
            in.D = pl.D_max;
            in.image_off = pl.image_words;
            pl.image_words += ((long long)image_words(in.n, in.D) + 3) & ~3ll;
        }
    }
    if (sweeps > 0 && (st = upload_tables(c, c->tables, betas, sweeps, 2, pl.scale, pl.nd, pl.row_len, stream)))
        return st;
    if (!c->batch_done && hipEventCreateWithFlags(&c->batch_done, hipEventDisableTiming) != hipSuccess)
        return set_err(c, SPV_EDEVICE, "event create");

    // Shape: explicit, tuned, or default.  The paired body serves batches whose images
    // have 4, 6 or 8 records per site on the byte-parallel path.
    const uint32_t flags = opts ? opts->flags : 0u;
    const bool paired_ok = pl.dk == 4 || pl.dk == 6 || pl.dk == 8;
    const size_t lds_cu = c->lds_max;  // LDS of one CU (the largest workgroup allocation)
    Shape sh{256, 2, 4};
    if (paired_ok) sh = Shape{1024, 2, 1, true};
    const std::vector<long long> tkey = {pl.n_max, pl.D_max, pl.nd, B, pl.total_quads / 64};
    bool have = false;
    if (opts && opts->threads > 0 && (flags & SPV_BATCH_PAIRED)) {
        if (!paired_ok)
            return set_err(c, SPV_EINVAL, "the paired body needs byte-parallel images of 4, 6 or 8 records per site");
        sh = Shape{opts->threads, 2, opts->wgs_per_cu > 0 ? opts->wgs_per_cu : 1, true};
        have = true;
    } else if (opts && opts->threads > 0 && opts->quads_per_item > 0) {
        sh = Shape{opts->threads, opts->quads_per_item, opts->wgs_per_cu > 0 ? opts->wgs_per_cu : 4, false};
        have = true;
    }
    if (!have)
        for (auto &t : c->tuned)
            if (t.key == tkey) {
                sh = Shape{t.threads, t.qw, t.wgs_per_cu, t.paired};
                have = true;
            }
    // Items, layout and (paired body) per-instance copies of a shape.
    PairPlan pp;
    auto items_of = [&](const Shape &x, std::vector<int32_t> *items) -> bool {
        if (x.paired) {
            if (!make_pair_items(pl, x.threads, lds_cu / (size_t)x.wgs_per_cu, &pp)) return false;
            *items = pp.items;
            return true;
        }
        if (batch_lds_bytes(pl.n_max, pl.D_max, pl.row_len, x.qw, pl.nd) + 512 > c->lds_max) return false;
        *items = make_items(pl, x.qw, x.threads);
        return true;
    };
    float tuned_ms = -1.f;
    if (!have && (flags & SPV_BATCH_TUNE)) {
        static const Shape cand[] = {{64, 2, 16},        {128, 2, 8},         {128, 4, 8},         {256, 1, 4},
                                     {256, 2, 4},        {512, 1, 2},         {512, 2, 2},         {512, 4, 2},
                                     {1024, 2, 1},       {1024, 4, 1},        {1024, 8, 1},        {1024, 2, 1, true},
                                     {512, 2, 2, true},  {512, 2, 1, true},   {256, 2, 4, true},   {256, 2, 2, true}};
        const int tsweeps = std::min(sweeps, 24);
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            return set_err(c, SPV_EDEVICE, "event create");
        float best = 1e30f;
        Shape bs = sh;
        for (const Shape &cs : cand) {
            if (cs.paired && !paired_ok) continue;
            std::vector<int32_t> items;
            if (!items_of(cs, &items)) continue;
            const Layout ly = layout_for(pl, items.size() / 3);
            if ((st = ensure_batch_buf(c, ly.total)) || (st = stage(c, pl, items, ly))) break;
            (void)hipEventRecord(e0, stream);
            st = enqueue(c, pl, ly, items.size() / 3, cs, tsweeps, 0, stream, &pp);
            (void)hipEventRecord(e1, stream);
            (void)hipEventRecord(c->batch_done, stream);
            if (st) break;
            float ms = 0.f;
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = set_err(c, SPV_EDEVICE, "tuning timing");
                break;
            }
            if (ms < best) {
                best = ms;
                bs = cs;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st) return st;
        sh = bs;
        tuned_ms = best;
        c->tuned.push_back({tkey, sh.threads, sh.qw, sh.wgs_per_cu, best, sh.paired});
    }
    if (sh.threads < 64 || sh.threads > 1024 || sh.threads % 64 || sh.qw < 1 || sh.qw > sh.threads ||
        sh.wgs_per_cu < 1 || sh.wgs_per_cu > 32)
        return set_err(c, SPV_EINVAL, "batch shape threads=%d quads_per_item=%d wgs_per_cu=%d", sh.threads,
                       sh.qw, sh.wgs_per_cu);
    std::vector<int32_t> items;
    if (!items_of(sh, &items)) {
        if (!sh.paired || have)
            return set_err(c, SPV_ECAPACITY, "largest instance (n=%d) needs more LDS than a workgroup has", pl.n_max);
        sh = Shape{256, 2, 4, false};  // default paired shape does not fit: the one-word body
        if (!items_of(sh, &items))
            return set_err(c, SPV_ECAPACITY, "largest instance (n=%d) needs more LDS than a workgroup has", pl.n_max);
    }
    c->last_shape[0] = sh.threads;
    c->last_shape[1] = sh.paired ? 0 : sh.qw;
    c->last_shape[2] = sh.wgs_per_cu;
    c->last_tuned_ms = tuned_ms;

    const size_t n_items = items.size() / 3;
    const Layout ly = layout_for(pl, n_items);
    if ((st = ensure_batch_buf(c, ly.total))) return st;
    if ((st = stage(c, pl, items, ly))) return st;
    if (n_items == 0) return SPV_OK;
    if (flags & SPV_BATCH_GRAPH) {
        const std::vector<long long> key = {B, (long long)n_items, pl.n_max, pl.D_max, pl.nd, pl.row_len,
                                            sweeps, sh.threads, sh.qw, sh.wgs_per_cu, sh.paired ? 1 : 0,
                                            pp.pairs_qw, pp.kmax,
                                            (long long)(uintptr_t)c->batch.p,
                                            (long long)(uintptr_t)c->batch_host,
                                            (long long)(uintptr_t)c->tables.p, (long long)(uintptr_t)stream};
        hipGraphExec_t exec = nullptr;
        for (auto &ge : c->graphs)
            if (ge.key == key) exec = ge.exec;
        if (!exec) {
            // Capture on a private stream (the caller's may be the legacy default
            // stream, which cannot be captured); the graph is launched on the caller's.
            if (!c->capture_stream &&
                hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess)
                return set_err(c, SPV_EDEVICE, "capture stream create");
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_check(c, e, "begin capture");
            st = enqueue(c, pl, ly, n_items, sh, sweeps, 0, c->capture_stream, &pp);
            e = hipStreamEndCapture(c->capture_stream, &graph);
            if (st) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_check(c, e, "graph capture");
            c->graphs.push_back({key, exec, stream});
        }
        hipError_t e = hipGraphLaunch(exec, stream);
        if (e != hipSuccess) return hip_check(c, e, "graph launch");
    } else {
        if ((st = enqueue(c, pl, ly, n_items, sh, sweeps, 0, stream, &pp))) return st;
    }
    return hip_check(c, hipEventRecord(c->batch_done, stream), "event record");
}

}  // namespace spv

extern "C" {

spv_status spv_sample_batch(spv_ctx *ctx, int32_t B, const spv_problem *problems, const double *betas,
                            int32_t sweeps, const int32_t *reads, const uint64_t *seeds,
                            int8_t *const *spins, int64_t *const *energies, const spv_batch_opts *opts,
                            hipStream_t stream) {
    if (!ctx) return SPV_EINVAL;
    Ctx *c = &ctx->c;
    DeviceGuard g(c->device);
    if (B < 0 || B > 65535 || (B > 0 && !problems))
        return set_err(c, SPV_EINVAL, "B=%d (at most 65535) or NULL problems", B);
    std::vector<Inst> Q((size_t)B);
    const spv_status st = ingest(c, problems, B, kIngestColours, stream, Q.data());
    if (st) return st;
    return sample_batch_inst(ctx, B, Q.data(), betas, sweeps, reads, seeds, spins, energies, opts, stream);
}

spv_status spv_batch_last_shape(const spv_ctx *ctx, int32_t *threads, int32_t *quads_per_item,
                                int32_t *wgs_per_cu, float *tuned_ms) {
    if (!ctx) return SPV_EINVAL;
    if (threads) *threads = ctx->c.last_shape[0];
    if (quads_per_item) *quads_per_item = ctx->c.last_shape[1];
    if (wgs_per_cu) *wgs_per_cu = ctx->c.last_shape[2];
    if (tuned_ms) *tuned_ms = ctx->c.last_tuned_ms;
    return SPV_OK;
}

}  // extern "C"
