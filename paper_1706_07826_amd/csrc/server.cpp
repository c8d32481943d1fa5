// Serving loop: continuous batching of sample(+fix) requests over a pool of
// execution slots (stream + stream-private scratch context each), FIFO
// admission under LDS and HBM budgets, and a progress thread that retires
// finished requests and admits waiting ones as capacity frees up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum State { kPending, kRunning, kDone };

struct Record {
    spv_request req;
    spv::Inst inst;  // the request's problem as ingested at submission
    std::vector<double> betas, gammas;
    int64_t lds = 0, hbm = 0;
    State state = kPending;
    bool fix_pending = false;  // tempering request whose persistence step follows the sampling
    spv_result res{};
};

struct Slot {
    spv_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    uint64_t ticket = 0;
};

}  // namespace

struct spv_server {
    spv_ctx *parent = nullptr;
    int device = 0;
    int64_t lds_budget = 0, hbm_budget = 0, lds_used = 0, hbm_used = 0;
    std::vector<Slot> slots;
    std::unordered_map<uint64_t, Record> recs;
    std::deque<uint64_t> queue;
    uint64_t next_ticket = 1;
    std::mutex mu;
    std::condition_variable cv;
    std::atomic<bool> stop{false};
    std::thread worker;
    hipStream_t ingest_stream = nullptr;  // validation of submitted problems
    std::mutex ingest_mu;                 // one submission ingests at a time (parent scratch)
};

using namespace spv;

namespace {

// LDS and scratch a request claims while in flight (default launch shapes).
void footprint(spv_server *s, const spv_request &r, const Inst &P, int64_t *lds, int64_t *hbm) {
    const int D = std::max(1, P.max_degree);
    const int nd = digits_for(P.x_bound), row_len = table_row_len(P.x_bound);
    int64_t L = 0, H = (int64_t)image_words(std::max(P.n, 1), D) * 4;
    int64_t R = 0;
    if (r.kind == SPV_REQ_SA) {
        const int qw = sa_use_swar(nd, row_len) ? 2 : 1;
        const int64_t wgs = ((int64_t)(r.reads + 3) / 4 + qw - 1) / qw;
        L = wgs * (int64_t)sa_lds_bytes(P.n, D, row_len, qw);
        H += (int64_t)r.sweeps * row_len * 4;
        R = r.reads;
    } else if (r.kind == SPV_REQ_SQA) {
        // one workgroup per read; the rows are sized for the largest (three-digit) table
        const int rl = 3 * kDigitSize;
        const int Pq = std::max(r.trotter, 8);
        const size_t in_lds = sqa_lds_bytes(P.n, D, rl, Pq);
        L = (int64_t)r.reads * (int64_t)(in_lds + 256 <= (size_t)s->parent->c.lds_max
                                             ? in_lds : sqa_lds_bytes(P.n, D, rl, Pq, true));
        H += (int64_t)r.sweeps * (rl * 4 + 4);
        R = r.reads;
    } else {
        if (pt_lds_footprint(&s->parent->c, &P, r.K, r.runs, r.chains, r.icm_lo, r.icm_hi, &L) != SPV_OK)
            L = 0;  // the launch itself reports the error
        R = (int64_t)r.runs * r.chains * (r.K / 2) * kTopK;
        H += (int64_t)r.K * row_len * 4 + (int64_t)r.K * 7 * kDigitSize * 4 + R * std::max(P.n, 1);
        // boundary messages: at most K / 4 groups per run, or K with cluster moves on
        const int64_t gmax = r.icm_hi > r.icm_lo ? r.K : r.K / 4;
        H += (int64_t)r.runs * gmax * 4 * r.chains * (int64_t)ptx_msg_words(std::max(P.n, 1)) * 4;
        if (r.elite_frac > 0) H += R * (std::max(P.n, 1) + 8);  // assembled sample
    }
    if (r.elite_frac > 0 && R > 0) {
        const int m = std::max(1, std::min((int)std::ceil(r.elite_frac * (double)R), (int)R));
        H += (int64_t)fix_scratch_bytes(P.n, (int)R, m);
    }
    *lds = L;
    *hbm = H;
}

spv_status launch(Slot &sl, Record &rec) {
    spv_ctx *x = sl.ctx;
    const spv_request &r = rec.req;
    spv_status st;
    if (r.kind == SPV_REQ_SA || r.kind == SPV_REQ_SQA) {
        st = r.kind == SPV_REQ_SA
                 ? sample_inst(x, &rec.inst, rec.betas.data(), r.sweeps, r.reads, r.seed, 0, nullptr, r.spins,
                               r.energies, sl.stream)
                 : sqa_inst(x, &rec.inst, rec.betas.data(), rec.gammas.data(), r.sweeps, r.trotter, r.reads,
                            r.seed, r.spins, r.energies, sl.stream);
        if (st == SPV_OK && r.elite_frac > 0)
            st = spv_persist_fix(x, &r.problem, r.spins, r.energies, r.reads, r.elite_frac, r.threshold,
                                 r.gauge, &r.fix_out, sl.stream);
    } else {
        spv_pt_params prm{};  // no checkpoint: serving runs start fresh
        prm.K = r.K;
        prm.runs = r.runs;
        prm.chains = r.chains;
        prm.sweeps = r.sweeps;
        prm.betas = rec.betas.data();
        prm.seed = r.seed;
        prm.sweep_offset = 0;
        prm.icm_lo = r.icm_lo;
        prm.icm_hi = r.icm_hi;
        st = pt_inst(x, &rec.inst, &prm, &r.pt_out, sl.stream);
        // The sample size (filled top-10 entries) is known once the run ends.
        rec.fix_pending = st == SPV_OK && r.elite_frac > 0;
    }
    if (st == SPV_OK) st = hipEventRecord(sl.done, sl.stream) == hipSuccess ? SPV_OK : SPV_EDEVICE;
    return st;
}

// Second phase of a tempering request with persistence: assemble the top-10
// sample in the slot's scratch, then fix and reduce.
spv_status launch_fix(Slot &sl, Record &rec) {
    spv_ctx *x = sl.ctx;
    Ctx *c = &x->c;
    const spv_request &r = rec.req;
    const int n = r.problem.n;
    const int lists = r.runs * r.chains * (r.K / 2);
    const size_t cap = (size_t)lists * kTopK;
    spv_status st = ensure(c, c->serve, cap * (size_t)n + cap * 8 + 256);
    if (st) return st;
    int64_t *E = static_cast<int64_t *>(c->serve.p);
    int8_t *S = reinterpret_cast<int8_t *>(E + cap);
    int32_t rows = 0;
    st = spv_top_sample(x, r.pt_out.top_spins, r.pt_out.top_E, r.pt_out.top_count, lists, n, S, E, &rows,
                        sl.stream);
    if (st == SPV_OK)
        st = spv_persist_fix(x, &r.problem, S, E, rows, r.elite_frac, r.threshold, r.gauge, &r.fix_out,
                             sl.stream);
    if (st == SPV_OK) st = hipEventRecord(sl.done, sl.stream) == hipSuccess ? SPV_OK : SPV_EDEVICE;
    return st;
}

// Retire finished slots, then admit from the head of the queue while it fits.
// Called with the lock held.
void progress_locked(spv_server *s) {
    for (size_t k = 0; k < s->slots.size(); ++k) {
        Slot &sl = s->slots[k];
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        Record &rec = s->recs[sl.ticket];
        if (q == hipSuccess && rec.fix_pending) {
            rec.fix_pending = false;
            DeviceGuard g(s->device);
            const spv_status st = launch_fix(sl, rec);
            if (st == SPV_OK) continue;
            rec.res.status = st;
        }
        if (q == hipSuccess && rec.res.status == SPV_OK && rec.req.elite_frac > 0 && rec.req.fix_out.info) {
            // The persistence step's device status (info[7]) becomes the request's status.
            int64_t dev_status = 0;
            DeviceGuard g(s->device);
            hipError_t e = hipMemcpyAsync(&dev_status, rec.req.fix_out.info + 7, sizeof dev_status,
                                          hipMemcpyDeviceToHost, sl.stream);
            if (e == hipSuccess) e = hipStreamSynchronize(sl.stream);
            if (e != hipSuccess) rec.res.status = SPV_EDEVICE;
            else if (dev_status != 0) rec.res.status = (spv_status)dev_status;
        }
        rec.res.done_ns = now_ns();
        if (q != hipSuccess && rec.res.status == SPV_OK) rec.res.status = SPV_EDEVICE;
        rec.state = kDone;
        s->lds_used -= rec.lds;
        s->hbm_used -= rec.hbm;
        sl.busy = false;
        s->cv.notify_all();
    }
    while (!s->queue.empty()) {
        const uint64_t t = s->queue.front();
        Record &rec = s->recs[t];
        if (s->lds_used + rec.lds > s->lds_budget) break;
        if (s->hbm_budget > 0 && s->hbm_used + rec.hbm > s->hbm_budget) break;
        int free_slot = -1;
        for (size_t k = 0; k < s->slots.size(); ++k)
            if (!s->slots[k].busy) {
                free_slot = (int)k;
                break;
            }
        if (free_slot < 0) break;
        s->queue.pop_front();
        Slot &sl = s->slots[free_slot];
        DeviceGuard g(s->device);
        rec.res.start_ns = now_ns();
        rec.res.slot = free_slot;
        rec.state = kRunning;
        const spv_status st = launch(sl, rec);
        if (st != SPV_OK) {
            rec.res.status = st;
            rec.res.done_ns = now_ns();
            rec.state = kDone;
            s->cv.notify_all();
            continue;
        }
        sl.busy = true;
        sl.ticket = t;
        s->lds_used += rec.lds;
        s->hbm_used += rec.hbm;
    }
}

void worker_loop(spv_server *s) {
    DeviceGuard g(s->device);
    while (!s->stop.load()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            progress_locked(s);
        }
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace

extern "C" {

spv_status spv_server_create(spv_ctx *ctx, const spv_server_cfg *cfg, spv_server **out) {
    if (!ctx || !out) return SPV_EINVAL;
    *out = nullptr;
    Ctx *c = &ctx->c;
    const int nslots = cfg && cfg->slots > 0 ? cfg->slots : 8;
    if (nslots > 64) return set_err(c, SPV_EINVAL, "slots=%d > 64", nslots);
    spv_server *s = new (std::nothrow) spv_server();
    if (!s) return SPV_ENOMEM;
    s->parent = ctx;
    s->device = c->device;
    s->lds_budget = cfg && cfg->lds_budget > 0 ? cfg->lds_budget : (int64_t)c->num_cus * 160 * 1024;
    s->hbm_budget = cfg && cfg->hbm_budget > 0 ? cfg->hbm_budget : 0;
    DeviceGuard g(c->device);
    s->slots.resize(nslots);
    for (auto &sl : s->slots) {
        spv_status st = spv_ctx_create(c->device, &sl.ctx);
        if (st == SPV_OK && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess)
            st = SPV_EDEVICE;
        if (st == SPV_OK && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
            st = SPV_EDEVICE;
        if (st != SPV_OK) {
            spv_server_destroy(s);
            return set_err(c, st, "server slot creation failed");
        }
        sl.ctx->c.stream_private = true;
        sl.ctx->c.own_stream = sl.stream;
    }
    if (hipStreamCreateWithFlags(&s->ingest_stream, hipStreamNonBlocking) != hipSuccess) {
        spv_server_destroy(s);
        return set_err(c, SPV_EDEVICE, "server stream creation failed");
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return SPV_OK;
}

spv_status spv_server_submit(spv_server *s, const spv_request *req, uint64_t *ticket) {
    if (!s || !req || !ticket) return SPV_EINVAL;
    Ctx *c = &s->parent->c;
    const spv_request &r = *req;
    if (r.kind != SPV_REQ_SA && r.kind != SPV_REQ_PT && r.kind != SPV_REQ_SQA)
        return set_err(c, SPV_EINVAL, "request kind %d", r.kind);
    const bool sampled = r.kind == SPV_REQ_SA || r.kind == SPV_REQ_SQA;
    const int nb = sampled ? r.sweeps : r.K;
    if (nb < 0 || (nb > 0 && !r.betas)) return set_err(c, SPV_EINVAL, "request betas");
    if (r.kind == SPV_REQ_SQA && (r.trotter < 8 || r.trotter > 256 || r.trotter % 8 != 0 || (nb > 0 && !r.gammas)))
        return set_err(c, SPV_EINVAL, "SQA request: trotter=%d or NULL gammas", r.trotter);
    if (sampled && (r.reads < 1 || !r.energies || (r.problem.n > 0 && !r.spins)))
        return set_err(c, SPV_EINVAL, "SA request outputs");
    if (r.kind == SPV_REQ_PT && r.elite_frac > 0 && (!r.pt_out.top_spins || !r.pt_out.top_E || !r.pt_out.top_count))
        return set_err(c, SPV_EINVAL, "PT request with persistence needs top_spins, top_E and top_count");
    Record rec;
    rec.req = r;
    rec.betas.assign(r.betas, r.betas + std::max(nb, 0));
    rec.req.betas = nullptr;
    if (r.kind == SPV_REQ_SQA) rec.gammas.assign(r.gammas, r.gammas + std::max(nb, 0));
    rec.req.gammas = nullptr;
    {
        // Validate the problem and derive its bounds once, on the server's own stream
        // (the problem arrays must be ready when the request is submitted).
        std::lock_guard<std::mutex> ilk(s->ingest_mu);
        const spv_status st = ingest(c, &r.problem, 1, kIngestColours, s->ingest_stream, &rec.inst);
        if (st) return st;
    }
    footprint(s, r, rec.inst, &rec.lds, &rec.hbm);
    rec.res.lds_bytes = rec.lds;
    rec.res.hbm_bytes = rec.hbm;
    if (rec.lds > s->lds_budget || (s->hbm_budget > 0 && rec.hbm > s->hbm_budget))
        return set_err(c, SPV_EBUDGET, "request needs %lld B LDS / %lld B scratch, budgets %lld / %lld",
                       (long long)rec.lds, (long long)rec.hbm, (long long)s->lds_budget,
                       (long long)s->hbm_budget);
    rec.res.status = SPV_OK;
    rec.res.submit_ns = now_ns();
    rec.res.slot = -1;
    std::lock_guard<std::mutex> lk(s->mu);
    const uint64_t t = s->next_ticket++;
    s->recs.emplace(t, std::move(rec));
    s->queue.push_back(t);
    progress_locked(s);
    *ticket = t;
    return SPV_OK;
}

spv_status spv_server_poll(spv_server *s, uint64_t ticket, spv_result *res) {
    if (!s || !res) return SPV_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->recs.find(ticket);
    if (it == s->recs.end()) return SPV_EINVAL;
    if (it->second.state != kDone) return SPV_EAGAIN;
    *res = it->second.res;
    return SPV_OK;
}

spv_status spv_server_wait(spv_server *s, uint64_t ticket, spv_result *res) {
    if (!s || !res) return SPV_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->recs.find(ticket);
    if (it == s->recs.end()) return SPV_EINVAL;
    s->cv.wait(lk, [&] { return it->second.state == kDone; });
    *res = it->second.res;
    return SPV_OK;
}

spv_status spv_server_drain(spv_server *s) {
    if (!s) return SPV_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] {
        if (!s->queue.empty()) return false;
        for (auto &sl : s->slots)
            if (sl.busy) return false;
        return true;
    });
    return SPV_OK;
}

void spv_server_destroy(spv_server *s) {
    if (!s) return;
    if (s->worker.joinable()) {
        (void)spv_server_drain(s);
        s->stop.store(true);
        s->worker.join();
    }
    DeviceGuard g(s->device);
    for (auto &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.ctx) spv_ctx_destroy(sl.ctx);
    }
    if (s->ingest_stream) (void)hipStreamDestroy(s->ingest_stream);
    delete s;
}

}  // extern "C"
