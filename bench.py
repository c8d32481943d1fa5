#!/usr/bin/env python3
"""Throughput benchmark of the sample-persistence hot path on one MI355X.

Default (headline): one JSON line carrying the metric's three clauses.
  * value: spin-updates/s of the residual batch -- 512 residual-shaped instances
    (n log-uniform 50..1000), 1000 reads x 1000 sweeps each, in one persistent,
    graph-replayed launch per step -- beside the plain path (one spv_sample
    launch per instance), their ratio and whether the outputs are bit-identical.
  * spvar_solves: SPVAR solves/s on the Chimera 8x8 instance (N = 512): one solve
    = spv_sample (SA, 10,000 reads x 2,000 sweeps) + spv_persist_fix.
  * serving: p50/p99 latency of a mixed request stream (SA N=512, PT N=1000,
    PT-ICM N=8000, each + persistence) at Poisson arrivals of 0.8 x saturation.
Inputs are resident in device memory before timing starts.  Each part carries
the roofline object of its dominant kernel (timed with HIP events on the stream
it runs on) and a cpu_baseline: the CPU oracle on a bounded sample of the same
workload.  --workload selects a single workload's own line instead.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC_NAME = "spin-updates/s (batched vs plain, bit-exact); SPVAR solves/s; p50/p99 latency"

# VALU lane-slots per Metropolis update (algorithmic count, the roofline's
# numerator).  A Philox4x32-10 block is 10 rounds of two 32x32->64 products
# (v_mad_u64_u32) and two 3-input xors (v_bitop3_b32): 40 instructions.  Its cost
# in issue slots is measured on the device by spv_philox_probe in every run
# (about 42 on gfx950: the products issue at full rate); one block serves the 4
# replicas of a word.  The byte-parallel path (every |J|, |h| small enough for
# one-byte lanes) then adds, per neighbour, one AND and one ADD on a word of 4
# replicas (2/4 slot per update) and about 4 slots per update for the field
# assembly, sign test, threshold compare and flip; the general path adds one
# multiply-add per neighbour and replica (1 slot) and the same 4.
PHILOX_INSTRUCTIONS = 10 * (2 + 2)
PEAK_VALU_TSLOTS = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 64 lanes x 2.4 GHz = 39.32 T lane-slots/s
SA_PROFILE_SOURCES = ["paper_1706_07826_amd/csrc/sa.hip", "paper_1706_07826_amd/csrc/swar_core.hpp",
                      "paper_1706_07826_amd/csrc/sa_core.hpp", "paper_1706_07826_amd/csrc/device.hpp"]


def sa_lds_bytes_per_update(D, words_per_lane):
    """LDS bytes a byte-parallel SA update moves (read + flip write), from its access
    pattern: per lane and site visit, the D neighbour records (8 B each), the neighbour
    spin words, the lane's own words, the site constants (8 B), one threshold word per
    replica (4 B) and the flipped words with their complements; W quad words per lane."""
    W = words_per_lane
    per_visit = 8 * D + 4 * W * D + 4 * W + 8 + 16 * W + 8 * W
    return per_visit / (4.0 * W)


def pt_lds_bytes_per_update(D, digits, records_in_lds):
    """LDS bytes a tempering Metropolis update moves: per quad task the own word, the D
    neighbour words, one threshold word per replica and digit, the flip write, and the
    D records when the instance is LDS-resident."""
    per_task = 4 + 4 * D + 16 * digits + 4 + (4 * D if records_in_lds else 0)
    return per_task / 4.0


def lds_object(updates_per_s, bytes_per_update, probe_bytes_per_s, note):
    achieved = updates_per_s * bytes_per_update
    return {"bytes_per_update": round(bytes_per_update, 2), "achieved_TBps": round(achieved / 1e12, 3),
            "probe_peak_TBps": round(probe_bytes_per_s / 1e12, 3),
            "frac": round(achieved / probe_bytes_per_s, 4), "note": note}


def slots_per_update(mean_degree, byte_parallel, philox_slots):
    per_neighbour = 0.5 if byte_parallel else 1.0
    return mean_degree * per_neighbour + 4 + philox_slots / 4.0


def sources_digest(paths):
    """sha256 over the concatenated bytes of the given repo-relative files."""
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_traffic_bytes(kernel, workload="chimera8_sa"):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter summary
    profiles/<kernel>_<workload>.json (FETCH_SIZE and WRITE_SIZE scaled by a copy of known
    size), or None when the summary covers another kernel or any of the kernel's sources
    changed after the counters were taken."""
    base = kernel.split("<")[0]
    try:
        with open(os.path.join(ROOT, "profiles", f"{base}_{workload}.json")) as f:
            prof = json.load(f)
        digest = sources_digest(prof["sources"])
    except (OSError, KeyError, ValueError):
        return None
    if prof.get("kernel") != kernel or not digest.startswith(prof["sources_sha256_prefix"]):
        return None
    kib = prof["fetch_kib"] * prof["fetch_scale"] + prof["write_kib"] * prof["write_scale"]
    return int(round(kib * 1024))


def pt_slots_per_update(mean_degree, digits, philox_slots):
    """VALU lane-slots per tempering Metropolis update (general body): one Philox block per
    quad and digit tested, one multiply-add per neighbour, about 4 for the field, sign,
    threshold compares and flip."""
    return digits * philox_slots / 4.0 + mean_degree + 4


def cpu_threads():
    return max(1, min(16, os.cpu_count() or 1))


_PROBES = {}


def measured_philox_slots(spv, ctx):
    """Issue slots one Philox block costs at full occupancy (spv_philox_probe): the median of
    five probe runs, measured once per process and shared by every roofline of the line."""
    if "philox" not in _PROBES:
        runs = sorted(PEAK_VALU_TSLOTS * 1e12 / spv.spv_philox_probe(ctx) for _ in range(5))
        _PROBES["philox"] = runs[2]
    return _PROBES["philox"]


def measured_lds_peak(spv, ctx):
    """The device's LDS read bandwidth (spv_lds_probe), best of two runs, once per process."""
    if "lds" not in _PROBES:
        _PROBES["lds"] = max(spv.spv_lds_probe(ctx) for _ in range(2))
    return _PROBES["lds"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reads", type=int, default=0, help="oracle reads (0 = 640 per thread, at most all)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, run one device copy of this size (counter calibration)")
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "chimera8_sa", "residual_batch", "cubic10_pt", "cubic20_pticm", "serving",
                             "spvar_round", "multistart", "spvar_tree", "cubic4_ispvar", "chimera32_sa",
                             "chimera8_sqa", "multistart_sqa"])
    ap.add_argument("--pt-runs", type=int, default=0, help="PT workloads: runs per step (0 = the config's)")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="serving workload: requests per load level (the headline uses 400 / 800)")
    ap.add_argument("--serving-slots", type=int, default=16)
    ap.add_argument("--hw-queues", type=int, default=-1,
                    help="GPU_MAX_HW_QUEUES for this process (-1: 32 for serving, unchanged otherwise)")
    args = ap.parse_args()
    hwq = args.hw_queues if args.hw_queues >= 0 else (32 if args.workload in ("serving", "headline") else 0)
    if hwq:
        # HIP reads it when the runtime starts: one hardware queue per serving slot keeps
        # a long request's kernel from blocking the slots that share its queue.
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(hwq, 32))
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (single-GPU build)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1706_07826_amd as spv
    from spvar_inputs import configs as cf

    if args.workload == "residual_batch":
        return bench_residual_batch(args)
    if args.workload == "cubic10_pt":
        return bench_pt(args, cf.CUBIC10_PT, "cubic10_pt: PT 32 betas 0.2..5.0, {runs} runs x 10^4 sweeps, "
                        "top-10 sample of the 16 colder slots, persistence elite 0.2")
    if args.workload == "cubic20_pticm":
        return bench_pt(args, cf.CUBIC20_PTICM, "cubic20_pticm: N=8000, PT-ICM 40 betas 0.2..5.0 x 2 chains, "
                        "Houdayer moves at every slot, {runs} run(s) x 10^4 sweeps, top-10 sample of the 20 "
                        "colder slots per chain, persistence elite 0.2")
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "spvar_round":
        return bench_spvar_round(args)
    if args.workload == "multistart":
        return bench_multistart(args)
    if args.workload == "multistart_sqa":
        return bench_multistart(args, sqa=True)
    if args.workload == "spvar_tree":
        return bench_spvar_tree(args)
    if args.workload == "cubic4_ispvar":
        return bench_cubic4_ispvar(args)
    if args.workload == "chimera32_sa":
        return bench_chimera32_sa(args)
    if args.workload == "chimera8_sqa":
        return bench_chimera8_sqa(args)

    if args.workload == "headline":
        return bench_headline(args)
    print(json.dumps(part_chimera8_sa(args)), flush=True)


def part_chimera8_sa(args, line=True):
    """Config 2: one step = spv_sample (SA, 10,000 reads x 2,000 sweeps, Chimera 8x8, N=512) +
    spv_persist_fix (elite 5 %, threshold 0.95).  Returns the bench line (line=True) or the
    block the headline line carries."""
    import numpy as np
    import torch

    import paper_1706_07826_amd as spv
    from spvar_inputs import configs as cf

    cfg = cf.CHIMERA8_SA
    inst = cf.instance(cfg)
    betas = cf.betas(cfg)
    reads, sweeps, n = cfg["reads"], cfg["sweeps"], inst.n
    updates = reads * n * sweeps

    ctx = spv.Context(0)
    P = spv.Problem.from_instance(inst)
    spv.spv_problem_check(ctx, P)
    stream = torch.cuda.current_stream()
    spins = torch.empty((reads, n), dtype=torch.int8, device="cuda")
    energies = torch.empty(reads, dtype=torch.int64, device="cuda")

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        spv.spv_sample(ctx, P, betas, reads, cfg["seed"], spins=spins, energies=energies)
        if ev is not None:
            ev[1].record(stream)
        return spv.spv_persist_fix(ctx, P, spins, energies, cfg["elite"], cfg["theta"], cfg["gauge"])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for k in range(args.steps):
        last = step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = last.info()
    ms_step = wall * 1e3 / args.steps
    sa_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    value = updates / (ms_step / 1e3)

    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()

    mean_deg = inst.nnz / inst.n
    max_degree, x_bound = spv.spv_problem_check(ctx, P)  # the bounds the library derives at ingest
    byte_parallel = x_bound <= 255  # the library's rule for its byte-parallel body
    philox_slots = measured_philox_slots(spv, ctx)  # measured issue slots per block
    spu = slots_per_update(mean_deg, byte_parallel, philox_slots)
    achieved = updates * spu / (sa_ms / 1e3) / 1e12
    shape = spv.spv_sample_last_shape(ctx)
    dk = max_degree if max_degree in (4, 6, 8) else 0
    if not byte_parallel:
        kernel = "sa_kernel<1>"
    elif shape["chunks"] > 1:
        big = "true" if shape["global_instance"] else "false"
        kernel = f"sa_stream_kernel<{dk}, {shape['words_per_lane']}, {big}>"
    else:
        kernel = f"sa_kernel<0, {dk}, {'true' if shape['global_instance'] else 'false'}>"
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TSLOTS, 3),
                "unit": "Tslot/s", "frac": round(achieved / PEAK_VALU_TSLOTS, 4),
                "traffic": profiled_traffic_bytes(kernel),
                "kernel": kernel, "kernel_ms": round(sa_ms, 4), "launch": shape,
                "slots_per_update": round(spu, 3)}
    roofline["philox_slots"] = round(philox_slots, 2)  # measured: spv_philox_probe
    roofline["philox_instructions"] = PHILOX_INSTRUCTIONS
    if byte_parallel:
        probe = measured_lds_peak(spv, ctx)
        roofline["lds"] = lds_object(updates / (sa_ms / 1e3),
                                     sa_lds_bytes_per_update(max_degree, shape["words_per_lane"]), probe,
                                     "competing bound: LDS traffic of the sweep against the measured LDS peak")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = max(1, min(16, os.cpu_count() or 1))
        cpu_reads = args.cpu_reads or min(reads, 640 * threads)
        t1 = time.perf_counter()
        oracle.sa_sample(inst, betas, seed=cfg["seed"], r_begin=0, r_end=cpu_reads, threads=threads)
        dt = time.perf_counter() - t1
        cpu = {"value": round(cpu_reads * n * sweeps / dt, 1), "unit": "spin-updates/s",
               "cores": threads, "kind": "oracle",
               "sample": f"reads 0..{cpu_reads - 1} of {reads} (all {sweeps} sweeps), "
                         f"{threads} threads, {dt:.1f} s wall"}

    out = {
        "metric": METRIC_NAME, "value": round(value, 1), "unit": "spin-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded Chimera U{+-1..+-6} instance; no paper instances available)",
        "config": {"workload": "chimera8_sa: Chimera 8x8 K4,4, N=512, couplers/biases "
                               "U{+-1..+-6}; SA 10000 reads x 2000 sweeps, beta 0.1->5.0; "
                               "persistence elite 0.05, threshold 0.95",
                   "reads": reads, "sweeps": sweeps, "n": n, "parallelism": "single GPU"},
        "spvar_solves_per_s": round(1e3 / ms_step, 3),
        "fixed_per_solve": info["n_fixed"],
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if line:
        return out
    return {"workload": out["config"]["workload"], "spvar_solves_per_s": out["spvar_solves_per_s"],
            "spin_updates_per_s": out["value"], "ms_per_step": out["ms_per_step"],
            "fixed_per_solve": out["fixed_per_solve"], "roofline": roofline, "cpu_baseline": cpu}


def bench_residual_batch(args):
    print(json.dumps(part_residual_batch(args)), flush=True)


def part_residual_batch(args):
    """Residual batch: 512 instances (n log-uniform 50..1000), 1000 reads x 1000 sweeps
    each.  Batched persistent launch (graph-replayed, autotuned shape) vs the plain path
    (one spv_sample launch per instance, default shape), outputs compared bit for bit."""
    import numpy as np
    import torch

    import paper_1706_07826_amd as spv
    from spvar_inputs import configs as cf

    cfg = cf.RESIDUAL_BATCH
    insts = cf.instance(cfg)
    betas = cf.betas(cfg)
    ctx = spv.Context(0)
    probs = [spv.Problem.from_instance(i) for i in insts]
    reads = [cfg["reads"]] * len(insts)
    seeds = [cfg["seed"] + b for b in range(len(insts))]
    updates = sum(i.n for i in insts) * cfg["reads"] * cfg["sweeps"]
    sp, en = spv.spv_sample_batch(ctx, probs, betas, reads, seeds, tune=True, graph=True)
    torch.cuda.synchronize()
    shape = spv.spv_batch_last_shape(ctx)
    for _ in range(args.warmup):
        spv.spv_sample_batch(ctx, probs, betas, reads, seeds, spins=sp, energies=en, graph=True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        # the replayed graph on this stream: descriptor copy, image prep, batch_sa_kernel
        events[k][0].record(stream)
        spv.spv_sample_batch(ctx, probs, betas, reads, seeds, spins=sp, energies=en, graph=True)
        events[k][1].record(stream)
    torch.cuda.synchronize()
    batched_s = (time.perf_counter() - t0) / args.steps
    graph_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    psp = [torch.empty_like(t) for t in sp]
    pen = [torch.empty_like(t) for t in en]
    for b, P in enumerate(probs):  # warm-up of the plain path
        spv.spv_sample(ctx, P, betas, reads[b], seeds[b], spins=psp[b], energies=pen[b])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, P in enumerate(probs):
        spv.spv_sample(ctx, P, betas, reads[b], seeds[b], spins=psp[b], energies=pen[b])
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    same = all(torch.equal(a, b) for a, b in zip(sp + en, psp + pen))
    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    # VALU roofline of the batched kernel: the byte-parallel body's algorithmic slots per update
    # at the batch's mean degree, over the replayed graph's duration (HIP events on its stream)
    bounds = [spv.spv_problem_check(ctx, P) for P in probs]
    byte_parallel = max(xb for _, xb in bounds) <= 255
    mean_deg = sum(i.nnz for i in insts) / sum(i.n for i in insts)
    philox_slots = measured_philox_slots(spv, ctx)
    spu = slots_per_update(mean_deg, byte_parallel, philox_slots)
    achieved = updates * spu / (graph_ms / 1e3) / 1e12
    dk = max(md for md, _ in bounds)
    if not byte_parallel:
        kernel = "batch_sa_kernel<1>"
    elif dk in (4, 6, 8):
        # quads_per_item 0: the paired body (a lane holds both words of a pair of quads)
        kernel = f"batch_sa_paired_kernel<{dk}>" if shape["quads_per_item"] == 0 else f"batch_sa_kernel<0, {dk}>"
    else:
        kernel = "batch_sa_kernel<0>"
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TSLOTS, 3),
                "unit": "Tslot/s", "frac": round(achieved / PEAK_VALU_TSLOTS, 4),
                "traffic": profiled_traffic_bytes(kernel, "residual_batch"), "kernel": kernel,
                "kernel_ms": round(graph_ms, 4), "slots_per_update": round(spu, 3),
                "philox_slots": round(philox_slots, 2), "mean_degree": round(mean_deg, 3),
                "note": "kernel_ms spans the replayed graph (descriptor copy + image prep + the batched "
                        "kernel), so it bounds the kernel's own duration from above"}
    if shape["quads_per_item"] == 0:
        roofline["traffic"] = profiled_traffic_bytes(kernel, "residual_batch")
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on the first 16 reads of every instance (all sweeps), instances spread
        # over the host threads
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        threads = cpu_threads()
        r_cpu = min(16, cfg["reads"])
        t1 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda b: oracle.sa_sample(insts[b], betas, seed=seeds[b], r_begin=0, r_end=r_cpu,
                                                  threads=1), range(len(insts))))
        cdt = time.perf_counter() - t1
        cu = sum(i.n for i in insts) * r_cpu * cfg["sweeps"]
        cpu = {"value": round(cu / cdt, 1), "unit": "spin-updates/s", "cores": threads, "kind": "oracle",
               "sample": f"reads 0..{r_cpu - 1} of every one of the {len(insts)} instances (all {cfg['sweeps']} "
                         f"sweeps), {threads} threads, {cdt:.1f} s wall"}
    out = {
        "metric": METRIC_NAME, "value": round(updates / batched_s, 1), "unit": "spin-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(batched_s * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic residual-shaped instances",
        "config": {"workload": "residual_batch: 512 BFS-ball residuals of a Chimera 16x16 parent, "
                               "n log-uniform 50..1000, 1000 reads x 1000 sweeps each",
                   "instances": len(insts), "total_n": sum(i.n for i in insts)},
        "plain_spin_updates_per_s": round(updates / plain_s, 1), "plain_ms": round(plain_s * 1e3, 3),
        "batched_over_plain": round(plain_s / batched_s, 3), "bit_identical": bool(same),
        "batch_shape": shape, "roofline": roofline, "cpu_baseline": cpu,
    }
    return out


def bench_pt(args, cfg, label):
    """PT workloads: `runs` tempering runs of K slots x `chains` chains (Houdayer moves at
    every slot when the config asks for them), then persistence on the top-10 sample of
    the colder half, assembled on the device."""
    import torch

    import paper_1706_07826_amd as spv
    from spvar_inputs import configs as cf

    inst = cf.instance(cfg)
    betas = cf.betas(cfg)
    K, chains = betas.size, cfg.get("chains", 1)
    runs = args.pt_runs or cfg["runs"]
    icm = (0, K) if cfg.get("icm") else None
    ctx = spv.Context(0)
    P = spv.Problem.from_instance(inst)
    updates = inst.n * K * chains * runs * cfg["sweeps"]

    def step():
        r = spv.spv_pt_sample(ctx, P, betas, runs, chains, cfg["sweeps"], cfg["seed"], icm=icm, final=False)
        S, E = spv.spv_top_sample(ctx, r)
        return spv.spv_persist_fix(ctx, P, S, E, cfg["elite"], cfg["theta"], cfg["gauge"])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fx = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    if args.calib_copy_mib:
        # a plain copy of known size, for scaling the HBM counters of a profiled run
        src = torch.ones(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    out = {
        "metric": METRIC_NAME, "value": round(updates / dt, 1), "unit": "spin-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": f"synthetic Gaussian cubic L={cfg['L']} instance",
        "config": {"workload": label.format(runs=runs)},
        "spvar_solves_per_s": round(1 / dt, 4), "fixed_per_solve": fx.info()["n_fixed"],
    }
    # the Metropolis part of the sweep against the measured LDS peak (the cluster moves and
    # the exchange add latency-bound work on top; records are LDS-resident at N = 1000)
    max_degree, x_bound = spv.spv_problem_check(ctx, P)
    nd = 2 if x_bound > 511 else 1
    probe = measured_lds_peak(spv, ctx)
    out["lds"] = lds_object(updates / dt, pt_lds_bytes_per_update(max_degree, nd, inst.n <= 4096), probe,
                            "Metropolis LDS traffic of the whole step against the measured LDS peak")
    print(json.dumps(out), flush=True)


def bench_serving(args):
    print(json.dumps(part_serving(args, args.serving_requests, (0.5, 0.8, 0.95))), flush=True)


def part_serving(args, nreq, load_fracs, line=True):
    """Serving stream: requests of three kinds (by count 60 % SA on the Chimera N=512 instance,
    1000 reads x 1000 sweeps + persistence; 30 % PT on the cubic N=1000 instance, 32 betas x 4
    runs x 1000 sweeps + persistence; 10 % PT with Houdayer moves on the cubic N=8000 instance,
    40 betas x 2 chains x 1 run x 1000 sweeps + persistence), seed = base + request id.  First
    a burst of all requests measures the saturation rate; then Poisson arrivals at 0.5, 0.8 and
    0.95 of it.  Latency = submit -> completion observed by the server's host thread."""
    import numpy as np
    import torch

    import paper_1706_07826_amd as spv
    from spvar_inputs import configs as cf

    ctx = spv.Context(0)
    c2, c3, c5 = cf.CHIMERA8_SA, cf.CUBIC10_PT, cf.CUBIC20_PTICM
    kinds = {
        "sa512": dict(P=spv.Problem.from_instance(cf.instance(c2)), betas=cf.betas(c2, 1000), cfg=c2),
        "pt1000": dict(P=spv.Problem.from_instance(cf.instance(c3)), betas=cf.betas(c3), cfg=c3),
        "pticm8000": dict(P=spv.Problem.from_instance(cf.instance(c5)), betas=cf.betas(c5), cfg=c5),
    }
    updates = {"sa512": 512 * 1000 * 1000, "pt1000": 1000 * 32 * 4 * 1000, "pticm8000": 8000 * 80 * 1000}
    rng = np.random.default_rng(31337)
    mix = rng.choice(["sa512", "pt1000", "pticm8000"], size=nreq, p=[0.6, 0.3, 0.1])
    base_seed = 5000
    srv = spv.Server(ctx, slots=args.serving_slots)

    def prepare(i):
        k = mix[i]
        d = kinds[k]
        c = d["cfg"]
        if k == "sa512":
            return srv.prepare_sa(d["P"], d["betas"], 1000, base_seed + i, c["elite"], c["theta"], c["gauge"])
        if k == "pt1000":
            return srv.prepare_pt(d["P"], d["betas"], 4, 1, 1000, base_seed + i, None, c["elite"], c["theta"],
                                  c["gauge"], final=False)
        K = d["betas"].size
        return srv.prepare_pt(d["P"], d["betas"], 1, 2, 1000, base_seed + i, (0, K), c["elite"], c["theta"],
                              c["gauge"], final=False)

    def run(rate):
        reqs = [prepare(i) for i in range(nreq)]
        torch.cuda.synchronize()
        gaps = rng.exponential(1.0 / rate, size=nreq) if rate else np.zeros(nreq)
        t0 = time.perf_counter()
        due = t0
        tickets = []
        for i in range(nreq):
            due += gaps[i]
            while True:
                now = time.perf_counter()
                if now >= due:
                    break
                if due - now > 2e-4:
                    time.sleep(due - now - 1e-4)
            tickets.append(srv.submit(*reqs[i]))
        res = [srv.wait(t)[0] for t in tickets]
        first = min(r.submit_ns for r in res)
        last = max(r.done_ns for r in res)
        lat = np.array([(r.done_ns - r.submit_ns) / 1e6 for r in res])
        for t in tickets:
            srv.release(t)
        span = (last - first) / 1e9
        upd = sum(updates[k] for k in mix)
        out = {"requests_per_s": round(nreq / span, 2), "spin_updates_per_s": round(upd / span, 1),
               "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3)}
        for k in kinds:
            sel = lat[mix == k]
            if sel.size:
                out[f"p50_ms_{k}"] = round(float(np.percentile(sel, 50)), 3)
                out[f"p99_ms_{k}"] = round(float(np.percentile(sel, 99)), 3)
        print(f"[serving] rate={rate or 'burst'} {out}", file=sys.stderr, flush=True)
        return out

    # warm up every kind (tables, buffers, code objects)
    for i in range(min(nreq, 12)):
        t = srv.submit(*prepare(i))
        srv.wait(t)
        srv.release(t)
    sat = run(0)
    loads = {}
    for f in load_fracs:
        loads[str(f)] = run(f * sat["requests_per_s"])
    srv.close()
    roofline, cpu = serving_roofline_and_cpu(args, ctx, kinds)
    out = {
        "metric": METRIC_NAME, "value": sat["spin_updates_per_s"], "unit": "spin-updates/s",
        "n_gpus": 1, "steps": nreq, "warmup": 12, "ms_per_step": round(1e3 / sat["requests_per_s"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic Chimera N=512, Gaussian cubic N=1000 and N=8000 instances",
        "config": {"workload": f"serving: {nreq} requests (60 % SA N=512 1000x1000 + fix, 30 % PT N=1000 "
                               "32 betas x 4 runs x 1000 sweeps + fix, 10 % PT-ICM N=8000 40 betas x 2 chains "
                               "x 1000 sweeps + fix), burst then Poisson at 0.5/0.8/0.95 of saturation",
                   "slots": args.serving_slots, "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES")},
        "saturation": sat, "poisson": loads, "roofline": roofline, "cpu_baseline": cpu,
    }
    if line:
        return out
    top = loads[str(load_fracs[-1])] if load_fracs else sat
    return {"workload": out["config"]["workload"], "load": load_fracs[-1] if load_fracs else "burst",
            "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"], "requests_per_s": sat["requests_per_s"],
            "spin_updates_per_s": sat["spin_updates_per_s"], "saturation": sat, "poisson": loads,
            "slots": args.serving_slots, "roofline": roofline, "cpu_baseline": cpu}


def serving_roofline_and_cpu(args, ctx, kinds):
    """The serving stream's dominant kernel by device time is the N=8000 tempering kernel with
    cluster moves (10 % of the requests, each about two orders of magnitude longer than an SA
    request): its VALU roofline from one request run alone, timed with HIP events on its
    stream.  cpu_baseline: the oracle's throughput on a bounded sample of every request kind
    (SA: 64 reads; PT N=1000: 4 runs of 250 sweeps; PT-ICM N=8000: one run of 20 sweeps), and
    the latency a request of each kind would have on the host threads at those rates."""
    import numpy as np
    import torch

    import paper_1706_07826_amd as spv

    d = kinds["pticm8000"]
    P, betas, c = d["P"], d["betas"], d["cfg"]
    K = betas.size
    stream = torch.cuda.current_stream()
    spv.spv_pt_sample(ctx, P, betas, 1, 2, 1000, 1, icm=(0, K), final=False)  # warm-up
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    spv.spv_pt_sample(ctx, P, betas, 1, 2, 1000, 2, icm=(0, K), final=False)
    ev[1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    md, xb = spv.spv_problem_check(ctx, P)
    digits = 1 if xb < 512 else (2 if xb < 512 * 512 else 3)
    philox_slots = measured_philox_slots(spv, ctx)
    upd = P.n * K * 2 * 1000
    spu = pt_slots_per_update(P.nnz / P.n, digits, philox_slots)
    achieved = upd * spu / (ms / 1e3) / 1e12
    probe = measured_lds_peak(spv, ctx)
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(PEAK_VALU_TSLOTS, 3),
                "unit": "Tslot/s", "frac": round(achieved / PEAK_VALU_TSLOTS, 5), "traffic": None,
                "kernel": f"ptx_kernel<{digits}, true, {md}>", "kernel_ms": round(ms, 3),
                "slots_per_update": round(spu, 3),
                "lds": lds_object(upd / (ms / 1e3), pt_lds_bytes_per_update(md, digits, False), probe,
                                  "LDS traffic of the Metropolis updates against the measured LDS peak"),
                "note": "one PT-ICM request alone (N=8000, 40 betas x 2 chains x 1000 sweeps, Houdayer moves "
                        "at every slot); a run spans at most one workgroup per slot (40 of 256 CUs), and its "
                        "sweeps are a chain of dependent steps"}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        from spvar_inputs import configs as cf
        threads = cpu_threads()
        sa, pt = kinds["sa512"], kinds["pt1000"]
        inst_sa, inst_pt, inst_icm = cf.instance(sa["cfg"]), cf.instance(pt["cfg"]), cf.instance(c)
        rates = {}
        t1 = time.perf_counter()
        oracle.sa_sample(inst_sa, sa["betas"], seed=5000, r_begin=0, r_end=64, threads=threads)
        dt = time.perf_counter() - t1
        rates["sa512"] = 64 * inst_sa.n * 1000 / dt
        t1 = time.perf_counter()
        oracle.pt_sample(inst_pt, pt["betas"], 4, 1, 250, seed=5001, threads=min(4, threads))
        dt = time.perf_counter() - t1
        rates["pt1000"] = 4 * 32 * inst_pt.n * 250 / dt
        t1 = time.perf_counter()
        oracle.pt_sample(inst_icm, betas, 1, 2, 20, seed=5002, icm=(0, K), threads=1)
        dt = time.perf_counter() - t1
        rates["pticm8000"] = 80 * inst_icm.n * 20 / dt
        upd_kind = {"sa512": 512 * 1000 * 1000, "pt1000": 1000 * 32 * 4 * 1000, "pticm8000": 8000 * 80 * 1000}
        mix = {"sa512": 0.6, "pt1000": 0.3, "pticm8000": 0.1}
        mean_upd = sum(mix[k] * upd_kind[k] for k in mix)
        mean_s = sum(mix[k] * upd_kind[k] / rates[k] for k in mix)
        cpu = {"value": round(mean_upd / mean_s, 1), "unit": "spin-updates/s", "cores": threads, "kind": "oracle",
               "latency_ms": {k: round(upd_kind[k] / rates[k] * 1e3, 1) for k in mix},
               "sample": f"SA N=512 64 reads x 1000 sweeps on {threads} threads; PT N=1000 4 runs x 250 sweeps "
                         f"on {min(4, threads)} threads (one run per thread); PT-ICM N=8000 1 run x 20 sweeps "
                         "on 1 thread (a run is sequential); value = the request mix's spin-updates/s at "
                         "those rates, latency_ms = one request of each kind at its rate"}
    return roofline, cpu


def bench_headline(args):
    """The metric's three clauses in one line: the config-4 residual batch, batched vs plain
    (value = batched spin-updates/s); config-2 SPVAR solves/s (SA + persistence); config-5
    serving p50/p99 (a burst for the saturation rate, then Poisson arrivals at 0.8 of it).
    Each carries the roofline of its dominant kernel and a CPU-oracle baseline."""
    batch = part_residual_batch(args)
    solves = part_chimera8_sa(args, line=False)
    serving = part_serving(args, 400, (0.8,), line=False)
    out = {k: batch[k] for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                                 "higher_is_better", "scaling", "vs_baseline", "dtype")}
    out["data"] = ("synthetic: residual-shaped instances cut from a seeded Chimera 16x16 parent; seeded Chimera "
                   "8x8 and Gaussian cubic L=10 / L=20 instances (no paper instances available)")
    out["config"] = dict(batch["config"])
    out["plain"] = {"spin_updates_per_s": batch["plain_spin_updates_per_s"], "ms": batch["plain_ms"],
                    "launches": batch["config"]["instances"]}
    out["batched_over_plain"] = batch["batched_over_plain"]
    out["bit_identical"] = batch["bit_identical"]
    out["batch_shape"] = batch["batch_shape"]
    out["roofline"] = batch["roofline"]
    out["cpu_baseline"] = batch["cpu_baseline"]
    out["spvar_solves"] = solves
    out["serving"] = serving
    print(json.dumps(out), flush=True)


def bench_spvar_round(args):
    """One SPVAR round with the recombination of Sec. II.C on the Chimera N=512 workload:
    SA (10,000 reads x 2,000 sweeps) -> persistence (elite 5 %, threshold 0.95) ->
    components of the residual -> SA on the residual (same reads and schedule) ->
    sorted-merge recombination over the components."""
    import numpy as np
    import torch

    import paper_1706_07826_amd as spv
    from spvar_inputs import configs as cf

    cfg = cf.CHIMERA8_SA
    inst = cf.instance(cfg)
    betas = cf.betas(cfg)
    reads, sweeps = cfg["reads"], cfg["sweeps"]
    ctx = spv.Context(0)
    P = spv.Problem.from_instance(inst)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        S, E = spv.spv_sample(ctx, P, betas, reads, cfg["seed"])
        fx = spv.spv_persist_fix(ctx, P, S, E, cfg["elite"], cfg["theta"], cfg["gauge"])
        red = fx.reduced()  # reads the sizes back (synchronises)
        comp, nc = spv.spv_components(ctx, red)
        RS, RE = spv.spv_sample(ctx, red, betas, reads, cfg["seed"] + 1)
        if ev is not None:
            ev[0].record(stream)
        merged, mE, _ = spv.spv_merge_components(ctx, red, comp, nc, RS)
        if ev is not None:
            ev[1].record(stream)
        return dict(E=E, fx=fx, red=red, nc=nc, RE=RE, mE=mE)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step(evs[k])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    merge_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    n_res = out["red"].n
    updates = reads * sweeps * (inst.n + n_res)
    off = out["fx"].info()["offset"]
    res = {
        "metric": METRIC_NAME, "value": round(updates / dt, 1), "unit": "spin-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded Chimera U{+-1..+-6} instance)",
        "config": {"workload": "spvar_round: chimera8 SA 10000 x 2000 -> persistence -> components of the "
                               "residual -> SA on the residual 10000 x 2000 -> sorted-merge recombination"},
        "residual_n": n_res, "components": out["nc"], "merge_ms": round(merge_ms, 4),
        "best_E_first_sample": int(out["E"].min().item()),
        "best_E_round_unmerged": int(out["RE"].min().item()) + off,
        "best_E_round_merged": int(out["mE"][0].item()) + off,
    }
    print(json.dumps(res), flush=True)


def bench_multistart(args, sqa=False):
    """Multi-start SPVAR (Algorithm 2) on the Chimera N=512 workload with parameters in the
    paper's ranges: 20 starts, fixing and solving samples of 1000 reads, 2000 sweeps, elite 5 %,
    threshold 0.95, recombination over components.  sqa=True: SQA as the sampler (16 slices,
    Gamma 3.0 -> 0.01 geometric; spin-updates then count every slice)."""
    import numpy as np
    import torch

    import paper_1706_07826_amd as spv
    from spvar_inputs import configs as cf

    cfg = cf.CHIMERA8_SA
    inst = cf.instance(cfg)
    betas = cf.betas(cfg)
    S, F, Rs = 20, 1000, 1000
    trotter = 16 if sqa else 1
    extra = dict(gammas=np.geomspace(3.0, 0.01, betas.size), trotter=trotter) if sqa else {}
    ctx = spv.Context(0)
    P = spv.Problem.from_instance(inst)

    def step():
        return spv.spv_multistart(ctx, P, betas, cfg["seed"], S, F, Rs, cfg["elite"], cfg["theta"], cfg["gauge"],
                                  merge=True, **extra)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    n_free = out["info"][:, 3]
    updates = trotter * cfg["sweeps"] * (S * F * inst.n + Rs * int(n_free.sum()))
    res = {
        "metric": METRIC_NAME, "value": round(updates / dt, 1), "unit": "spin-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded Chimera U{+-1..+-6} instance)",
        "config": {"workload": f"multistart{'_sqa' if sqa else ''}: chimera8, {S} starts x ({F} fixing + {Rs} "
                               f"solving reads) x {cfg['sweeps']} sweeps"
                               f"{f', SQA {trotter} slices' if sqa else ''}, elite {cfg['elite']}, "
                               f"threshold {cfg['theta']}, recombination over components"},
        "starts_per_s": round(S / dt, 2), "mean_free": round(float(n_free.mean()), 1),
        "mean_components": round(float(out["info"][:, 5].mean()), 1), "best_E": out["best_E"],
    }
    print(json.dumps(res), flush=True)


def bench_spvar_tree(args):
    """One SPVAR round with the tree pre-processing of Sec. II.C on the Chimera N=512 workload:
    SA (10,000 reads x 2,000 sweeps) -> persistence (elite 5 %, threshold 0.95) -> tree /
    degree-1 pre-processing of the residual -> SA on the peeled residual (same reads and
    schedule) -> completion of every sample to the residual's variables."""
    import numpy as np
    import torch

    import paper_1706_07826_amd as spv
    from spvar_inputs import configs as cf

    cfg = cf.CHIMERA8_SA
    inst = cf.instance(cfg)
    betas = cf.betas(cfg)
    reads, sweeps = cfg["reads"], cfg["sweeps"]
    ctx = spv.Context(0)
    P = spv.Problem.from_instance(inst)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        S, E = spv.spv_sample(ctx, P, betas, reads, cfg["seed"])
        fx = spv.spv_persist_fix(ctx, P, S, E, cfg["elite"], cfg["theta"], cfg["gauge"])
        red = fx.reduced()  # reads the sizes back (synchronises)
        if ev is not None:
            ev[0].record(stream)
        tr = spv.spv_tree_reduce(ctx, red)
        if ev is not None:
            ev[1].record(stream)
        core = tr.reduced()  # synchronises
        RS, RE = spv.spv_sample(ctx, core, betas, reads, cfg["seed"] + 1)
        if ev is not None:
            ev[2].record(stream)
        full = spv.spv_tree_complete(ctx, tr, RS)
        if ev is not None:
            ev[3].record(stream)
        return dict(E=E, fx=fx, red=red, tr=tr, RE=RE, full=full)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step(evs[k])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    tree_us = float(np.mean([e[0].elapsed_time(e[1]) for e in evs])) * 1e3
    complete_us = float(np.mean([e[2].elapsed_time(e[3]) for e in evs])) * 1e3
    ti = out["tr"].info()
    # the pre-processing alone on a larger tree-rich graph (N=8000, mean degree 1.5)
    from spvar_inputs import random_sparse
    big = spv.Problem.from_instance(random_sparse(8000, 1.5, seed=1))
    bt = spv.spv_tree_reduce(ctx, big)
    bt.info()

    def back_to_back(prob, res, k=20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(k):
            spv.spv_tree_reduce(ctx, prob, out=res)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k * 1e3

    big_us = back_to_back(big, bt)
    res_us = back_to_back(out["red"], out["tr"])
    updates = reads * sweeps * (inst.n + ti["n_free"])
    off = out["fx"].info()["offset"] + ti["offset"]
    res = {
        "metric": METRIC_NAME, "value": round(updates / dt, 1), "unit": "spin-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded Chimera U{+-1..+-6} instance)",
        "config": {"workload": "spvar_tree: chimera8 SA 10000 x 2000 -> persistence -> tree / degree-1 "
                               "pre-processing of the residual -> SA on the peeled residual 10000 x 2000 -> "
                               "completion"},
        "residual_n": out["red"].n, "peeled": ti["n_removed"], "core_n": ti["n_free"], "tree_rounds": ti["rounds"],
        "tree_call_us": round(tree_us, 2), "complete_call_us": round(complete_us, 2),
        "tree_back_to_back_us": round(res_us, 2),
        "tree_sparse8000_us": round(big_us, 2), "tree_sparse8000": bt.info(),
        "best_E_first_sample": int(out["E"].min().item()),
        "best_E_round": int(out["RE"].min().item()) + off,
    }
    print(json.dumps(res), flush=True)


def bench_cubic4_ispvar(args):
    """SPVAR solves/s on the 3D +-1 spin glass L=4 (N=64): one solve = 5 iterated SPVAR
    rounds (SA 100 reads x 1000 sweeps, elite 0.1, threshold 1.0, zero-bias gauge), the
    same call timed on the GPU and, as cpu_baseline, in the oracle on one host core."""
    import torch

    import paper_1706_07826_amd as spv
    from spvar_inputs import configs as cf

    cfg = cf.CUBIC4_SA
    inst = cf.instance(cfg)
    betas = cf.betas(cfg)
    ctx = spv.Context(0)
    P = spv.Problem.from_instance(inst)

    def step():
        return spv.spv_ispvar(ctx, P, betas, cfg["reads"], cfg["seed"], cfg["rounds"], cfg["elite"], cfg["theta"],
                              cfg["gauge"])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    updates = sum(cfg["reads"] * int(r[0]) * cfg["sweeps"] for r in res["round_info"])
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t1 = time.perf_counter()
        ores = oracle.ispvar(inst, betas, cfg["reads"], cfg["seed"], cfg["rounds"], cfg["elite"], cfg["theta"],
                             cfg["gauge"])
        cdt = time.perf_counter() - t1
        same = bool((ores["fixed_val"] == res["fixed_val"].cpu().numpy()).all())
        cpu = {"value": round(1.0 / cdt, 3), "unit": "SPVAR solves/s", "cores": 1, "kind": "oracle",
               "sample": f"one full solve ({cfg['rounds']} rounds), {cdt:.2f} s, identical fixes: {same}"}
    out = {
        "metric": METRIC_NAME, "value": round(1.0 / dt, 3), "unit": "SPVAR solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded +-1 cubic L=4 instance)",
        "config": {"workload": "cubic4_ispvar: periodic cubic L=4 (N=64) +-1 couplers, 5 ISPVAR rounds of SA "
                               "100 reads x 1000 sweeps, elite 0.1, threshold 1.0, zero-bias gauge"},
        "spin_updates_per_s": round(updates / dt, 1), "rounds_run": res["rounds_run"],
        "round_info": [[int(v) for v in r] for r in res["round_info"]],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_chimera32_sa(args):
    """SA beyond the LDS: Chimera 32x32 (N=8192, couplers/biases U{+-1..+-6}), 10,000 reads x
    2,000 sweeps (the chimera8 schedule): the byte-parallel body with its instance in global
    memory, streamed."""
    import torch

    import paper_1706_07826_amd as spv
    from spvar_inputs import chimera, linear_betas

    inst = chimera(32, seed=1032)
    betas = linear_betas(0.1, 5.0, 2000)
    reads = 10000
    ctx = spv.Context(0)
    P = spv.Problem.from_instance(inst)
    spins = torch.empty((reads, inst.n), dtype=torch.int8, device="cuda")
    energies = torch.empty(reads, dtype=torch.int64, device="cuda")
    for _ in range(args.warmup):
        spv.spv_sample(ctx, P, betas, reads, 9, spins=spins, energies=energies)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        spv.spv_sample(ctx, P, betas, reads, 9, spins=spins, energies=energies)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    updates = reads * inst.n * betas.size
    out = {
        "metric": METRIC_NAME, "value": round(updates / dt, 1), "unit": "spin-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded Chimera U{+-1..+-6} instance)",
        "config": {"workload": "chimera32_sa: Chimera 32x32 K4,4 N=8192, SA 10000 reads x 2000 sweeps, "
                               "instance in global memory"},
        "launch": spv.spv_sample_last_shape(ctx),
        "best_E": int(energies.min().item()),
    }
    print(json.dumps(out), flush=True)


def bench_chimera8_sqa(args):
    """SQA on the Chimera 8x8 instance of the SA workload: 16 Trotter slices, 1000 reads x 2000
    sweeps, beta 0.1 -> 5.0 (linear), Gamma 3.0 -> 0.01 (geometric), then persistence (elite 0.05,
    threshold 0.95) on the reads' lowest-energy slices.  Spin-updates count every slice."""
    import numpy as np
    import torch

    import paper_1706_07826_amd as spv
    from spvar_inputs import configs as cf, linear_betas

    cfg = cf.CHIMERA8_SA
    inst = cf.instance(cfg)
    trotter, reads, sweeps = 16, 1000, 2000
    betas, gammas = linear_betas(0.1, 5.0, sweeps), np.geomspace(3.0, 0.01, sweeps)
    ctx = spv.Context(0)
    P = spv.Problem.from_instance(inst)
    stream = torch.cuda.current_stream()
    spins = torch.empty((reads, inst.n), dtype=torch.int8, device="cuda")
    energies = torch.empty(reads, dtype=torch.int64, device="cuda")

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        spv.spv_sqa_sample(ctx, P, betas, gammas, trotter, reads, 11, spins=spins, energies=energies)
        if ev is not None:
            ev[1].record(stream)
        return spv.spv_persist_fix(ctx, P, spins, energies, cfg["elite"], cfg["theta"], cfg["gauge"])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    t0 = time.perf_counter()
    last = None
    for k in range(args.steps):
        last = step(events[k])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    sqa_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    updates = reads * trotter * inst.n * sweeps
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = max(1, min(16, os.cpu_count() or 1))
        cpu_reads = 4 * threads
        t1 = time.perf_counter()
        oracle.sqa_sample(inst, betas, gammas, trotter, seed=11, r_begin=0, r_end=cpu_reads, threads=threads)
        cdt = time.perf_counter() - t1
        cpu = {"value": round(cpu_reads * trotter * inst.n * sweeps / cdt, 1), "unit": "spin-updates/s",
               "cores": threads, "kind": "oracle",
               "sample": f"reads 0..{cpu_reads - 1} of {reads} (all {sweeps} sweeps, {trotter} slices), "
                         f"{threads} threads, {cdt:.1f} s wall"}
    out = {
        "metric": METRIC_NAME, "value": round(updates / dt, 1), "unit": "spin-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded Chimera U{+-1..+-6} instance)",
        "config": {"workload": "chimera8_sqa: Chimera 8x8 K4,4 N=512, SQA 16 slices, 1000 reads x 2000 "
                               "sweeps, beta 0.1->5.0, Gamma 3.0->0.01; persistence elite 0.05, threshold 0.95"},
        "sqa_kernel_ms": round(sqa_ms, 3),
        "kernel_spin_updates_per_s": round(updates / (sqa_ms / 1e3), 1),
        "fixed_per_solve": last.info()["n_fixed"],
        "best_E": int(energies.min().item()),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
