#!/usr/bin/env python3
"""Throughput benchmark of the sample-persistence hot path on one MI355X.

One step = one full pass of the path over one batch of synthetic input:
spv_sample (Metropolis simulated annealing, 10,000 reads x 2,000 sweeps on the
Chimera 8x8 instance, N = 512) followed by spv_persist_fix (elite 5 %,
threshold 0.95).  Inputs are resident in device memory before timing starts.

Prints ONE JSON line.  `value` is spin-updates/s of the whole step
(reads x n x sweeps / step time).  The roofline object covers the dominant
kernel (the SA sweep), timed with events on the stream it runs on.  The
cpu_baseline object times the CPU oracle on a bounded sample of the same
workload (a subset of reads, all sweeps).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

BASELINE_METRIC = "spin-updates/s (batched vs plain, bit-exact); SPVAR solves/s; p50/p99 latency"

# VALU lane-slots per Metropolis update on the Chimera workload (single-digit
# threshold test): local field over the mean degree (one conditional add per
# coupler), 4 slots for x = -s f / sign test / threshold compare / flip, and a
# quarter of one Philox4x32-10 block: 10 rounds of two 32x32->64 products
# (v_mad_u64_u32, 2 issue slots each on gfx950) and two 3-input xors, i.e. 60
# slots per block (a chained-Philox probe measures 59-66 slots per block).
PHILOX_SLOTS = 10 * (2 * 2 + 2)
PEAK_VALU_TSLOTS = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 64 lanes x 2.4 GHz = 39.32 T lane-slots/s


def slots_per_update(mean_degree):
    return mean_degree + 4 + PHILOX_SLOTS / 4.0


def profiled_traffic_bytes():
    """HBM bytes per launch of the SA kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a copy of known size), or None
    when the kernel source changed after the counters were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "sa_kernel_chimera8_sa.json")) as f:
            prof = json.load(f)
        with open(os.path.join(ROOT, prof["source"]), "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except (OSError, KeyError, ValueError):
        return None
    if not digest.startswith(prof["source_sha256_prefix"]):
        return None
    kib = prof["fetch_kib"] * prof["fetch_scale"] + prof["write_kib"] * prof["write_scale"]
    return int(round(kib * 1024))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reads", type=int, default=0, help="oracle reads (0 = 64 per thread)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, run one device copy of this size (counter calibration)")
    ap.add_argument("--workload", default="chimera8_sa",
                    choices=["chimera8_sa", "residual_batch", "cubic10_pt"])
    args = ap.parse_args()
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
        return bench_cubic10_pt(args)

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
    spu = slots_per_update(mean_deg)
    achieved = updates * spu / (sa_ms / 1e3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TSLOTS, 3),
                "unit": "Tslot/s", "frac": round(achieved / PEAK_VALU_TSLOTS, 4),
                "traffic": profiled_traffic_bytes(),
                "kernel": "sa_kernel<1>", "kernel_ms": round(sa_ms, 4),
                "slots_per_update": round(spu, 3)}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = max(1, min(16, os.cpu_count() or 1))
        cpu_reads = args.cpu_reads or 64 * threads
        t1 = time.perf_counter()
        oracle.sa_sample(inst, betas, seed=cfg["seed"], r_begin=0, r_end=cpu_reads, threads=threads)
        dt = time.perf_counter() - t1
        cpu = {"value": round(cpu_reads * n * sweeps / dt, 1), "unit": "spin-updates/s",
               "cores": threads, "kind": "oracle",
               "sample": f"reads 0..{cpu_reads - 1} of {reads} (all {sweeps} sweeps), "
                         f"{threads} threads, {dt:.1f} s wall"}

    out = {
        "metric": BASELINE_METRIC, "value": round(value, 1), "unit": "spin-updates/s",
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
    print(json.dumps(out), flush=True)


def bench_residual_batch(args):
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
    t0 = time.perf_counter()
    for _ in range(args.steps):
        spv.spv_sample_batch(ctx, probs, betas, reads, seeds, spins=sp, energies=en, graph=True)
    torch.cuda.synchronize()
    batched_s = (time.perf_counter() - t0) / args.steps
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
    out = {
        "metric": BASELINE_METRIC, "value": round(updates / batched_s, 1), "unit": "spin-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(batched_s * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic residual-shaped instances",
        "config": {"workload": "residual_batch: 512 BFS-ball residuals of a Chimera 16x16 parent, "
                               "n log-uniform 50..1000, 1000 reads x 1000 sweeps each",
                   "instances": len(insts), "total_n": sum(i.n for i in insts)},
        "plain_spin_updates_per_s": round(updates / plain_s, 1), "plain_ms": round(plain_s * 1e3, 3),
        "batched_over_plain": round(plain_s / batched_s, 3), "bit_identical": bool(same),
        "batch_shape": shape,
    }
    print(json.dumps(out), flush=True)


def bench_cubic10_pt(args):
    """cubic10_pt: 64 PT runs x 32 slots x 10^4 sweeps on the L=10 lattice, then persistence
    on the 10,240-state top-10 sample."""
    import torch

    import paper_1706_07826_amd as spv
    from spvar_inputs import configs as cf

    cfg = cf.CUBIC10_PT
    inst = cf.instance(cfg)
    betas = cf.betas(cfg)
    ctx = spv.Context(0)
    P = spv.Problem.from_instance(inst)
    updates = inst.n * cfg["K"] * cfg["runs"] * cfg["sweeps"]

    def step():
        r = spv.spv_pt_sample(ctx, P, betas, cfg["runs"], 1, cfg["sweeps"], cfg["seed"], final=False)
        S = r["top_spins"].reshape(-1, inst.n)
        E = r["top_E"].reshape(-1)
        return spv.spv_persist_fix(ctx, P, S, E, cfg["elite"], cfg["theta"], cfg["gauge"])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fx = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    out = {
        "metric": BASELINE_METRIC, "value": round(updates / dt, 1), "unit": "spin-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic Gaussian cubic L=10 instance",
        "config": {"workload": "cubic10_pt: PT 32 betas 0.2..5.0, 64 runs x 10^4 sweeps, top-10 "
                               "sample of the 16 colder slots, persistence elite 0.2"},
        "spvar_solves_per_s": round(1 / dt, 4), "fixed_per_solve": fx.info()["n_fixed"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
