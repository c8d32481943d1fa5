"""Runs the sampling kernels of the race-detection build (libspvar_shadow.so, loaded with
SPVAR_LIBRARY=shadow) over every SA body and launch shape and the tempering kernels, checks
each result bit for bit against the oracle, and prints the detector's counts as one JSON line
per phase:

* "clean": valid colourings through the byte-parallel body (two words per lane, one word per
  lane, streamed, instance in global memory), the general body (x_bound > 255, in LDS and in
  global memory), the batched launch (one-word and paired bodies) and the tempering kernels
  (one workgroup per run; the ladder split over workgroups with the instance in LDS and in
  global memory, and into groups of 2 slots and of 1 slot that own part of each quad word;
  cluster moves on) and SQA (instance in LDS and in global memory);
* "one_class": a colouring with every site in one class (edges inside the class), let through
  ingest by SPVAR_SHADOW_ALLOW_COLOUR_EDGES, where every class pass reads neighbours that the
  same pass writes, through SA and through tempering.

Run by tests/test_gpu_lds_shadow.py in a process of its own."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import paper_1706_07826_amd as spv  # noqa: E402
import spvar_inputs as si  # noqa: E402


def say(*a):
    print(*a, flush=True)


def with_env(env, fn):
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return fn()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def sample_case(ctx, name, inst, env, reads=40, sweeps=30, seed=5):
    say(f"[shadow] {name}: n={inst.n} reads={reads} env={env}")
    P = spv.Problem.from_instance(inst)
    betas = si.linear_betas(0.1, 3.0, sweeps)
    S, E = with_env(env, lambda: spv.spv_sample(ctx, P, betas, reads, seed))
    oS, oE = oracle.sa_sample(inst, betas, reads=reads, seed=seed)
    assert np.array_equal(S.cpu().numpy(), oS) and np.array_equal(E.cpu().numpy(), oE), name


def main():
    assert "race detection" in spv._lib.spv_version().decode(), spv._lib.spv_version()
    ctx = spv.Context(0)
    spv.spv_debug_lds_shadow(ctx, reset=True)
    swar = si.chimera(4, seed=3)  # x_bound <= 255: byte-parallel body
    general = si.cubic_lattice(4, "gauss", seed=4, scale_log2=10)  # x_bound > 255: general body
    sample_case(ctx, "swar_w2", swar, {})
    sample_case(ctx, "swar_w1", swar, {"SPVAR_SA_WPL": 1, "SPVAR_SA_THREADS": 512})
    sample_case(ctx, "swar_streamed", swar, {"SPVAR_SA_STREAM": 8}, reads=300)
    sample_case(ctx, "swar_big", swar, {"SPVAR_SA_BIG": 1})
    sample_case(ctx, "swar_w2_big", swar, {"SPVAR_SA_BIG": 1, "SPVAR_SA_WPL": 2, "SPVAR_SA_THREADS": 256})
    sample_case(ctx, "general", general, {})
    sample_case(ctx, "general_big", general, {"SPVAR_SA_BIG": 1})
    insts = [si.random_sparse(n, 2.0, seed=70 + n, j_max=3, h_max=3) for n in (12, 30, 47, 64, 90)]
    for i in insts:
        i.colour, i.n_colours = si.greedy_colouring(i)
    reads = [200, 99, 57, 130, 33]
    seeds = [40 + b for b in range(len(insts))]
    betas = si.linear_betas(0.1, 3.0, 25)
    probs = [spv.Problem.from_instance(i) for i in insts]
    for label, kw in (("batch_paired", dict(threads=1024, wgs_per_cu=1, paired=True)),
                      ("batch_one_word", dict(threads=256, quads_per_item=2, wgs_per_cu=4))):
        say(f"[shadow] {label}")
        sp, en = spv.spv_sample_batch(ctx, probs, betas, reads, seeds, **kw)
        for b, inst in enumerate(insts):
            oS, oE = oracle.sa_sample(inst, betas, reads=reads[b], seed=seeds[b])
            assert np.array_equal(sp[b].cpu().numpy(), oS) and np.array_equal(en[b].cpu().numpy(), oE), (label, b)
    cube = si.cubic_lattice(4, "gauss", seed=9, scale_log2=10)
    for label, env, K in (("pt_one_workgroup", {"SPVAR_PT_SPLIT": 0}, 6),
                          ("pt_split", {"SPVAR_PT_SPLIT": 1, "SPVAR_PT_GROUPS": 2}, 8),
                          ("pt_split_big", {"SPVAR_PT_SPLIT": 1, "SPVAR_PT_GROUPS": 2, "SPVAR_PT_BIG": 1}, 8),
                          ("pt_split_half_quads", {"SPVAR_PT_SPLIT": 1, "SPVAR_PT_GROUPS": 4}, 8),
                          ("pt_split_single_slots", {"SPVAR_PT_SPLIT": 1, "SPVAR_PT_GROUPS": 8}, 8)):
        say(f"[shadow] {label}: K={K}")
        betas_pt = si.geometric_betas(0.2, 5.0, K)
        Pc = spv.Problem.from_instance(cube)
        got = with_env(env, lambda: spv.spv_pt_sample(ctx, Pc, betas_pt, 2, 2, 30, 4, icm=(0, K)))
        want = oracle.pt_sample(cube, betas_pt, 2, 2, 30, seed=4, icm=(0, K))
        for key in ("final_spins", "final_E", "top_E", "top_count", "top_spins"):
            assert np.array_equal(got[key].cpu().numpy(), want[key]), (label, key)
    for label, env in (("sqa", {}), ("sqa_big", {"SPVAR_SQA_BIG": 1})):
        say(f"[shadow] {label}: P=8")
        b = si.linear_betas(0.2, 3.0, 20)
        g = np.geomspace(3.0, 0.05, 20)
        Ps = spv.Problem.from_instance(swar)
        sp, E = with_env(env, lambda: spv.spv_sqa_sample(ctx, Ps, b, g, 8, 6, 43))
        osp, oE, _ = oracle.sqa_sample(swar, b, g, 8, reads=6, seed=43)
        assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE), label
    clean = spv.spv_debug_lds_shadow(ctx, reset=True)
    print(json.dumps(dict(phase="clean", **clean)), flush=True)

    # every site in one class: refused by ingest unless the debug switch lets it through
    bad = si.chimera(2, seed=6)
    P = spv.Problem.from_instance(bad)
    P.colour.zero_()
    P.n_colours = 1
    betas = si.linear_betas(0.1, 3.0, 10)
    try:
        spv.spv_sample(ctx, P, betas, 16, 1)
        refused = False
    except spv.SpvError as e:
        refused = e.code == -3  # SPV_ECOLOUR
    say(f"[shadow] one_class: refused without the switch: {refused}")
    with_env({"SPVAR_SHADOW_ALLOW_COLOUR_EDGES": 1}, lambda: spv.spv_sample(ctx, P, betas, 16, 1))
    races = spv.spv_debug_lds_shadow(ctx, reset=True)
    print(json.dumps(dict(phase="one_class", refused=refused, **races)), flush=True)
    say("[shadow] one_class through tempering")
    with_env({"SPVAR_SHADOW_ALLOW_COLOUR_EDGES": 1, "SPVAR_PT_SPLIT": 1, "SPVAR_PT_GROUPS": 1},
             lambda: spv.spv_pt_sample(ctx, P, si.geometric_betas(0.2, 3.0, 4), 1, 1, 5, 2))
    races_pt = spv.spv_debug_lds_shadow(ctx, reset=True)
    print(json.dumps(dict(phase="one_class_pt", **races_pt)), flush=True)


if __name__ == "__main__":
    main()
