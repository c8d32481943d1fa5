"""Full-size parity of the five workloads through the C ABI, against the oracle run on the host's
threads: the Chimera 8x8 SA sample (all 10,000 reads x 2,000 sweeps) and its persistence; the
L=10 cube's 64 tempering runs x 10^4 sweeps (final states, every top-10 list) and persistence on
the 10,240-row top-10 sample; one full N=8000 PT-ICM run (10^4 sweeps, final states, every top-10
list, persistence); and the residual batch by the subset rule: every read of 64 instances drawn
at random and the first 16 reads of every other instance, with every energy equal to its state's.
The iterated cubic L=4 workload runs in full in test_gpu_sa.py."""
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from spvar_inputs import configs as cf

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def spv():
    import paper_1706_07826_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(spv):
    return spv.Context(0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same_fix(fx, want):
    info = fx.info()
    assert info["n_free"] == want["n_free"] and info["offset"] == want["offset"]
    assert np.array_equal(fx.fixed_mask.cpu().numpy(), want["fixed_mask"])
    assert np.array_equal(fx.fixed_val.cpu().numpy(), want["fixed_val"])
    red = fx.reduced()
    r = want["reduced"]
    assert np.array_equal(red.row_ptr.cpu().numpy(), r.row_ptr)
    assert np.array_equal(red.col[:red.nnz].cpu().numpy(), r.col)
    assert np.array_equal(red.J[:red.nnz].cpu().numpy(), r.J)
    assert np.array_equal(red.h[:red.n].cpu().numpy(), r.h)
    assert np.array_equal(fx.orig_index.cpu().numpy(), want["orig_index"])


def test_config2_chimera8_every_read_and_persistence(spv, ctx):
    cfg = cf.CHIMERA8_SA
    inst, betas = cf.instance(cfg), cf.betas(cfg)
    P = spv.Problem.from_instance(inst)
    _say(f"[full] chimera8_sa: {cfg['reads']} reads x {cfg['sweeps']} sweeps; oracle on {THREADS} threads")
    S, E = spv.spv_sample(ctx, P, betas, cfg["reads"], cfg["seed"])
    t0 = time.time()
    osp, oE = oracle.sa_sample(inst, betas, reads=cfg["reads"], seed=cfg["seed"], threads=THREADS)
    _say(f"[full] chimera8_sa oracle {time.time() - t0:.1f} s")
    assert np.array_equal(S.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)
    fx = spv.spv_persist_fix(ctx, P, S, E, cfg["elite"], cfg["theta"], cfg["gauge"])
    _same_fix(fx, oracle.persist_fix(inst, osp, oE, cfg["elite"], cfg["theta"], cfg["gauge"]))


def test_config3_cubic10_every_run_and_persistence(spv, ctx):
    cfg = cf.CUBIC10_PT
    inst, betas = cf.instance(cfg), cf.betas(cfg)
    P = spv.Problem.from_instance(inst)
    runs, sweeps = cfg["runs"], cfg["sweeps"]
    _say(f"[full] cubic10_pt: {runs} runs x {betas.size} slots x {sweeps} sweeps; oracle on {THREADS} threads")
    got = spv.spv_pt_sample(ctx, P, betas, runs, 1, sweeps, cfg["seed"])
    t0 = time.time()
    want = oracle.pt_sample(inst, betas, runs, 1, sweeps, seed=cfg["seed"], threads=THREADS)
    _say(f"[full] cubic10_pt oracle {time.time() - t0:.1f} s")
    for key in ("final_spins", "final_E", "top_E", "top_count", "top_spins"):
        assert np.array_equal(got[key].cpu().numpy(), want[key]), key
    S, E = spv.spv_top_sample(ctx, got)
    oS, oE = oracle.top_sample(want)
    assert S.shape[0] == oS.shape[0] == runs * (betas.size // 2) * 10
    assert np.array_equal(S.cpu().numpy(), oS) and np.array_equal(E.cpu().numpy(), oE)
    fx = spv.spv_persist_fix(ctx, P, S, E, cfg["elite"], cfg["theta"], cfg["gauge"])
    _same_fix(fx, oracle.persist_fix(inst, oS, oE, cfg["elite"], cfg["theta"], cfg["gauge"]))


def test_config5_cubic20_pticm_full_run_and_persistence(spv, ctx):
    cfg = cf.CUBIC20_PTICM
    inst, betas = cf.instance(cfg), cf.betas(cfg)
    K = betas.size
    P = spv.Problem.from_instance(inst)
    _say(f"[full] cubic20_pticm: 1 run x 2 chains x {K} slots x {cfg['sweeps']} sweeps, cluster moves at every "
         f"slot; oracle slots on {THREADS} threads")
    got = spv.spv_pt_sample(ctx, P, betas, 1, 2, cfg["sweeps"], cfg["seed"], icm=(0, K))
    t0 = time.time()
    oracle.set_slot_threads(THREADS)
    try:
        want = oracle.pt_sample(inst, betas, 1, 2, cfg["sweeps"], seed=cfg["seed"], icm=(0, K))
    finally:
        oracle.set_slot_threads(1)
    _say(f"[full] cubic20_pticm oracle {time.time() - t0:.1f} s")
    for key in ("final_spins", "final_E", "top_E", "top_count", "top_spins"):
        assert np.array_equal(got[key].cpu().numpy(), want[key]), key
    S, E = spv.spv_top_sample(ctx, got)
    oS, oE = oracle.top_sample(want)
    assert np.array_equal(S.cpu().numpy(), oS) and np.array_equal(E.cpu().numpy(), oE)
    fx = spv.spv_persist_fix(ctx, P, S, E, cfg["elite"], cfg["theta"], cfg["gauge"])
    _same_fix(fx, oracle.persist_fix(inst, oS, oE, cfg["elite"], cfg["theta"], cfg["gauge"]))


def test_config4_residual_batch_subset_rule(spv, ctx):
    cfg = cf.RESIDUAL_BATCH
    insts, betas = cf.instance(cfg), cf.betas(cfg)
    B, R = len(insts), cfg["reads"]
    probs = [spv.Problem.from_instance(i) for i in insts]
    seeds = [cfg["seed"] + b for b in range(B)]
    _say(f"[full] residual_batch: {B} instances x {R} reads x {cfg['sweeps']} sweeps (graph-replayed default shape)")
    sp, en = spv.spv_sample_batch(ctx, probs, betas, [R] * B, seeds, graph=True)
    full = set(np.random.default_rng(4).choice(B, 64, replace=False).tolist())
    got = [(sp[b].cpu().numpy(), en[b].cpu().numpy()) for b in range(B)]

    def one(b):
        r_end = R if b in full else 16
        return oracle.sa_sample(insts[b], betas, seed=seeds[b], r_begin=0, r_end=r_end, threads=1)

    t0 = time.time()
    with ThreadPoolExecutor(THREADS) as ex:
        want = list(ex.map(one, range(B)))
    _say(f"[full] residual_batch oracle {time.time() - t0:.1f} s")
    for b in range(B):
        s_b, e_b = got[b]
        osp, oE = want[b]
        k = osp.shape[0]
        assert np.array_equal(s_b[:k], osp) and np.array_equal(e_b[:k], oE), b
        assert np.array_equal(e_b, oracle.energy(insts[b], s_b)), b
