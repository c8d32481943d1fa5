"""GPU parity of the batched persistent launch: bit-identical to the oracle and to
one spv_sample launch per instance, for every launch shape, with and without
hipGraph replay and the autotuner."""
import numpy as np
import pytest

import oracle
import spvar_inputs as si
from spvar_inputs import configs as cf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spv():
    import paper_1706_07826_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(spv):
    return spv.Context(0)


def _small_batch():
    insts = si.residual_batch(14, parent_M=5, n_min=10, n_max=160, seed=3)
    insts.append(si.chimera(2, seed=4))
    insts.append(si.from_edges(5, [], [], [], [1, -2, 3, -4, 5], np.zeros(5), 1))  # no couplers
    reads = [37, 8, 0, 64, 5, 100, 12, 1, 3, 40, 21, 9, 16, 77, 30, 6]
    seeds = [900 + 7 * b for b in range(len(insts))]
    return insts, reads, seeds


def _as_np(lst):
    return [t.cpu().numpy() for t in lst]


def test_batch_matches_oracle_and_plain(spv, ctx):
    insts, reads, seeds = _small_batch()
    betas = si.linear_betas(0.1, 5.0, 60)
    probs = [spv.Problem.from_instance(i) for i in insts]
    sp, en = spv.spv_sample_batch(ctx, probs, betas, reads, seeds)
    sp, en = _as_np(sp), _as_np(en)
    for b, inst in enumerate(insts):
        osp, oE = oracle.sa_sample(inst, betas, reads=reads[b], seed=seeds[b])
        assert np.array_equal(sp[b], osp), b
        assert np.array_equal(en[b], oE), b
        if reads[b]:
            ps, pe = spv.spv_sample(ctx, probs[b], betas, reads[b], seeds[b])
            assert np.array_equal(ps.cpu().numpy(), sp[b]) and np.array_equal(pe.cpu().numpy(), en[b])


@pytest.mark.parametrize("threads,qpi,wpc", [(64, 1, 1), (256, 3, 2), (512, 8, 1), (1024, 4, 1)])
def test_batch_every_shape_gives_the_same_bits(spv, ctx, threads, qpi, wpc):
    insts, reads, seeds = _small_batch()
    betas = si.linear_betas(0.1, 5.0, 40)
    probs = [spv.Problem.from_instance(i) for i in insts]
    ref_sp, ref_en = spv.spv_sample_batch(ctx, probs, betas, reads, seeds)
    sp, en = spv.spv_sample_batch(ctx, probs, betas, reads, seeds, threads=threads,
                                  quads_per_item=qpi, wgs_per_cu=wpc)
    for a, b in zip(_as_np(ref_sp) + _as_np(ref_en), _as_np(sp) + _as_np(en)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("threads,wpc", [(1024, 1), (512, 1), (256, 4)])
def test_batch_paired_body_matches_oracle_and_one_word_body(spv, ctx, threads, wpc):
    """The paired body (a lane holds both quad words of a pair; an item runs k pairs of one
    instance in separate LDS regions sharing its records) against the oracle and the
    one-word body, ragged read counts included (odd quad counts leave a half-used pair)."""
    insts, reads, seeds = _small_batch()
    betas = si.linear_betas(0.1, 5.0, 50)
    probs = [spv.Problem.from_instance(i) for i in insts]
    print(f"[batch] paired body threads={threads} wgs_per_cu={wpc}", flush=True)
    sp, en = spv.spv_sample_batch(ctx, probs, betas, reads, seeds, threads=threads, wgs_per_cu=wpc, paired=True)
    assert spv.spv_batch_last_shape(ctx)["quads_per_item"] == 0
    one_sp, one_en = spv.spv_sample_batch(ctx, probs, betas, reads, seeds, threads=256, quads_per_item=2,
                                          wgs_per_cu=4)
    for b, inst in enumerate(insts):
        osp, oE = oracle.sa_sample(inst, betas, reads=reads[b], seed=seeds[b])
        assert np.array_equal(sp[b].cpu().numpy(), osp), b
        assert np.array_equal(en[b].cpu().numpy(), oE), b
        assert np.array_equal(one_sp[b].cpu().numpy(), osp) and np.array_equal(one_en[b].cpu().numpy(), oE), b


def test_batch_paired_body_many_pairs_per_item(spv, ctx):
    """Small instances with many reads: items of up to 64 pairs (512 replicas) of one instance,
    sweeps past the table prefetch of both buffers, against the oracle on sampled reads."""
    insts = [si.random_sparse(n, 2.0, seed=70 + n, j_max=3, h_max=3) for n in (12, 30, 47, 64, 90)]
    for i in insts:
        i.colour, i.n_colours = si.greedy_colouring(i)
    degs = [int(np.diff(i.row_ptr).max()) for i in insts]
    assert max(degs) in (4, 6, 8), degs  # the paired body needs padded images of 4, 6 or 8 records
    reads = [1000, 999, 517, 1000, 333]
    seeds = [40 + b for b in range(len(insts))]
    betas = si.linear_betas(0.1, 3.0, 33)
    probs = [spv.Problem.from_instance(i) for i in insts]
    print("[batch] paired body, many pairs per item", flush=True)
    sp, en = spv.spv_sample_batch(ctx, probs, betas, reads, seeds, threads=1024, wgs_per_cu=1, paired=True)
    for b, inst in enumerate(insts):
        s_b, e_b = sp[b].cpu().numpy(), en[b].cpu().numpy()
        assert np.array_equal(e_b, oracle.energy(inst, s_b)), b
        for lo in (0, reads[b] // 2, reads[b] - 9):
            osp, oE = oracle.sa_sample(inst, betas, seed=seeds[b], r_begin=lo, r_end=lo + 9)
            assert np.array_equal(s_b[lo:lo + 9], osp) and np.array_equal(e_b[lo:lo + 9], oE), (b, lo)


def test_batch_graph_replay_and_tuner(spv, ctx):
    insts, reads, seeds = _small_batch()
    betas = si.linear_betas(0.1, 5.0, 40)
    probs = [spv.Problem.from_instance(i) for i in insts]
    want = [oracle.sa_sample(i, betas, reads=r, seed=s) for i, r, s in zip(insts, reads, seeds)]
    # capture, then replay with new seeds and fresh output buffers
    for rep, shift in enumerate([0, 0, 11, 0]):
        sd = [s + shift for s in seeds]
        sp, en = spv.spv_sample_batch(ctx, probs, betas, reads, sd, graph=True)
        sp, en = _as_np(sp), _as_np(en)
        for b, inst in enumerate(insts):
            w = want[b] if shift == 0 else oracle.sa_sample(inst, betas, reads=reads[b], seed=sd[b])
            assert np.array_equal(sp[b], w[0]) and np.array_equal(en[b], w[1]), (rep, b)
    sp, en = spv.spv_sample_batch(ctx, probs, betas, reads, seeds, tune=True)
    shape = spv.spv_batch_last_shape(ctx)
    assert shape["threads"] in (256, 512, 1024) and shape["tuned_ms"] > 0
    for b in range(len(insts)):
        assert np.array_equal(sp[b].cpu().numpy(), want[b][0])


def test_batch_residual_config_full_size_sampled(spv, ctx):
    """512 residual instances, 1000 reads x 1000 sweeps each, one launch; the oracle
    recomputes sampled reads of sampled instances."""
    cfg = cf.RESIDUAL_BATCH
    insts = cf.instance(cfg)
    betas = cf.betas(cfg)
    probs = [spv.Problem.from_instance(i) for i in insts]
    reads = [cfg["reads"]] * len(insts)
    seeds = [cfg["seed"] + b for b in range(len(insts))]
    sp, en = spv.spv_sample_batch(ctx, probs, betas, reads, seeds, graph=True)
    rng = np.random.default_rng(1)
    for b in sorted(set([0, 1, 255, 511] + rng.integers(0, 512, 6).tolist())):
        s_b, e_b = sp[b].cpu().numpy(), en[b].cpu().numpy()
        assert np.array_equal(e_b, oracle.energy(insts[b], s_b)), b
        for r in (0, 999, int(rng.integers(0, 1000))):
            osp, oE = oracle.sa_sample(insts[b], betas, seed=seeds[b], r_begin=r, r_end=r + 1)
            assert np.array_equal(s_b[r], osp[0]) and e_b[r] == oE[0], (b, r)
