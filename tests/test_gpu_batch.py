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
