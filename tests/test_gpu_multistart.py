"""GPU parity of the multi-start SPVAR driver (Algorithm 2) through the C ABI, bit for
bit against the oracle: correlation, fixing and solving energies, fixed values, per-start
sizes and pivots, the pre-processing info, per-start best energies, the best energy and the
best state; with and without the zero-bias correlation step (before or after the SPVAR step),
the tree pre-processing (before the loop and after each SPVAR step) and component
recombination; SA and SQA as the sampler."""
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


def _run(spv, ctx, inst, betas, **kw):
    P = spv.Problem.from_instance(inst)
    got = spv.spv_multistart(ctx, P, betas, **kw)
    want = oracle.multistart(inst, betas, **kw)
    for key in ("corr_E", "fixing_E", "solving_E", "fixed_mask", "fixed_val"):
        assert np.array_equal(got[key].cpu().numpy(), want[key]), key
    for key in ("info", "info_pre", "start_best"):
        assert np.array_equal(got[key], want[key]), key
    assert got["best_E"] == want["best_E"]
    assert np.array_equal(got["best_spins"].cpu().numpy(), want["best_spins"])
    return got


CASES = [
    ("chimera2_3starts", lambda: si.chimera(2, seed=1), dict(seed=7, starts=3, fixing_reads=40, solving_reads=33,
                                                              elite_frac=0.2, threshold=1.0)),
    ("union_merge", lambda: si.disjoint_union([si.chimera(1, seed=2), si.random_sparse(25, 2.0, seed=3),
                                               si.random_sparse(12, 1.5, seed=4)], perm_seed=2),
     dict(seed=9, starts=4, fixing_reads=50, solving_reads=41, elite_frac=0.1, threshold=0.9, merge=True)),
    ("cubic4_gauge_auto", lambda: si.cubic_lattice(4, "pm1", seed=5),
     dict(seed=11, starts=2, fixing_reads=64, solving_reads=64, elite_frac=0.1, threshold=1.0, gauge=2)),
    ("no_solving_sample", lambda: si.chimera(1, seed=6), dict(seed=13, starts=2, fixing_reads=20, solving_reads=0,
                                                              elite_frac=0.5, threshold=1.0)),
    ("everything_fixed", lambda: si.weak_strong_toy(-50), dict(seed=15, starts=3, fixing_reads=16, solving_reads=8,
                                                               elite_frac=0.1, threshold=0.5)),
    # the zero-bias correlation step with the appendix split (40/30/30 of 100 reads)
    ("cubic4_corr_before", lambda: si.cubic_lattice(4, "pm1", seed=31),
     dict(seed=17, starts=4, corr_reads=40, fixing_reads=30, solving_reads=30, elite_frac=0.2, threshold=1.0,
          corr_elite_frac=0.3)),
    ("cubic4_corr_after", lambda: si.cubic_lattice(4, "pm1", seed=32),
     dict(seed=19, starts=3, corr_reads=40, fixing_reads=30, solving_reads=30, elite_frac=0.2, threshold=1.0,
          corr_elite_frac=0.3, corr_after=1)),
    ("chimera3_h0_corr_merge", lambda: si.chimera(3, seed=33, h_zero=True),
     dict(seed=21, starts=5, corr_reads=37, fixing_reads=29, solving_reads=23, elite_frac=0.2, threshold=1.0,
          corr_elite_frac=0.2, merge=True)),
    ("sparse_h0_corr_theta09", lambda: si.random_sparse(60, 2.5, seed=34, h_zero=True),
     dict(seed=23, starts=3, corr_reads=50, fixing_reads=25, solving_reads=25, elite_frac=0.2, threshold=1.0,
          corr_elite_frac=0.4, corr_threshold=0.9)),
    # tree pre-processing before the loop, after each SPVAR step, and both
    ("tree_before_loop", lambda: si.random_sparse(120, 1.6, seed=35),
     dict(seed=25, starts=3, fixing_reads=30, solving_reads=20, elite_frac=0.2, threshold=1.0, preprocess=1)),
    ("tree_after_spvar", lambda: si.random_sparse(80, 3.0, seed=36),
     dict(seed=27, starts=4, fixing_reads=40, solving_reads=20, elite_frac=0.3, threshold=1.0, preprocess=2)),
    ("tree_both_corr_merge", lambda: si.random_sparse(90, 1.8, seed=37, h_zero=True),
     dict(seed=29, starts=3, corr_reads=30, fixing_reads=20, solving_reads=20, elite_frac=0.2, threshold=1.0,
          corr_elite_frac=0.3, preprocess=3, merge=True)),
    ("tree_both_corr_after", lambda: si.random_sparse(90, 1.8, seed=38, h_zero=True),
     dict(seed=31, starts=2, corr_reads=30, fixing_reads=20, solving_reads=20, elite_frac=0.2, threshold=1.0,
          corr_elite_frac=0.3, corr_after=1, preprocess=3)),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_multistart_matches_oracle(spv, ctx, name, make, kw):
    inst = make()
    # a hot schedule for the tree-after-SPVAR case, so the SPVAR step leaves a core with trees on it
    betas = si.linear_betas(0.1, 1.0, 20) if name == "tree_after_spvar" else si.linear_betas(0.1, 3.0, 70)
    print(f"[multistart] {name} n={inst.n}", flush=True)
    _run(spv, ctx, inst, betas, **kw)


def test_multistart_chimera8_paper_parameters(spv, ctx):
    """The Chimera N=512 workload with parameters in the paper's ranges (10 starts, samples
    of a few hundred, elite 5 %), a short schedule so the oracle finishes quickly."""
    inst = cf.instance(cf.CHIMERA8_SA)
    betas = si.linear_betas(0.1, 5.0, 100)
    got = _run(spv, ctx, inst, betas, seed=2002, starts=10, fixing_reads=200, solving_reads=100,
               elite_frac=0.05, threshold=0.95, merge=True)
    assert got["best_E"] == int(oracle.energy(inst, got["best_spins"].cpu().numpy()[None])[0])


SQA_CASES = [
    ("chimera2_sqa_3starts", lambda: si.chimera(2, seed=21), 8,
     dict(seed=23, starts=3, fixing_reads=24, solving_reads=17, elite_frac=0.25, threshold=1.0)),
    ("union_sqa_merge_P16", lambda: si.disjoint_union([si.chimera(1, seed=22), si.random_sparse(20, 2.0, seed=23)],
                                                      perm_seed=4), 16,
     dict(seed=25, starts=2, fixing_reads=20, solving_reads=13, elite_frac=0.2, threshold=1.0, merge=True)),
    ("cubic4_sqa_gauge_auto", lambda: si.cubic_lattice(4, "pm1", seed=24), 8,
     dict(seed=27, starts=2, fixing_reads=32, solving_reads=9, elite_frac=0.1, threshold=1.0, gauge=2)),
    ("cubic4_sqa_corr_tree", lambda: si.cubic_lattice(4, "pm1", seed=25), 8,
     dict(seed=29, starts=3, corr_reads=24, fixing_reads=16, solving_reads=11, elite_frac=0.2, threshold=1.0,
          corr_elite_frac=0.3, preprocess=2)),
]


@pytest.mark.parametrize("name,make,P,kw", SQA_CASES, ids=[c[0] for c in SQA_CASES])
def test_multistart_with_sqa_matches_oracle(spv, ctx, name, make, P, kw):
    """SQA as the driver's sampler (both samples): every recorded quantity bit for bit."""
    inst = make()
    betas, gammas = si.linear_betas(0.2, 3.0, 40), np.geomspace(3.0, 0.05, 40)
    print(f"[multistart] {name} n={inst.n} P={P}", flush=True)
    _run(spv, ctx, inst, betas, gammas=gammas, trotter=P, **kw)


def test_multistart_sqa_workload_size_sampled(spv, ctx):
    """The multistart_sqa workload as the benchmark launches it (Chimera 8x8, 20 starts x (1000 +
    1000 reads) x 2000 sweeps, 16 slices): sampled fixing rows of the first and last starts
    recomputed by the oracle, and the best state's energy re-evaluated."""
    inst = cf.instance(cf.CHIMERA8_SA)
    betas = cf.betas(cf.CHIMERA8_SA)
    gammas = np.geomspace(3.0, 0.01, betas.size)
    cfg = cf.CHIMERA8_SA
    print("[multistart] SQA workload size", flush=True)
    got = spv.spv_multistart(ctx, spv.Problem.from_instance(inst), betas, cfg["seed"], 20, 1000, 1000, cfg["elite"],
                             cfg["theta"], cfg["gauge"], merge=True, gammas=gammas, trotter=16)
    fE = got["fixing_E"].cpu().numpy()
    for s, r in ((0, 0), (0, 999), (19, 500)):
        _, oE, _ = oracle.sqa_sample(inst, betas, gammas, 16, seed=cfg["seed"], r_begin=1000 * s + r,
                                     r_end=1000 * s + r + 1)
        assert fE[s, r] == oE[0], (s, r)
    best = got["best_spins"].cpu().numpy()
    assert got["best_E"] == int(oracle.energy(inst, best[None])[0])
    allE = np.concatenate([fE.ravel(), got["solving_E"].cpu().numpy().ravel()])
    assert got["best_E"] == allE.min()


def test_multistart_zero_bias_chimera8_appendix_split(spv, ctx):
    """A zero-bias Chimera 8x8 instance with the appendix's parameters for such problems: 20
    starts, a total of 1000 reads per start split 400/300/300, elite thresholds 0.2 and 0.2,
    fixing threshold 1.0 (a short schedule so the oracle finishes quickly)."""
    inst = si.chimera(8, seed=41, h_zero=True)
    c, f, s_ = spv.spv_multistart_split(1000, True)
    assert (c, f, s_) == oracle.ms_split(1000, True) == (400, 300, 300)
    betas = si.linear_betas(0.1, 5.0, 60)
    got = _run(spv, ctx, inst, betas, seed=4001, starts=20, corr_reads=c, fixing_reads=f, solving_reads=s_,
               elite_frac=0.2, threshold=1.0, corr_elite_frac=0.2, merge=True)
    assert np.all(got["info"][:, 0] >= 1)


def test_multistart_rejects_bad_arguments(spv, ctx):
    inst = si.chimera(1, seed=42)
    P = spv.Problem.from_instance(inst)
    b = si.linear_betas(0.1, 3.0, 10)
    for kw in (dict(corr_reads=10, corr_elite_frac=0.0), dict(corr_reads=10, corr_threshold=1.5),
               dict(corr_after=2), dict(preprocess=4), dict(starts=0), dict(starts=4097)):
        args = dict(seed=1, starts=2, fixing_reads=8, solving_reads=4, elite_frac=0.5, threshold=1.0)
        args.update(kw)
        with pytest.raises(spv.SpvError) as e:
            spv.spv_multistart(ctx, P, b, **args)
        assert e.value.code == -1


def test_r99_of_a_device_run_against_brute_force(spv, ctx):
    """R99 (Sec. III.A) from a device run on a 14-variable instance whose ground energy is known
    by brute force: the library's and the oracle's R99 agree, and p is the share of starts whose
    records reach the ground energy."""
    from ._brute import ground
    inst = si.random_sparse(14, 2.5, seed=60)
    g = int(ground(inst)[1].min())
    betas = si.linear_betas(0.1, 1.0, 2)
    got = _run(spv, ctx, inst, betas, seed=0, starts=16, fixing_reads=2, solving_reads=2, elite_frac=0.5,
               threshold=1.0)
    v, p = spv.spv_r99(got["start_best"], g, 4)
    assert (v, p) == oracle.r99(got["start_best"], g, 4)
    assert 0 < p < 1 and p == np.mean(got["start_best"] <= g)
