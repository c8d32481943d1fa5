"""GPU parity of the multi-start SPVAR driver (Algorithm 2) through the C ABI, bit for
bit against the oracle: fixing and solving energies, fixed values, per-start sizes,
the best energy and the best state, with and without component recombination."""
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
    for key in ("fixing_E", "solving_E", "fixed_mask", "fixed_val"):
        assert np.array_equal(got[key].cpu().numpy(), want[key]), key
    assert np.array_equal(got["info"], want["info"])
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
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_multistart_matches_oracle(spv, ctx, name, make, kw):
    inst = make()
    betas = si.linear_betas(0.1, 3.0, 70)
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
