"""Pins of the oracle's multi-start SPVAR driver (Algorithm 2): the recorded energies
are full-problem energies of real states, the fixing samples are the stated read
ranges of one SA job, a start that fixes nothing reduces to plain SA with the
solving seed, and on small instances the best state reaches the brute-force ground
state."""
import itertools

import numpy as np
import pytest

import oracle
import spvar_inputs as si


def _brute_ground(inst):
    best = None
    for bits in itertools.product((-1, 1), repeat=inst.n):
        e = int(oracle.energy(inst, np.array(bits, np.int8)[None])[0])
        best = e if best is None or e < best else best
    return best


@pytest.mark.parametrize("merge", [False, True])
def test_best_state_energy_and_fixing_ranges(merge):
    inst = si.disjoint_union([si.chimera(1, seed=3), si.random_sparse(20, 2.0, seed=4)], perm_seed=1)
    betas = si.linear_betas(0.1, 3.0, 60)
    out = oracle.multistart(inst, betas, seed=77, starts=3, fixing_reads=40, solving_reads=30, elite_frac=0.2,
                            threshold=1.0, gauge=0, merge=merge)
    # the best state is a real state of the full problem with the recorded energy
    assert out["best_E"] == int(oracle.energy(inst, out["best_spins"][None])[0])
    allE = np.concatenate([out["fixing_E"].ravel(), out["solving_E"].ravel()])
    assert out["best_E"] == allE.min()
    # the fixing samples are reads [s*F, (s+1)*F) of one SA job
    for s in range(3):
        _, E = oracle.sa_sample(inst, betas, seed=77, r_begin=40 * s, r_end=40 * (s + 1))
        assert np.array_equal(out["fixing_E"][s], E)
    # every variable is either fixed or free in each start
    assert np.all(out["info"][:, 1] + out["info"][:, 0] == inst.n)


def test_start_that_fixes_nothing_is_plain_sa():
    """With beta = 0 the fixing rows are random, so no variable is unanimous among 64 elite
    rows; the solving sample is then SA on the full problem with seed + 1 + s."""
    inst = si.chimera(2, seed=9)
    betas = np.zeros(30)
    out = oracle.multistart(inst, betas, seed=5, starts=2, fixing_reads=64, solving_reads=25, elite_frac=1.0,
                            threshold=1.0)
    assert np.all(out["info"][:, 0] == 0) and np.all(out["info"][:, 2] == 0)
    for s in range(2):
        _, E = oracle.sa_sample(inst, betas, seed=5 + 1 + s, reads=25)
        assert np.array_equal(out["solving_E"][s], E)


def test_solving_energies_are_offset_residual_energies():
    """Solving energies = E' + offset: check against the reduced problem of each start sampled
    with the solving seed (the reduction itself is pinned elsewhere)."""
    inst = si.chimera(2, seed=11)
    betas = si.linear_betas(0.1, 3.0, 80)
    out = oracle.multistart(inst, betas, seed=21, starts=2, fixing_reads=50, solving_reads=20, elite_frac=0.2,
                            threshold=0.9)
    for s in range(2):
        S, E = oracle.sa_sample(inst, betas, seed=21, r_begin=50 * s, r_end=50 * (s + 1))
        fx = oracle.persist_fix(inst, S, E, 0.2, 0.9, 0)
        assert np.array_equal(out["fixed_mask"][s], fx["fixed_mask"])
        assert out["info"][s, 2] == fx["offset"]
        if fx["n_free"]:
            _, E2 = oracle.sa_sample(fx["reduced"], betas, seed=21 + 1 + s, reads=20)
            assert np.array_equal(out["solving_E"][s], E2 + fx["offset"])


@pytest.mark.parametrize("seed", range(3))
def test_reaches_brute_force_ground_state(seed):
    inst = si.random_sparse(14, 2.5, seed=30 + seed)
    ground = _brute_ground(inst)
    betas = si.linear_betas(0.1, 4.0, 200)
    out = oracle.multistart(inst, betas, seed=seed, starts=4, fixing_reads=32, solving_reads=32, elite_frac=0.25,
                            threshold=1.0)
    assert out["best_E"] == ground
    assert int(oracle.energy(inst, out["best_spins"][None])[0]) == ground


def test_recombination_never_worsens_the_best_solving_energy():
    inst = si.disjoint_union([si.random_sparse(12, 2.0, seed=40 + k) for k in range(4)], perm_seed=3)
    betas = si.linear_betas(0.1, 1.0, 15)   # a hot, short schedule: components rarely all solved at once
    a = oracle.multistart(inst, betas, seed=8, starts=3, fixing_reads=40, solving_reads=40, elite_frac=0.1,
                          threshold=1.0, merge=False)
    b = oracle.multistart(inst, betas, seed=8, starts=3, fixing_reads=40, solving_reads=40, elite_frac=0.1,
                          threshold=1.0, merge=True)
    assert np.array_equal(a["fixing_E"], b["fixing_E"])
    assert np.all(b["solving_E"].min(axis=1) <= a["solving_E"].min(axis=1))
    assert np.all(np.diff(b["solving_E"], axis=1) >= 0)


# ------------------------------------------------ SQA as the sampler (SQA_SPVAR) --
@pytest.mark.parametrize("merge", [False, True])
def test_sqa_driver_records_real_states_and_its_own_samples(merge):
    """With SQA as the sampler: the best state is a real state with the recorded energy, the
    fixing energies are reads [s*F, (s+1)*F) of one SQA job, and the solving energies are SQA
    jobs on each start's reduced problem (seed + 1 + s) plus its offset."""
    inst = si.disjoint_union([si.chimera(1, seed=5), si.random_sparse(16, 2.0, seed=6)], perm_seed=2)
    b, g = si.linear_betas(0.2, 3.0, 50), np.geomspace(3.0, 0.05, 50)
    out = oracle.multistart(inst, b, seed=13, starts=3, fixing_reads=24, solving_reads=16, elite_frac=0.25,
                            threshold=1.0, merge=merge, gammas=g, trotter=8)
    assert out["best_E"] == int(oracle.energy(inst, out["best_spins"][None])[0])
    assert out["best_E"] == np.concatenate([out["fixing_E"].ravel(), out["solving_E"].ravel()]).min()
    for s in range(3):
        S, E, _ = oracle.sqa_sample(inst, b, g, 8, seed=13, r_begin=24 * s, r_end=24 * (s + 1))
        assert np.array_equal(out["fixing_E"][s], E)
        if not merge:
            fx = oracle.persist_fix(inst, S, E, 0.25, 1.0, 0)
            assert np.array_equal(out["fixed_mask"][s], fx["fixed_mask"])
            if fx["n_free"]:
                _, E2, _ = oracle.sqa_sample(fx["reduced"], b, g, 8, seed=13 + 1 + s, reads=16)
                assert np.array_equal(out["solving_E"][s], E2 + fx["offset"])


@pytest.mark.parametrize("seed", range(2))
def test_sqa_driver_reaches_brute_force_ground_state(seed):
    inst = si.random_sparse(14, 2.5, seed=50 + seed)
    ground = _brute_ground(inst)
    sw = 200
    out = oracle.multistart(inst, si.linear_betas(0.1, 4.0, sw), seed=seed, starts=3, fixing_reads=16,
                            solving_reads=16, elite_frac=0.25, threshold=1.0, gammas=np.geomspace(3.0, 0.02, sw),
                            trotter=8)
    assert out["best_E"] == ground
