"""Pins of the oracle's multi-start SPVAR driver (Algorithm 2, the zero-bias handling of
Sec. II.C and the sample split of the parameter appendix): the recorded energies are
full-problem energies of real states; the first stage samples the stated read ranges of one
job; a start that fixes nothing reduces to plain SA with its stage seed; the correlation step
fixes exactly the pivot's class of perfectly (anti)correlated variables, re-derived here from
the elite columns; the split matches the appendix's 40/30/30 and 50/50 shares; R99 follows the
benchmarking procedure of Sec. III.A by hand; and on small instances the best state reaches the
brute-force ground state, with the tree pre-processing on or off."""
import math

import numpy as np
import pytest

import oracle
import spvar_inputs as si

from ._brute import ground as _dense_ground


def _brute_ground(inst):
    _, E = _dense_ground(inst)
    return int(E.min())


def _elite_rows(E, frac):
    m = max(1, math.ceil(frac * len(E)))
    return sorted(range(len(E)), key=lambda r: (int(E[r]), r))[:m]


# ------------------------------------------------------------- sample split --
@pytest.mark.parametrize("total,zero_bias,want", [
    (500, True, (200, 150, 150)), (1000, True, (400, 300, 300)), (100, True, (40, 30, 30)),
    (500, False, (0, 250, 250)), (1000, False, (0, 500, 500)), (7, True, (2, 3, 2)), (7, False, (0, 4, 3)),
    (1, True, (0, 1, 0)), (0, True, (0, 0, 0)),
])
def test_sample_split_matches_the_appendix(total, zero_bias, want):
    assert oracle.ms_split(total, zero_bias) == want


def test_sample_split_always_sums_to_the_total():
    for t in range(0, 300):
        for zb in (False, True):
            c, f, s = oracle.ms_split(t, zb)
            assert c + f + s == t and f >= s >= 0 and (zb or c == 0)
            if zb and t % 10 == 0:
                assert (c, f, s) == (4 * t // 10, 3 * t // 10, 3 * t // 10)


# ------------------------------------------------------------------- R99 --
def test_r99_by_hand():
    T = 100.0
    v, p = oracle.r99([1, 2, 1, 5], 1, T)        # 2 of 4 starts reach the target
    assert p == 0.5 and v == pytest.approx(T * math.log(0.01) / math.log(0.5))
    assert v == pytest.approx(664.3856189774724)
    v, p = oracle.r99([3, 3, 0, 3], 0, T)        # 1 of 4
    assert p == 0.25 and v == pytest.approx(T * 16.0078455593)  # -4.605170 / -0.287682
    v, p = oracle.r99([0, -1, 0], 0, T)          # every start (<= counts: a lower energy also reaches it)
    assert p == 1.0 and v == T
    v, p = oracle.r99([0] * 199 + [1], 0, T)     # p = 0.995 >= 0.99: one start suffices
    assert p == 0.995 and v == T
    v, p = oracle.r99([4, 5], 3, T)              # never: not measurable
    assert p == 0.0 and v == -1.0


@pytest.mark.parametrize("seed", range(2))
def test_r99_against_brute_force_ground_truth(seed):
    """R99 of a run on a 14-variable instance whose ground energy is known by brute force: the
    success fraction is the share of starts whose records reach it, and R99 = n99 x the total
    sample of one start."""
    inst = si.random_sparse(14, 2.5, seed=60 + seed)
    g = _brute_ground(inst)
    # two sweeps and two reads per stage: some starts miss the ground state (0 < p < 1)
    out = oracle.multistart(inst, si.linear_betas(0.1, 1.0, 2), seed=seed, starts=16, fixing_reads=2,
                            solving_reads=2, elite_frac=0.5, threshold=1.0)
    allE = np.concatenate([out["fixing_E"], out["solving_E"]], axis=1)
    assert np.array_equal(out["start_best"], allE.min(axis=1))
    hits = sum(int(allE[s].min()) == g for s in range(16))
    assert 0 < hits < 16
    v, p = oracle.r99(out["start_best"], g, 4)
    assert p == hits / 16
    assert v == pytest.approx(4 * max(1.0, math.log(0.01) / math.log(1 - hits / 16)))


# ----------------------------------------------------- recorded energies --
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
    assert np.all(out["info"][:, 1] + out["info"][:, 3] == inst.n)
    assert np.all(out["info"][:, 0] == 0) and np.all(out["info"][:, 6] == -1)


def test_start_that_fixes_nothing_is_plain_sa():
    """With beta = 0 the fixing rows are random, so no variable is unanimous among 64 elite
    rows; the solving sample is then SA on the full problem with seed + 1 + s."""
    inst = si.chimera(2, seed=9)
    betas = np.zeros(30)
    out = oracle.multistart(inst, betas, seed=5, starts=2, fixing_reads=64, solving_reads=25, elite_frac=1.0,
                            threshold=1.0)
    assert np.all(out["info"][:, 1] == 0) and np.all(out["info"][:, 4] == 0)
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
        assert out["info"][s, 4] == fx["offset"]
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


# -------------------------------------------- the zero-bias correlation step --
def _pivot_class(S_elite):
    """Classes of variables whose elite columns agree up to a global sign; the pivot is the
    lowest index of the largest class (ties: the class holding the lower index).  Written
    from the definition with plain Python loops."""
    n = S_elite.shape[1]
    cls = {}
    for j in range(n):
        col = S_elite[:, j]
        key = tuple(int(v) * int(col[0]) for v in col)
        cls.setdefault(key, []).append(j)
    groups = sorted(cls.values(), key=lambda g: (-len(g), min(g)))
    return groups[0]


@pytest.mark.parametrize("seed", range(3))
def test_correlation_step_fixes_the_pivot_class(seed):
    """h = 0: the correlation step (its own sample: reads [s*Rc, (s+1)*Rc) of one job) fixes
    exactly the pivot's class, the pivot to +1 and each member j to s_j * s_pivot of any elite
    row; its energies are that job's."""
    inst = si.cubic_lattice(4, "pm1", seed=70 + seed)
    betas = si.linear_betas(0.1, 2.0, 60)
    Rc, ce = 40, 0.3
    out = oracle.multistart(inst, betas, seed=seed, starts=3, fixing_reads=20, solving_reads=10, elite_frac=0.2,
                            threshold=1.0, corr_reads=Rc, corr_elite_frac=ce, corr_threshold=1.0)
    for s in range(3):
        S, E = oracle.sa_sample(inst, betas, seed=seed, r_begin=Rc * s, r_end=Rc * (s + 1))
        assert np.array_equal(out["corr_E"][s], E)
        Se = S[_elite_rows(E, ce)].astype(np.int64)
        members = _pivot_class(Se)
        piv = members[0]
        assert out["info"][s, 6] == piv and out["info"][s, 0] == len(members)
        want = {j: int(Se[0, j] * Se[0, piv]) for j in members}
        assert want[piv] == 1
        for j, v in want.items():
            assert out["fixed_mask"][s][j] == 1 and out["fixed_val"][s][j] == v
        # the SPVAR step then fixes more from the now-biased residual (never fewer in total)
        assert out["info"][s, 0] + out["info"][s, 1] == int(out["fixed_mask"][s].sum())


def test_correlation_step_after_spvar_uses_the_later_seed():
    """corr_after = 1 (the order of the algorithm box): the SPVAR step samples first (one job,
    seed), then the correlation step samples the SPVAR-modified problem with seed + 1 + s and the
    solving step with seed + 1 + starts + s."""
    inst = si.cubic_lattice(4, "pm1", seed=80)
    betas = si.linear_betas(0.1, 2.0, 50)
    out = oracle.multistart(inst, betas, seed=3, starts=2, fixing_reads=30, solving_reads=10, elite_frac=0.2,
                            threshold=1.0, gauge=0, corr_reads=30, corr_elite_frac=0.3, corr_after=1)
    for s in range(2):
        S, E = oracle.sa_sample(inst, betas, seed=3, r_begin=30 * s, r_end=30 * (s + 1))
        assert np.array_equal(out["fixing_E"][s], E)
        fx = oracle.persist_fix(inst, S, E, 0.2, 1.0, 0)
        red = fx["reduced"] if fx["n_free"] < inst.n else inst
        S2, E2 = oracle.sa_sample(red, betas, seed=3 + 1 + s, reads=30)
        assert np.array_equal(out["corr_E"][s], E2 + fx["offset"])
        fx2 = oracle.persist_fix(red, S2, E2, 0.3, 1.0, 1)
        if fx2["n_free"]:
            _, E3 = oracle.sa_sample(fx2["reduced"], betas, seed=3 + 1 + 2 + s, reads=10)
            assert np.array_equal(out["solving_E"][s], E3 + fx["offset"] + fx2["offset"])


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("corr_after", [0, 1])
def test_zero_bias_driver_reaches_brute_force_ground_state(seed, corr_after):
    """h = 0 instances of 14 variables with the appendix split of 100 reads per start
    (40/30/30): the best recorded state is a brute-force ground state."""
    inst = si.random_sparse(14, 2.5, seed=90 + seed, h_zero=True)
    ground = _brute_ground(inst)
    c, f, s = oracle.ms_split(100, True)
    out = oracle.multistart(inst, si.linear_betas(0.1, 4.0, 150), seed=seed, starts=4, fixing_reads=f,
                            solving_reads=s, elite_frac=0.2, threshold=1.0, corr_reads=c, corr_elite_frac=0.3,
                            corr_after=corr_after)
    assert out["best_E"] == ground
    assert int(oracle.energy(inst, out["best_spins"][None])[0]) == ground
    assert np.all(out["info"][:, 0] >= 1)  # the pivot at least


# --------------------------------------------------- tree pre-processing --
@pytest.mark.parametrize("preprocess", [1, 2, 3])
def test_tree_preprocessing_keeps_real_states_and_ground_energy(preprocess):
    """Trees hanging off a small cycle (the tree step removes them exactly): with the
    pre-processing before the loop, after each SPVAR step, or both, every recorded best state is
    a real state whose energy is the record, and the brute-force ground energy is reached."""
    rng = np.random.default_rng(5)
    n = 16
    ei, ej = [0, 1, 2, 3], [1, 2, 3, 0]              # a 4-cycle
    for v in range(4, n):                           # each new vertex hangs off an earlier one
        ei.append(int(rng.integers(0, v)))
        ej.append(v)
    w = rng.choice([-3, -2, -1, 1, 2, 3], size=len(ei))
    h = rng.choice([-2, -1, 0, 1, 2], size=n)
    inst = si.from_edges(n, np.array(ei), np.array(ej), w, h, np.zeros(n, np.uint8), 1)
    inst.colour, inst.n_colours = si.greedy_colouring(inst)
    ground = _brute_ground(inst)
    out = oracle.multistart(inst, si.linear_betas(0.1, 3.0, 80), seed=4, starts=3, fixing_reads=20,
                            solving_reads=20, elite_frac=0.2, threshold=1.0, preprocess=preprocess)
    assert out["best_E"] == int(oracle.energy(inst, out["best_spins"][None])[0])
    assert out["best_E"] == ground
    if preprocess & 1:
        assert out["info_pre"][0] == 4 and out["info_pre"][3] + out["info_pre"][4] == n - 4


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
