"""Pins of the oracle's persistence step (Algorithm 1) and reduction.

* Exhaustive energy consistency of the reduction: E(s) = E'(s_U) + offset for
  every completion of the fixed values (brute force, N <= 14).
* Hand-made samples whose elite set, counts and fixes are known by
  construction (elite size rounding, (E, row) tie-break, threshold).
* Unanimous samples fix everything; the reduced problem is empty.
* Zero bias (Sec. II.C): a sample made of states and their reversals fixes
  nothing without the gauge, and fixes the pivot's correlated cluster with it.
* Gauge covariance: relabelling s_i -> tau_i s_i of problem and sample maps the
  fixes to tau_i v_i and leaves the offset unchanged.
"""
import numpy as np
import pytest

import oracle
import spvar_inputs as si
from tests import _brute


def _completions_check(inst, res):
    red, fm, fv = res["reduced"], res["fixed_mask"].astype(bool), res["fixed_val"]
    free = np.nonzero(~fm)[0]
    assert np.array_equal(res["orig_index"], free)
    S_red = _brute.all_states(red.n) if red.n <= 14 else si.random_spins(4096, red.n, seed=1)
    full = np.zeros((S_red.shape[0], inst.n), np.int8)
    full[:, fm] = fv[fm]
    full[:, free] = S_red
    lhs = _brute.energies(inst, full)
    rhs = _brute.energies(red, S_red) + res["offset"]
    assert np.array_equal(lhs, rhs)


@pytest.mark.parametrize("seed", range(4))
def test_reduction_energy_is_exact_for_every_completion(seed):
    inst = si.random_sparse(18, 3.5, seed=100 + seed)
    spins, E = oracle.sa_sample(inst, si.linear_betas(0.05, 0.4, 10), reads=64, seed=seed)
    res = oracle.persist_fix(inst, spins, E, 0.5, 0.9, gauge=0)
    assert 0 < res["n_fixed"] < inst.n
    assert res["reduced"].n == inst.n - res["n_fixed"]
    _completions_check(inst, res)


def test_reduced_csr_is_symmetric_sorted_and_coloured():
    inst = si.chimera(3, seed=4)
    spins, E = oracle.sa_sample(inst, si.linear_betas(0.1, 5.0, 300), reads=200, seed=3)
    res = oracle.persist_fix(inst, spins, E, 0.1, 1.0)
    red = res["reduced"]
    Jd = _brute.dense(red)
    assert np.array_equal(Jd, Jd.T)
    for u in range(red.n):
        c = red.col[red.row_ptr[u]:red.row_ptr[u + 1]]
        assert np.all(np.diff(c) > 0)
        assert np.all(red.colour[c] != red.colour[u])
    assert np.array_equal(red.colour, inst.colour[res["orig_index"]])
    orig = res["orig_index"]
    full_J = _brute.dense(inst)
    assert np.array_equal(Jd, full_J[np.ix_(orig, orig)])


def test_elite_rounding_ties_and_threshold_by_construction():
    inst = si.random_sparse(5, 2.0, seed=7)
    # 10 rows; elite 0.25 -> m = ceil(2.5) = 3; rows 2, 5, 7 share the lowest
    # energy, rows 1 and 8 the next one.  Elite = {2, 5, 7} regardless of
    # any other row.  Variable 0 is +1 in all of them, variable 1 is +1 in two
    # of three (|c| = 1), variable 2 is -1 in all.
    S = -np.ones((10, 5), np.int8)
    S[[2, 5, 7], 0] = 1
    S[[2, 5], 1] = 1
    S[:, 3] = np.array([1, -1] * 5)
    S[[2, 5, 7], 4] = [1, -1, 1]
    S[[0, 1, 3, 4, 6, 8, 9], 2] = 1  # non-elite rows disagree on variable 2
    E = np.array([5, 3, -9, 4, 7, -9, 8, -9, 3, 6], np.int64)
    r = oracle.persist_fix(inst, S, E, 0.25, 1.0)
    assert r["m"] == 3 and r["k_min"] == 3
    assert r["fixed_mask"].tolist() == [1, 0, 1, 0, 0]
    assert r["fixed_val"].tolist() == [1, 0, -1, 0, 0]
    # theta = 0.3 -> k_min = ceil(0.9) = 1: every variable with a nonzero sum
    r = oracle.persist_fix(inst, S, E, 0.25, 0.3)
    assert r["k_min"] == 1
    assert r["fixed_mask"].tolist() == [1, 1, 1, 1, 1]
    assert r["fixed_val"].tolist() == [1, 1, -1, -1, 1]
    # a fourth tied row at index 9 does not enter: (E, row) order
    E2 = E.copy()
    E2[9] = -9
    r = oracle.persist_fix(inst, S, E2, 0.25, 1.0)
    assert r["fixed_mask"].tolist() == [1, 0, 1, 0, 0]
    # elite = 0.5 -> m = 5 takes rows 1 and 8 (E = 3) too
    r = oracle.persist_fix(inst, S, E, 0.5, 1.0)
    assert r["m"] == 5 and r["fixed_mask"].tolist() == [0, 0, 0, 0, 0]


def test_config_products_round_as_stated():
    inst = si.random_sparse(4, 2.0, seed=1)
    for R, eps, theta, m, kmin in [(100, 0.1, 1.0, 10, 10), (10000, 0.05, 0.95, 500, 475),
                                   (10240, 0.2, 1.0, 2048, 2048), (7, 0.1, 1.0, 1, 1)]:
        S = np.ones((R, 4), np.int8)
        r = oracle.persist_fix(inst, S, np.zeros(R, np.int64), eps, theta)
        assert (r["m"], r["k_min"]) == (m, kmin)


def test_unanimous_sample_fixes_everything():
    inst = si.chimera(2, seed=9)
    s = si.random_spins(1, inst.n, seed=2)
    S = np.repeat(s, 12, axis=0)
    r = oracle.persist_fix(inst, S, oracle.energy(inst, S), 0.5, 1.0)
    assert r["n_free"] == 0 and r["nnz_free"] == 0
    assert r["offset"] == oracle.energy(inst, s)[0]
    assert np.array_equal(r["fixed_val"], s[0])


def test_zero_bias_needs_the_gauge():
    inst = si.cubic_lattice(4, "pm1", seed=6)
    spins, E = oracle.sa_sample(inst, si.linear_betas(0.1, 3.0, 300), reads=40, seed=6)
    both = np.concatenate([spins, -spins])
    Eb = np.concatenate([E, E])
    assert np.array_equal(oracle.energy(inst, -spins), E)
    off = oracle.persist_fix(inst, both, Eb, 0.2, 1.0, gauge=0)
    assert off["n_fixed"] == 0 and off["pivot"] == -1
    on = oracle.persist_fix(inst, both, Eb, 0.2, 1.0, gauge=1)
    assert on["pivot"] >= 0 and on["fixed_val"][on["pivot"]] == 1
    # Every fixed variable is perfectly (anti)correlated with the pivot over
    # the elite, and the largest such class was chosen.
    order = np.lexsort((np.arange(both.shape[0]), Eb))
    elite = both[np.sort(order[:on["m"]])]
    p = on["pivot"]
    corr = (elite * elite[:, [p]]).sum(0)
    fixed = on["fixed_mask"].astype(bool)
    assert np.all(np.abs(corr[fixed]) == on["m"])
    assert np.array_equal(on["fixed_val"][fixed], np.sign(corr[fixed]))
    # class sizes: no other variable's class is larger
    canon = elite * elite[:1]
    _, counts = np.unique(canon.T, axis=0, return_counts=True)
    assert fixed.sum() == counts.max()
    _completions_check(inst, on) if on["reduced"].n <= 14 else None
    auto = oracle.persist_fix(inst, both, Eb, 0.2, 1.0, gauge=2)
    assert np.array_equal(auto["fixed_mask"], on["fixed_mask"])


def test_gauge_covariance():
    inst = si.random_sparse(16, 3.0, seed=41)
    spins, E = oracle.sa_sample(inst, si.linear_betas(0.1, 4.0, 200), reads=80, seed=4)
    base = oracle.persist_fix(inst, spins, E, 0.2, 0.8, gauge=0)
    rng = np.random.default_rng(3)
    tau = rng.choice([-1, 1], size=inst.n).astype(np.int64)
    rows = np.repeat(np.arange(inst.n), np.diff(inst.row_ptr))
    g = si.Instance(**{**inst.__dict__, "J": (inst.J * tau[rows] * tau[inst.col]).astype(np.int32),
                       "h": (inst.h * tau).astype(np.int32)})
    gs = (spins * tau[None, :]).astype(np.int8)
    assert np.array_equal(oracle.energy(g, gs), E)
    other = oracle.persist_fix(g, gs, E, 0.2, 0.8, gauge=0)
    assert np.array_equal(other["fixed_mask"], base["fixed_mask"])
    assert np.array_equal(other["fixed_val"], (base["fixed_val"] * tau).astype(np.int8))
    assert other["offset"] == base["offset"]


def test_invalid_arguments_are_rejected():
    inst = si.random_sparse(5, 2.0, seed=1)
    S = np.ones((4, 5), np.int8)
    E = np.zeros(4, np.int64)
    for eps, th in [(0.0, 1.0), (1.5, 1.0), (0.5, 0.0), (0.5, 1.1)]:
        with pytest.raises(oracle.OracleError):
            oracle.persist_fix(inst, S, E, eps, th)
    bad = S.copy()
    bad[0, 0] = 0
    with pytest.raises(oracle.OracleError):
        oracle.persist_fix(inst, bad, E, 0.5, 1.0)


def test_bias_overflow_is_a_range_error():
    # chain 0-1-2 with couplers 2^30: fixing 0 and 2 to +1 folds 2^31 into h'_1
    inst = si.from_edges(3, [0, 1], [1, 2], [2**30, 2**30], [0, 0, 0], [0, 1, 0], 2)
    S = np.array([[1, 1, 1], [1, -1, 1], [1, 1, 1], [1, 1, 1]], np.int8)
    with pytest.raises(oracle.OracleError) as e:
        oracle.persist_fix(inst, S, np.array([0, 0, 1, 1], np.int64), 0.5, 1.0, gauge=0)
    assert e.value.code == -4


def test_ispvar_rounds_compose():
    inst = si.cubic_lattice(4, "pm1", seed=1001)
    betas = si.linear_betas(0.1, 3.0, 300)
    res = oracle.ispvar(inst, betas, 50, 11, 3, 0.1, 1.0, gauge=2)
    info = res["round_info"]
    assert res["rounds_run"] == 3
    assert np.all(np.diff(info[:, 0]) <= 0)  # fixes are never undone
    assert res["fixed_mask"].sum() == inst.n - info[-1, 0]
    # round 0 by hand
    sp, E = oracle.sa_sample(inst, betas, reads=50, seed=11)
    r0 = oracle.persist_fix(inst, sp, E, 0.1, 1.0, gauge=2)
    assert info[0, 0] == r0["n_free"] and info[0, 1] == r0["offset"] and info[0, 2] == E.min()
    sp1, E1 = oracle.sa_sample(r0["reduced"], betas, reads=50, seed=12)
    r1 = oracle.persist_fix(r0["reduced"], sp1, E1, 0.1, 1.0, gauge=2)
    assert info[1, 0] == r1["n_free"] and info[1, 2] == E1.min() + r0["offset"]
    assert info[1, 1] == r0["offset"] + r1["offset"]
