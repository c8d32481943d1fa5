"""Pins of the oracle's tempering checkpoint (continuing a run, Sec. III.D.1).

A tempering run is a Markov chain driven by counter-based random words (keyed by sweep, slot
and run), so stopping after N sweeps and continuing from the final states and top-10 lists
with the sweep counter advanced to N must give the uninterrupted run bit for bit:

* one run of N + M sweeps equals N sweeps followed by M resumed sweeps, for plain tempering,
  tempering with cluster moves, odd ladders, several runs and pieces of a run range, and for
  a split into three pieces;
* N = 0 (the checkpoint of a fresh run is its initial state) gives the fresh run;
* a list resumed from arbitrary distinct entries (some that survive, some that are evicted)
  equals the post-hoc selection of the 10 lowest distinct states by (E, first seen) over the
  checkpoint entries, taken first in their listed order, and every state offered after;
* a count outside 0..10 starts that list empty and reports -1; a byte > 0 is spin +1 and any
  other byte -1; with no sweeps the checkpoint comes back unchanged.
"""
import numpy as np
import pytest

import oracle
import spvar_inputs as si
from tests import _brute

KEYS = ("final_spins", "final_E", "top_spins", "top_E", "top_count")


def _same(a, b):
    for key in KEYS:
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("chains,icm,K,runs", [(1, None, 6, 2), (2, (0, 6), 6, 1), (1, None, 5, 3),
                                               (2, (1, 4), 7, 2)])
@pytest.mark.parametrize("split", [0, 1, 37])
def test_split_run_equals_one_run(chains, icm, K, runs, split):
    inst = si.cubic_lattice(4, "gauss", seed=5, scale_log2=10)
    betas = si.geometric_betas(0.2, 5.0, K)
    total = 80
    whole = oracle.pt_sample(inst, betas, runs, chains, total, seed=13, icm=icm)
    first = oracle.pt_sample(inst, betas, runs, chains, split, seed=13, icm=icm)
    rest = oracle.pt_sample(inst, betas, runs, chains, total - split, seed=13, icm=icm, sweep_offset=split,
                            resume=first)
    _same(whole, rest)


def test_three_pieces_and_run_ranges():
    inst = si.cubic_lattice(4, "gauss", seed=6, scale_log2=10, h_dist="gauss")
    betas = si.geometric_betas(0.3, 4.0, 8)
    whole = oracle.pt_sample(inst, betas, 4, 2, 90, seed=3, icm=(2, 8))
    a = oracle.pt_sample(inst, betas, 4, 2, 25, seed=3, icm=(2, 8))
    b = oracle.pt_sample(inst, betas, 4, 2, 40, seed=3, icm=(2, 8), sweep_offset=25, resume=a)
    c = oracle.pt_sample(inst, betas, 4, 2, 25, seed=3, icm=(2, 8), sweep_offset=65, resume=b)
    _same(whole, c)
    # the checkpoint of runs 1..2 resumes those runs alone
    part = {k: a[k][1:3] for k in KEYS}
    c12 = oracle.pt_sample(inst, betas, 4, 2, 65, seed=3, icm=(2, 8), sweep_offset=25, run_begin=1,
                           run_end=3, resume=part)
    for key in KEYS:
        assert np.array_equal(whole[key][1:3], c12[key]), key


def _posthoc(entries):
    """10 lowest distinct states by (E, first seen) over (E, time, state) in time order."""
    seen = {}
    for E, t, s in entries:
        key = s.tobytes()
        if key not in seen:
            seen[key] = (E, t, s)
    best = sorted(seen.values(), key=lambda v: (v[0], v[1]))[:10]
    return [b[0] for b in best], [b[2] for b in best]


def test_resumed_lists_equal_posthoc_selection_over_checkpoint_and_new_states():
    inst = si.cubic_lattice(4, "gauss", seed=3, scale_log2=10)
    n, K, chains = inst.n, 6, 2
    half = K // 2
    betas = si.geometric_betas(0.2, 5.0, K)
    # low-energy states from a long cold run survive the resumed run; random states do not
    cold = oracle.pt_sample(inst, betas, 1, chains, 400, seed=99)
    low_S = cold["top_spins"].reshape(-1, n)
    assert int(cold["top_count"].sum()) == low_S.shape[0] == 60
    rng = np.random.default_rng(5)
    rand_S = np.where(rng.random((30, n)) < 0.5, 1, -1).astype(np.int8)
    ck = oracle.pt_sample(inst, betas, 1, chains, 0, seed=21)  # the run's initial states
    ck["top_spins"] = np.zeros((1, chains, half, 10, n), np.int8)
    ck["top_E"] = np.full((1, chains, half, 10), np.iinfo(np.int64).max, np.int64)
    ck["top_count"] = np.zeros((1, chains, half), np.int32)
    given = {}
    for li, c in enumerate([0, 3, 10, 7, 10, 1]):
        ch, j = divmod(li, half)
        pool = np.unique(np.concatenate([low_S[li * 10:li * 10 + 6], rand_S[li * 5:li * 5 + 5]]), axis=0)
        assert pool.shape[0] >= c
        pool = pool[rng.permutation(pool.shape[0])[:c]]
        rng.shuffle(pool)  # listed order need not be energy order
        E = _brute.energies(inst, pool) if c else np.zeros(0, np.int64)
        ck["top_spins"][0, ch, j, :c] = pool
        ck["top_E"][0, ch, j, :c] = E
        ck["top_count"][0, ch, j] = c
        given[(ch, j)] = [(int(E[e]), e - 10, pool[e].copy()) for e in range(c)]
    res = oracle.pt_sample(inst, betas, 1, chains, 150, seed=21, sweep_offset=0, resume=ck, log=True)
    first = K - half
    for ch in range(chains):
        for j in range(half):
            offered = [(int(res["log_E"][t, ch, first + j]), t, res["log_spins"][t, ch, first + j])
                       for t in range(150)]
            want_E, want_S = _posthoc(given[(ch, j)] + offered)
            c = int(res["top_count"][0, ch, j])
            assert c == len(want_E)
            assert res["top_E"][0, ch, j, :c].tolist() == want_E
            assert np.array_equal(res["top_spins"][0, ch, j, :c], np.array(want_S))
    # the lists' survivors include checkpoint entries (the test is not vacuous)
    kept = sum(any(np.array_equal(s, g[2]) for g in given[key] for s in res["top_spins"][0, key[0], key[1]])
               for key in given)
    assert kept >= 3


def test_bad_counts_start_empty_and_report_minus_one():
    inst = si.cubic_lattice(4, "gauss", seed=7, scale_log2=10)
    betas = si.geometric_betas(0.2, 5.0, 6)
    a = oracle.pt_sample(inst, betas, 2, 1, 30, seed=4)
    bad = {k: a[k].copy() for k in KEYS}
    bad["top_count"][0, 0, 1] = -1
    bad["top_count"][1, 0, 2] = 11
    empty = {k: a[k].copy() for k in KEYS}
    empty["top_count"][0, 0, 1] = 0
    empty["top_count"][1, 0, 2] = 0
    rb = oracle.pt_sample(inst, betas, 2, 1, 30, seed=4, sweep_offset=30, resume=bad)
    re = oracle.pt_sample(inst, betas, 2, 1, 30, seed=4, sweep_offset=30, resume=empty)
    assert rb["top_count"][0, 0, 1] == -1 and rb["top_count"][1, 0, 2] == -1
    rb["top_count"][0, 0, 1] = re["top_count"][0, 0, 1]
    rb["top_count"][1, 0, 2] = re["top_count"][1, 0, 2]
    _same(rb, re)


def test_spin_bytes_sign_and_no_sweeps_identity():
    inst = si.cubic_lattice(4, "gauss", seed=8, scale_log2=10, h_dist="gauss")
    betas = si.geometric_betas(0.2, 5.0, 6)
    a = oracle.pt_sample(inst, betas, 1, 2, 20, seed=6, icm=(0, 6))
    odd = {k: a[k].copy() for k in KEYS}
    rng = np.random.default_rng(1)
    mag = rng.integers(1, 128, size=odd["final_spins"].shape).astype(np.int8)
    odd["final_spins"] = np.where(a["final_spins"] > 0, mag, np.where(mag % 2 == 0, 0, -mag)).astype(np.int8)
    t1 = odd["top_spins"]
    odd["top_spins"] = np.where(t1 > 0, 77, np.where(t1 < 0, -5, 0)).astype(np.int8)
    b1 = oracle.pt_sample(inst, betas, 1, 2, 15, seed=6, icm=(0, 6), sweep_offset=20, resume=a)
    b2 = oracle.pt_sample(inst, betas, 1, 2, 15, seed=6, icm=(0, 6), sweep_offset=20, resume=odd)
    _same(b1, b2)
    z = oracle.pt_sample(inst, betas, 1, 2, 0, seed=6, icm=(0, 6), sweep_offset=20, resume=a)
    _same(a, z)
    fs = z["final_spins"].reshape(-1, inst.n)
    assert np.array_equal(z["final_E"].reshape(-1), _brute.energies(inst, fs))


def test_partial_list_checkpoint_is_rejected():
    inst = si.cubic_lattice(4, "gauss", seed=8, scale_log2=10)
    betas = si.geometric_betas(0.2, 5.0, 4)
    a = oracle.pt_sample(inst, betas, 1, 1, 5, seed=6)
    with pytest.raises(oracle.OracleError):
        oracle.pt_sample(inst, betas, 1, 1, 5, seed=6, resume={"final_spins": a["final_spins"],
                                                              "top_count": a["top_count"]})
