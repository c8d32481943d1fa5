"""Pins of the oracle's parallel tempering, cluster moves and top-10 sample.

* Replica exchange (Sec. III.D.1 PTICM): D <= 0 always swaps; otherwise the
  empirical swap rate over independent random words matches
  exp(-dbeta * D / 2^scale).
* Each PT slot, and each slot with Houdayer cluster moves between two
  chains, samples the exact Boltzmann distribution at its own beta (chi-square
  on a tiny instance): replica exchange and cluster moves preserve the
  product of the slot distributions.
* Houdayer move: the pair energy E_A + E_B is conserved exactly; the flipped
  set is the connected component (scipy csgraph) of the chosen seed inside
  the sites where the replicas disagree; identical replicas are left alone.
* Top-10 sample (Sec. III.D.1): the online lists equal a post-hoc selection
  from the full per-sweep log (10 smallest distinct states by (E, first sweep
  seen)).
"""
import numpy as np
import pytest
from scipy import sparse, stats
from scipy.sparse import csgraph

import oracle
import spvar_inputs as si
from tests import _brute
from tests.test_oracle_pins import _chi2_pvalue


def test_swap_rule_direction_and_rate():
    for D in (0, -5, -10**9):
        assert all(oracle.swap_test(D, 0.3, 0, 1, t, 0, 9) for t in range(50))
    for dbeta, D, scale in [(0.3, 4, 0), (0.05, 3000, 10), (0.02, 200000, 10)]:
        p = np.exp(-dbeta * D / 2 ** scale)
        acc = np.mean([oracle.swap_test(D, dbeta, scale, 3, t, 1, 5) for t in range(20000)])
        sd = np.sqrt(p * (1 - p) / 20000)
        assert abs(acc - p) < 5 * sd + 1e-4, (dbeta, D, acc, p)
    # far beyond the last digit: rejected
    assert not any(oracle.swap_test(2**40, 0.05, 10, 0, t, 0, 1) for t in range(100))


def test_pt_slots_sample_boltzmann():
    inst = si.random_sparse(6, 3.0, j_max=2, h_max=2, seed=11)
    betas = si.geometric_betas(0.2, 1.0, 4)
    res = oracle.pt_sample(inst, betas, runs=12000, chains=1, sweeps=40, seed=5, top=False,
                           threads=8)
    for k in range(4):
        assert _chi2_pvalue(res["final_spins"][:, 0, k], inst, betas[k]) > 1e-4, k


def test_pt_with_cluster_moves_samples_boltzmann():
    inst = si.random_sparse(6, 3.0, j_max=2, h_max=2, seed=13)
    betas = si.geometric_betas(0.3, 1.2, 4)
    res = oracle.pt_sample(inst, betas, runs=10000, chains=2, sweeps=40, seed=6, icm=(0, 4),
                           top=False, threads=8)
    for ch in range(2):
        for k in range(4):
            assert _chi2_pvalue(res["final_spins"][:, ch, k], inst, betas[k]) > 1e-4, (ch, k)


def _component(inst, mask, seed_site):
    rows = np.repeat(np.arange(inst.n), np.diff(inst.row_ptr))
    keep = mask[rows] & mask[inst.col] & (inst.J != 0)
    A = sparse.csr_matrix((np.ones(keep.sum()), (rows[keep], inst.col[keep])),
                          shape=(inst.n, inst.n))
    _, lab = csgraph.connected_components(A, directed=False)
    return mask & (lab == lab[seed_site])


@pytest.mark.parametrize("seed", range(6))
def test_houdayer_move_conserves_pair_energy_and_flips_a_component(seed):
    inst = si.cubic_lattice(4, "gauss", seed=seed, scale_log2=10, h_dist="gauss") if seed % 2 \
        else si.chimera(3, seed=seed)
    A = si.random_spins(1, inst.n, seed=10 + seed)[0]
    B = si.random_spins(1, inst.n, seed=20 + seed)[0]
    rng = np.random.default_rng(seed)
    for w in [0, 2**32 - 1, int(rng.integers(0, 2**32))]:
        A2, B2, EA, EB, cl, flipped = oracle.icm_step(inst, A, B, w)
        E0 = _brute.energies(inst, np.stack([A, B]))
        assert flipped
        assert EA + EB == E0.sum()
        assert [EA, EB] == _brute.energies(inst, np.stack([A2, B2])).tolist()
        diff = A != B
        sites = np.nonzero(diff)[0]
        seed_site = sites[(w * sites.size) >> 32]
        assert np.array_equal(cl, _component(inst, diff, seed_site))
        assert np.array_equal(A2[cl], -A[cl]) and np.array_equal(A2[~cl], A[~cl])
        assert np.array_equal(B2[cl], -B[cl]) and np.array_equal(B2[~cl], B[~cl])
    _, _, _, _, cl, flipped = oracle.icm_step(inst, A, A, 12345)
    assert not flipped and not cl.any()


def _posthoc_top10(log_E, log_spins, ch, k):
    seen = {}
    for t in range(log_E.shape[0]):
        key = log_spins[t, ch, k].tobytes()
        if key not in seen:
            seen[key] = (int(log_E[t, ch, k]), t, log_spins[t, ch, k].copy())
    best = sorted(seen.values(), key=lambda v: (v[0], v[1]))[:10]
    return [b[0] for b in best], [b[2] for b in best]


@pytest.mark.parametrize("chains,icm,K", [(1, None, 6), (2, (0, 6), 6), (1, None, 5), (2, (1, 4), 7)])
def test_top10_equals_posthoc_selection(chains, icm, K):
    inst = si.cubic_lattice(4, "gauss", seed=3, scale_log2=10)
    betas = si.geometric_betas(0.2, 5.0, K)
    first = K - K // 2  # the K/2 coldest slots
    res = oracle.pt_sample(inst, betas, runs=1, chains=chains, sweeps=300, seed=8, icm=icm,
                           log=True)
    log_E, log_spins = res["log_E"], res["log_spins"]
    flat = log_spins.reshape(-1, inst.n)
    assert np.array_equal(log_E.reshape(-1), _brute.energies(inst, flat))
    for ch in range(chains):
        for k in range(first, K):
            want_E, want_S = _posthoc_top10(log_E, log_spins, ch, k)
            got_E = res["top_E"][0, ch, k - first]
            c = int(res["top_count"][0, ch, k - first])
            assert c == len(want_E)
            assert got_E[:c].tolist() == want_E
            assert np.array_equal(res["top_spins"][0, ch, k - first, :c], np.array(want_S))


def test_pt_final_energies_and_run_subsets():
    inst = si.cubic_lattice(4, "gauss", seed=4, scale_log2=10)
    betas = si.geometric_betas(0.2, 5.0, 8)
    full = oracle.pt_sample(inst, betas, runs=4, chains=1, sweeps=50, seed=2)
    sub = oracle.pt_sample(inst, betas, runs=4, chains=1, sweeps=50, seed=2, run_begin=2, run_end=4)
    for key in ("final_spins", "final_E", "top_spins", "top_E", "top_count"):
        assert np.array_equal(full[key][2:4], sub[key])
    fs = full["final_spins"].reshape(-1, inst.n)
    assert np.array_equal(full["final_E"].reshape(-1), _brute.energies(inst, fs))
    S, E = oracle.top_sample(full)
    assert S.shape[0] == int(full["top_count"].sum()) and np.array_equal(E, _brute.energies(inst, S))


def test_slot_threads_leave_the_run_unchanged():
    """Spreading a run's independent slots, cluster-move pairs and top-10 lists over host
    threads gives the sequential run's bits (final states, energies, top-10 lists)."""
    inst = si.cubic_lattice(6, "gauss", seed=12, scale_log2=10)
    betas = si.geometric_betas(0.2, 5.0, 10)
    seq = oracle.pt_sample(inst, betas, 2, 2, 40, seed=9, icm=(0, 10))
    oracle.set_slot_threads(4)
    try:
        par = oracle.pt_sample(inst, betas, 2, 2, 40, seed=9, icm=(0, 10))
    finally:
        oracle.set_slot_threads(1)
    for key in ("final_spins", "final_E", "top_E", "top_count", "top_spins"):
        assert np.array_equal(seq[key], par[key]), key
