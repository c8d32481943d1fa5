"""Pins of the oracle's simulated quantum annealing (Sec. III, "SQA": discrete-time
path-integral Monte Carlo over P Trotter slices, written from the Suzuki-Trotter mapping
of Martonak, Santoro and Tosatti 2002).

* The inter-slice coupling inverts to the closed form it comes from:
  exp(-2 beta Jperp) = tanh(beta Gamma / P), within the rounding of Jp to integer units.
* At fixed beta and Gamma the sweeps sample the Trotter weight
  exp(-(beta/P) (sum_k E(s^k) - Jp sum_k sum_i s^k_i s^{k+1}_i) / 2^scale) over whole paths
  (chi-square over every path state of tiny instances, weights by dense enumeration); the
  same samples fail against the uncoupled weight (power check).
* The returned sample is the lowest-energy slice (energies recomputed densely), the reads
  are independent counter streams, and annealing reaches brute-force ground states.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
import spvar_inputs as si
from tests import _brute


@pytest.mark.parametrize("beta,gamma,P,scale", [(1.0, 1.0, 8, 10), (3.0, 0.1, 8, 10), (0.5, 2.0, 16, 0),
                                                  (2.0, 0.02, 32, 4), (1.0, 1.5, 4, 0)])
def test_sqa_coupling_inverts_to_tanh(beta, gamma, P, scale):
    jp = oracle.sqa_coupling(beta, gamma, P, scale)
    unit = P * 2.0 ** scale
    # |Jp - P Jperp 2^scale| <= 1/2, and exp(-2 beta Jperp) = tanh(beta Gamma / P)
    lo, hi = np.exp(-2 * beta * (jp + 0.5) / unit), np.exp(-2 * beta * (jp - 0.5) / unit)
    assert lo <= np.tanh(beta * gamma / P) <= hi


def test_sqa_coupling_limits_and_rejections():
    assert oracle.sqa_coupling(1.0, 60.0, 8, 10) == 0          # strong field: slices decouple
    a = [oracle.sqa_coupling(1.0, g, 8, 10) for g in (0.05, 0.2, 1.0, 3.0)]
    assert a == sorted(a, reverse=True) and a[0] > a[-1]      # weaker field, stiffer ring
    for bad in ((0.0, 1.0), (1.0, 0.0), (-1.0, 1.0), (float("inf"), 1.0)):
        with pytest.raises(oracle.OracleError):
            oracle.sqa_coupling(bad[0], bad[1], 8, 10)
    with pytest.raises(oracle.OracleError):
        oracle.sqa_coupling(5.0, 1e-12, 8, 20)                # Jp beyond 2^24


def _path_pvalue(slices, inst, beta, jp, min_expected=5.0):
    """Chi-square p-value of sampled paths [R][P][n] against the Trotter weight."""
    R, P, n = slices.shape
    S = _brute.all_states(P * n).reshape(-1, P, n)
    Ek = _brute.energies(inst, S.reshape(-1, n)).reshape(-1, P).sum(1).astype(np.float64)
    ring = (S.astype(np.int64) * np.roll(S, -1, axis=1)).sum((1, 2)).astype(np.float64)
    a = -(beta / P) * (Ek - jp * ring) / 2 ** inst.scale_log2
    p = np.exp(a - a.max())
    p /= p.sum()
    bits = (slices.reshape(R, P * n) > 0).astype(np.int64)
    codes = (bits << np.arange(P * n)).sum(1)
    obs = np.bincount(codes, minlength=2 ** (P * n)).astype(np.float64)
    exp = p * R
    keep = exp >= min_expected
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] == 0:
        o, e = o[:-1], e[:-1]
    return stats.chi2.sf(((o - e) ** 2 / e).sum(), o.size - 1)


PATH_CASES = [
    # n = 2 (one coupler), P = 4: 256 path states; Jp = 2
    ("pair_P4", lambda: si.from_edges(2, [0], [1], [1], [1, -2], [0, 1], 2), 1.0, 1.5, 4),
    # n = 1 (a biased spin), P = 8: the ring alone, 256 path states; Jp = 6
    ("single_P8", lambda: si.from_edges(1, [], [], [], [1], [0], 1), 1.0, 2.0, 8),
]


@pytest.mark.parametrize("name,make,beta,gamma,P", PATH_CASES, ids=[c[0] for c in PATH_CASES])
def test_sqa_paths_sample_the_trotter_weight(name, make, beta, gamma, P):
    inst = make()
    jp = oracle.sqa_coupling(beta, gamma, P, inst.scale_log2)
    assert jp > 0
    sw = 30
    _, _, _, slices, _ = oracle.sqa_sample(inst, np.full(sw, beta), np.full(sw, gamma), P, reads=40000,
                                           seed=91, slices=True, threads=8)
    assert _path_pvalue(slices, inst, beta, jp) > 1e-4
    # power checks: the same paths are rejected without the ring coupling and with its sign flipped
    assert _path_pvalue(slices, inst, beta, 0) < 1e-6
    assert _path_pvalue(slices, inst, beta, -jp) < 1e-6


def test_sqa_sample_is_the_lowest_energy_slice():
    inst = si.chimera(2, seed=4)
    P = 8
    sp, E, best, slices, ecl = oracle.sqa_sample(inst, si.linear_betas(0.2, 2.0, 40), np.linspace(3.0, 0.3, 40),
                                                 P, reads=23, seed=3, slices=True)
    dense = _brute.energies(inst, slices.reshape(-1, inst.n)).reshape(23, P)
    assert np.array_equal(ecl, dense)
    assert np.array_equal(best, np.argmin(dense, axis=1))      # first minimum
    assert np.array_equal(E, dense[np.arange(23), best])
    assert np.array_equal(sp, slices[np.arange(23), best])


def test_sqa_reads_are_independent_streams():
    inst = si.cubic_lattice(4, "pm1", seed=6)
    b, g = si.linear_betas(0.1, 3.0, 30), np.linspace(2.0, 0.1, 30)
    full = oracle.sqa_sample(inst, b, g, 8, reads=12, seed=8)
    part = oracle.sqa_sample(inst, b, g, 8, seed=8, r_begin=5, r_end=9)
    for x, y in zip(full, part):
        assert np.array_equal(x[5:9], y)
    other = oracle.sqa_sample(inst, b, g, 8, reads=12, seed=9)
    assert not np.array_equal(full[0], other[0])


@pytest.mark.parametrize("seed", [31, 32])
def test_sqa_annealing_reaches_brute_force_ground_state(seed):
    inst = si.random_sparse(13, 3.0, seed=seed)
    _, Eb = _brute.ground(inst)
    sw = 600
    _, E, _ = oracle.sqa_sample(inst, si.linear_betas(0.2, 5.0, sw), np.geomspace(3.0, 0.01, sw), 8,
                                reads=16, seed=seed, threads=8)
    assert E.min() == Eb.min()


def test_sqa_rejects_odd_trotter_number():
    inst = si.chimera(2, seed=1)
    with pytest.raises(oracle.OracleError):
        oracle.sqa_sample(inst, np.ones(3), np.ones(3), 5, reads=2)
