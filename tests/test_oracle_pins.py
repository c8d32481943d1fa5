"""Pins of the CPU oracle's sampler against facts fixed outside the oracle.

* Philox4x32-10 known-answer vectors published with the Random123 library
  (the generator of Salmon et al., SC'11).
* The energy convention of Sec. I pinned by the weak-strong degeneracy point
  stated in Sec. III.B (doubly degenerate ground state at h_w = -0.5).
* Closed forms: ferromagnet and gauge-planted ferromagnet ground energies.
* Acceptance thresholds against an exact decimal evaluation of 2^32 exp(.).
* Metropolis at fixed beta reproduces the exact Boltzmann distribution of a
  tiny instance (chi-square), for one-digit and two-digit threshold tables.
* Simulated annealing reaches the brute-force ground state of small instances.
* Counter-based randomness: in-class visiting order, read subsets and resume
  do not change a single bit.
"""
import decimal
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import spvar_inputs as si
from tests import _brute


# ---------------------------------------------------------------- Philox --
KAT = [
    ([0, 0, 0, 0], [0, 0], [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
    ([0xffffffff] * 4, [0xffffffff] * 2, [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
    ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0],
     [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    assert [int(v) for v in oracle.philox(ctr, key)] == want


def test_philox_bits_balanced():
    n = 200_000
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 3] = 2 << 24
    out = oracle.philox_batch(ctr, [123, 456])
    bits = np.unpackbits(out.view(np.uint8)).reshape(-1, 32 * 4 // 1)
    frac = bits.mean(axis=0)
    # 200k samples per bit: sd = 0.5/sqrt(2e5) ~ 1.1e-3
    assert np.all(np.abs(frac - 0.5) < 0.006)


# ---------------------------------------------------------------- energy --
def test_energy_matches_dense_evaluation():
    inst = si.random_sparse(20, 4.0, seed=3)
    S = si.random_spins(500, 20, seed=4)
    assert np.array_equal(oracle.energy(inst, S), _brute.energies(inst, S))


def test_weak_strong_degeneracy_pins_single_counting():
    # Sec. III.B: at h_w = -0.5 the ground state is doubly degenerate (weak
    # cluster aligned with or opposite to the strong one); at h_w = -0.42 it
    # is the aligned state.  Integer units of 1/100.
    S = _brute.all_states(16)
    inst = si.weak_strong_toy(-50)
    E = oracle.energy(inst, S)
    assert np.array_equal(E, _brute.energies(inst, S))
    gs = S[E == E.min()]
    assert gs.shape[0] == 2
    strong, weak = gs[:, :8], gs[:, 8:]
    assert np.all(strong == -1)
    assert sorted(weak[:, 0].tolist()) == [-1, 1] and np.all(weak == weak[:, :1])
    inst42 = si.weak_strong_toy(-42)
    E42 = oracle.energy(inst42, S)
    gs42 = S[E42 == E42.min()]
    assert gs42.shape[0] == 1 and np.all(gs42 == -1)
    # Counting each coupler twice (s^T J s with J symmetric) would break the
    # stated degeneracy at h_w = -0.5.
    doubled = si.weak_strong_toy(-50, j=-200)
    Ed = oracle.energy(doubled, S)
    assert (Ed == Ed.min()).sum() == 1


def test_ferromagnet_and_planted_ground_energy():
    inst = si.cubic_lattice(4, "pm1", seed=1)
    ferro = si.Instance(**{**inst.__dict__, "J": -np.abs(inst.J)})
    up = np.ones((1, inst.n), np.int8)
    assert oracle.energy(ferro, up)[0] == -(inst.nnz // 2)
    rng = np.random.default_rng(5)
    tau = rng.choice([-1, 1], size=inst.n).astype(np.int8)
    rows = np.repeat(np.arange(inst.n), np.diff(inst.row_ptr))
    mag = rng.integers(1, 7, size=inst.nnz)
    mag = np.minimum(mag, mag[_transpose_index(inst)])  # symmetric magnitudes
    planted = si.Instance(**{**inst.__dict__, "J": (-mag * tau[rows] * tau[inst.col]).astype(np.int32)})
    assert oracle.energy(planted, tau[None, :])[0] == -int(mag.sum()) // 2


def _transpose_index(inst):
    rows = np.repeat(np.arange(inst.n), np.diff(inst.row_ptr))
    pos = {}
    for k, (a, b) in enumerate(zip(rows, inst.col)):
        pos[(int(a), int(b))] = k
    return np.array([pos[(int(b), int(a))] for a, b in zip(rows, inst.col)])


# ------------------------------------------------------------ thresholds --
@pytest.mark.parametrize("beta,unit,scale,digit", [
    (0.1, 2, 0, 0), (3.0, 2, 0, 0), (5.0, 2, 0, 0), (0.2, 2, 10, 0), (0.2, 2, 10, 1),
    (5.0, 2, 10, 1), (0.0172, 1, 10, 2), (0.39, 1, 10, 1), (0.0, 2, 0, 0)])
def test_thresholds_within_one_of_exact(beta, unit, scale, digit):
    decimal.getcontext().prec = 60
    B = decimal.Decimal(beta)  # the exact binary value of the double
    for d in [0, 1, 2, 3, 7, 50, 255, 511]:
        arg = B * unit * d * (512 ** digit) / decimal.Decimal(2) ** scale
        exact = (-arg).exp() * decimal.Decimal(2) ** 32
        want = min(int(exact), 2 ** 32 - 1)
        got = oracle.threshold(beta, unit, scale, digit, d)
        assert abs(got - want) <= 1, (d, got, want)


def test_swap_digit_count_is_first_zero_digit():
    for db in [0.0172, 0.05, 0.396, 1.0]:
        nd = oracle.swap_digits(db, 10)
        assert oracle.threshold(db, 1, 10, nd, 1) == 0
        assert oracle.threshold(db, 1, 10, nd - 1, 1) > 0 or nd == 1


# ------------------------------------------------------------- Boltzmann --
def _chi2_pvalue(states, inst, beta, min_expected=5.0):
    S = _brute.all_states(inst.n)
    E = _brute.energies(inst, S).astype(np.float64) / 2 ** inst.scale_log2
    w = np.exp(-beta * (E - E.min()))
    p = w / w.sum()
    codes = ((np.asarray(states, np.int64) > 0).astype(np.int64) << np.arange(inst.n)).sum(1)
    obs = np.bincount(codes, minlength=2 ** inst.n).astype(np.float64)
    exp = p * obs.sum()
    keep = exp >= min_expected
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] == 0:
        o, e = o[:-1], e[:-1]
    chi2 = ((o - e) ** 2 / e).sum()
    return stats.chi2.sf(chi2, o.size - 1)


def _small_instance(scale=0):
    if scale == 0:
        return si.random_sparse(6, 3.0, j_max=2, h_max=2, seed=11)
    # couplers of several hundred units: Metropolis uphill moves span two
    # base-512 digits, so the two-digit test is exercised
    return si.random_sparse(6, 3.0, seed=12, scale_log2=scale,
                            dist=("uniform_nonzero", 700))


@pytest.mark.parametrize("scale,beta", [(0, 0.6), (10, 0.9)])
def test_metropolis_samples_boltzmann(scale, beta):
    inst = _small_instance(scale)
    if scale:
        assert oracle.x_max(inst) >= 512
    betas = np.full(60, beta)
    spins, _ = oracle.sa_sample(inst, betas, reads=30000, seed=77, threads=8)
    assert _chi2_pvalue(spins, inst, beta) > 1e-4


def test_metropolis_chi2_detects_wrong_temperature():
    # Power check: the same samples are rejected against half the temperature.
    inst = _small_instance(0)
    spins, _ = oracle.sa_sample(inst, np.full(60, 0.6), reads=30000, seed=78, threads=8)
    assert _chi2_pvalue(spins, inst, 1.2) < 1e-6


# ------------------------------------------------------------ annealing --
@pytest.mark.parametrize("seed", [21, 22, 23])
def test_annealing_reaches_brute_force_ground_state(seed):
    inst = si.random_sparse(14, 3.0, seed=seed)
    _, Eb = _brute.ground(inst)
    _, E = oracle.sa_sample(inst, si.linear_betas(0.1, 5.0, 1500), reads=32, seed=seed, threads=8)
    assert E.min() == Eb.min()


def test_sample_energies_are_recomputed_energies():
    inst = si.chimera(2, seed=5)
    spins, E = oracle.sa_sample(inst, si.linear_betas(0.1, 3.0, 50), reads=37, seed=9)
    assert np.array_equal(E, _brute.energies(inst, spins))


# ---------------------------------------------- counter-based invariances --
def test_in_class_order_is_immaterial():
    inst = si.chimera(3, seed=8)
    betas = si.linear_betas(0.1, 4.0, 40)
    a, Ea = oracle.sa_sample(inst, betas, reads=16, seed=31)
    rng = np.random.default_rng(0)
    order = np.concatenate([rng.permutation(np.nonzero(inst.colour == c)[0])
                            for c in range(inst.n_colours)])
    b, Eb = oracle.sa_sample(inst, betas, reads=16, seed=31, order=order)
    assert np.array_equal(a, b) and np.array_equal(Ea, Eb)


def test_read_subset_and_resume_are_exact():
    inst = si.cubic_lattice(4, "pm1", seed=2)
    betas = si.linear_betas(0.1, 3.0, 30)
    full, Ef = oracle.sa_sample(inst, betas, reads=20, seed=5)
    sub, Es = oracle.sa_sample(inst, betas, seed=5, r_begin=7, r_end=13)
    assert np.array_equal(sub, full[7:13]) and np.array_equal(Es, Ef[7:13])
    half, _ = oracle.sa_sample(inst, betas[:12], reads=20, seed=5)
    rest, Er = oracle.sa_sample(inst, betas[12:], reads=20, seed=5, sweep_offset=12, init=half)
    assert np.array_equal(rest, full) and np.array_equal(Er, Ef)


def test_seeds_change_the_stream():
    inst = si.cubic_lattice(4, "pm1", seed=2)
    betas = si.linear_betas(0.1, 3.0, 10)
    a, _ = oracle.sa_sample(inst, betas, reads=4, seed=1)
    b, _ = oracle.sa_sample(inst, betas, reads=4, seed=2)
    assert not np.array_equal(a, b)
