"""GPU parity of the persistence step (elite selection, ballot/popcount counts,
zero-bias gauge, fixing, reduction) through the C ABI, against the oracle on
the same seeded samples.  Samples come from the oracle sampler or from
seeded synthetic generators, never from the HIP path."""
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


def _noisy_sample(R, n, seed, mirror=False, energies_range=None, inst=None):
    """Rows = a base state with per-column flip rates from 0 to 0.5 (some columns unanimous)."""
    rng = np.random.default_rng(seed)
    base = rng.choice([-1, 1], size=n).astype(np.int8)
    rate = np.where(rng.random(n) < 0.4, 0.0, rng.random(n) * 0.5)
    flips = rng.random((R, n)) < rate[None, :]
    S = np.where(flips, -base[None, :], base[None, :]).astype(np.int8)
    if mirror:
        S[rng.random(R) < 0.5] *= -1
    if energies_range is not None:
        E = rng.integers(0, energies_range, size=R).astype(np.int64)
    else:
        E = oracle.energy(inst, S)
    return S, E


def _compare(spv, ctx, inst, S, E, eps, theta, gauge):
    import torch
    P = spv.Problem.from_instance(inst)
    got = spv.spv_persist_fix(ctx, P, torch.as_tensor(S).cuda(), torch.as_tensor(E).cuda(), eps,
                              theta, gauge)
    want = oracle.persist_fix(inst, S, E, eps, theta, gauge)
    info = got.info()
    for k in ("n_free", "nnz_free", "offset", "n_fixed", "pivot", "m", "k_min"):
        assert info[k] == want[k], (k, info[k], want[k])
    assert np.array_equal(got.fixed_mask.cpu().numpy(), want["fixed_mask"])
    assert np.array_equal(got.fixed_val.cpu().numpy(), want["fixed_val"])
    red = got.reduced().to_host()
    w = want["reduced"]
    assert np.array_equal(red["row_ptr"], w.row_ptr)
    assert np.array_equal(red["col"], w.col)
    assert np.array_equal(red["J"], w.J)
    assert np.array_equal(red["h"], w.h)
    assert np.array_equal(red["colour"], w.colour)
    assert np.array_equal(got.orig_index.cpu().numpy(), want["orig_index"])
    return info


CASES = [
    # name, instance, R, eps, theta, gauge, mirror, energy range (None = true energies)
    ("chimera8_config_size", lambda: cf.instance(cf.CHIMERA8_SA), 10000, 0.05, 0.95, 0, False, None),
    ("cubic10_config_size_gauge", lambda: si.cubic_lattice(10, "gauss", seed=3, scale_log2=10), 10240,
     0.2, 1.0, 2, True, None),
    ("ties_everywhere", lambda: si.chimera(3, seed=5), 777, 0.1, 1.0, 0, False, 4),
    ("m_is_one", lambda: si.random_sparse(40, 3.0, seed=6), 9, 0.01, 1.0, 0, False, None),
    ("single_row", lambda: si.random_sparse(40, 3.0, seed=7), 1, 1.0, 1.0, 0, False, None),
    ("m_multiple_of_64", lambda: si.chimera(2, seed=8), 640, 0.2, 0.9, 0, False, None),
    ("gauge_forced_on_with_bias", lambda: si.chimera(3, seed=9), 300, 0.3, 1.0, 1, True, None),
    ("gauge_auto_with_bias_is_off", lambda: si.chimera(3, seed=10), 300, 0.3, 1.0, 2, True, None),
    ("gauge_zero_bias_ties", lambda: si.cubic_lattice(4, "pm1", seed=11), 1000, 0.2, 1.0, 2, True, 3),
    ("n_not_multiple_of_4", lambda: si.random_sparse(77, 3.0, seed=12), 501, 0.3, 0.8, 0, False, None),
]


@pytest.mark.parametrize("name,make,R,eps,theta,gauge,mirror,erange", CASES, ids=[c[0] for c in CASES])
def test_persist_parity(spv, ctx, name, make, R, eps, theta, gauge, mirror, erange):
    inst = make()
    print(f"[persist] {name} n={inst.n} R={R}", flush=True)
    S, E = _noisy_sample(R, inst.n, seed=R + inst.n, mirror=mirror, energies_range=erange, inst=inst)
    info = _compare(spv, ctx, inst, S, E, eps, theta, gauge)
    if name == "cubic10_config_size_gauge":
        assert info["pivot"] >= 0


ELITE_KEYS = [
    ("full_int64_range", lambda rng, R: rng.integers(-2**62, 2**62, size=R)),
    ("all_equal", lambda rng, R: np.full(R, -5)),
    ("common_high_bytes_low_byte_ties", lambda rng, R: -10**12 + rng.integers(0, 200, size=R)),
    ("sign_crossing", lambda rng, R: rng.integers(-1, 1, size=R)),
    ("wide_40_bit", lambda rng, R: rng.integers(-2**40, 2**40, size=R)),
]


@pytest.mark.parametrize("name,make_E", ELITE_KEYS, ids=[c[0] for c in ELITE_KEYS])
def test_persist_elite_selection_over_key_ranges(spv, ctx, name, make_E):
    """Elite selection (the m lowest (E, row) keys) over energies that share all, some or none of
    their high bytes, with ties at the cut; random rows and a low threshold make the fixed set
    depend on exactly which rows are elite."""
    inst = si.random_sparse(200, 3.0, seed=31)
    R = 3000
    rng = np.random.default_rng(32)
    S = si.random_spins(R, inst.n, seed=33)
    E = np.asarray(make_E(rng, R), dtype=np.int64)
    print(f"[persist] elite keys: {name}", flush=True)
    _compare(spv, ctx, inst, S, E, 0.02, 0.2, 0)


def test_persist_on_oracle_sampler_output(spv, ctx):
    inst = si.cubic_lattice(4, "pm1", seed=21)
    S, E = oracle.sa_sample(inst, si.linear_betas(0.1, 3.0, 300), reads=200, seed=5, threads=8)
    for gauge in (0, 1, 2):
        _compare(spv, ctx, inst, S, E, 0.1, 1.0, gauge)


def test_everything_fixed_and_nothing_fixed(spv, ctx):
    inst = si.chimera(2, seed=3)
    s = si.random_spins(1, inst.n, seed=4)
    S = np.repeat(s, 50, axis=0)
    info = _compare(spv, ctx, inst, S, oracle.energy(inst, S), 0.5, 1.0, 0)
    assert info["n_free"] == 0
    S2 = np.concatenate([S, -S])
    info = _compare(spv, ctx, inst, S2, np.zeros(100, np.int64), 1.0, 1.0, 0)
    assert info["n_fixed"] == 0


def test_device_status_for_bad_sample_and_range(spv, ctx):
    import torch
    inst = si.random_sparse(20, 3.0, seed=1)
    P = spv.Problem.from_instance(inst)
    S = si.random_spins(64, 20, seed=2)
    S[3, 5] = 0
    r = spv.spv_persist_fix(ctx, P, torch.as_tensor(S).cuda(), torch.zeros(64, dtype=torch.int64).cuda(),
                            0.5, 1.0, 0)
    with pytest.raises(spv.SpvError) as e:
        r.info()
    assert e.value.code == -1
    # h'_0 = h_0 + J_01 v_1 leaves int32.  A sampling call would refuse this
    # instance at ingest (max |h| + sum |J| >= 2^26); persistence does not ingest,
    # so its own device-side check is exercised.
    big_h = si.from_edges(3, [0, 1], [1, 2], [30000, 30000], [2**31 - 20000, 0, 0], [0, 1, 0], 2)
    P = spv.Problem(3, 4, *[torch.as_tensor(a).cuda() for a in
                            (big_h.row_ptr, big_h.col, big_h.J, big_h.h, big_h.colour)],
                    2, 0)
    S = np.array([[1, 1, 1], [-1, 1, 1], [1, 1, 1], [1, 1, 1]], np.int8)
    E = np.array([0, 0, 1, 1], np.int64)
    r = spv.spv_persist_fix(ctx, P, torch.as_tensor(S).cuda(), torch.as_tensor(E).cuda(), 0.5, 1.0, 0)
    with pytest.raises(spv.SpvError) as e:
        r.info()
    assert e.value.code == -4
    with pytest.raises(oracle.OracleError) as e:
        oracle.persist_fix(big_h, S, E, 0.5, 1.0, 0)
    assert e.value.code == -4


def test_invalid_arguments_rejected_on_host(spv, ctx):
    import torch
    inst = si.random_sparse(10, 2.0, seed=1)
    P = spv.Problem.from_instance(inst)
    S = torch.ones((4, 10), dtype=torch.int8).cuda()
    E = torch.zeros(4, dtype=torch.int64).cuda()
    for eps, th in [(0.0, 1.0), (1.5, 1.0), (0.5, 0.0), (0.5, 1.5)]:
        with pytest.raises(spv.SpvError):
            spv.spv_persist_fix(ctx, P, S, E, eps, th, 0)
