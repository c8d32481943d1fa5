"""GPU parity of simulated quantum annealing (path-integral Monte Carlo over P Trotter slices)
through the C ABI, bit for bit against the oracle: each read's lowest-energy slice and its
energy, over one-, two- and three-digit acceptance tables, several Trotter numbers, ragged
read counts and the degenerate cases; argument and range errors from the host."""
import sys

import numpy as np
import pytest

import oracle
import spvar_inputs as si

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spv():
    import paper_1706_07826_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(spv):
    return spv.Context(0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sched(sweeps, b0=0.2, b1=3.0, g0=3.0, g1=0.05):
    return si.linear_betas(b0, b1, sweeps), np.geomspace(g0, g1, sweeps) if sweeps else np.zeros(0)


def _no_edges(n):
    return si.from_edges(n, [], [], [], np.arange(1, n + 1) * (-1) ** np.arange(n), np.zeros(n), 1)


CASES = [
    # name, instance, trotter, reads, sweeps
    ("chimera2_P8", lambda: si.chimera(2, seed=1), 8, 13, 40),
    ("chimera3_P16", lambda: si.chimera(3, seed=2), 16, 9, 30),
    ("cubic4_pm1_P32", lambda: si.cubic_lattice(4, "pm1", seed=3), 32, 5, 25),
    ("cubic4_gauss_two_digits_P8", lambda: si.cubic_lattice(4, "gauss", seed=4, scale_log2=10), 8, 11, 30),
    ("sparse40_greedy_P24", lambda: si.random_sparse(40, 3.0, seed=5), 24, 7, 30),
    ("no_edges_P8", lambda: _no_edges(9), 8, 6, 20),
    ("single_spin_P8", lambda: _no_edges(1), 8, 5, 15),
    ("zero_sweeps_P8", lambda: si.chimera(2, seed=6), 8, 4, 0),
]


@pytest.mark.parametrize("name,make,P,reads,sweeps", CASES, ids=[c[0] for c in CASES])
def test_sqa_parity(spv, ctx, name, make, P, reads, sweeps):
    inst = make()
    b, g = _sched(sweeps)
    _say(f"[sqa] {name} n={inst.n} P={P} reads={reads} sweeps={sweeps}")
    Pr = spv.Problem.from_instance(inst)
    sp, E = spv.spv_sqa_sample(ctx, Pr, b, g, P, reads, 41)
    osp, oE, _ = oracle.sqa_sample(inst, b, g, P, reads=reads, seed=41, threads=8)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


def test_sqa_three_digit_tables(spv, ctx):
    """A weak final field makes the slice coupling large: x_bound + 2 Jp spans three digits."""
    inst = si.cubic_lattice(4, "gauss", seed=7, scale_log2=10)
    b, g = _sched(30, 0.1, 0.3, 0.1, 0.05)
    jmax = max(oracle.sqa_coupling(x, y, 8, 10) for x, y in zip(b, g))
    assert oracle.x_max(inst) + 2 * jmax >= 512 ** 2
    _say("[sqa] three digits")
    sp, E = spv.spv_sqa_sample(ctx, spv.Problem.from_instance(inst), b, g, 8, 6, 42)
    osp, oE, _ = oracle.sqa_sample(inst, b, g, 8, reads=6, seed=42, threads=6)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


def _beta_for_top_coupling(gamma, trotter, scale_log2):
    """The beta (bisected on the oracle's coupling) whose slice coupling rounds to 2^24, the
    largest the library accepts."""
    lo, hi = 1e-4, 0.01  # coupling out of range at lo, inside at hi (it falls with beta)

    def jp(b):
        try:
            return oracle.sqa_coupling(b, gamma, trotter, scale_log2)
        except oracle.OracleError:
            return None
    assert jp(lo) is None and jp(hi) is not None
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid in (lo, hi):
            break
        if jp(mid) is None:
            lo = mid
        else:
            hi = mid
    return hi, jp(hi)


def test_sqa_slice_coupling_above_2_23(spv, ctx):
    """Slice couplings in [2^23, 2^24] (tiny beta at strong Gamma): the slice term needs the full
    32-bit product; a signed 24-bit multiply would wrap these couplings negative. The first sweep
    sits exactly at the accepted maximum 2^24."""
    inst = si.cubic_lattice(4, "pm1", seed=13, scale_log2=10)
    b_top, j_top = _beta_for_top_coupling(3.0, 8, 10)
    assert j_top == 1 << 24, j_top
    b = np.r_[b_top, np.linspace(0.0021, 0.0031, 11), si.linear_betas(0.05, 3.0, 20)]
    g = np.r_[np.full(12, 3.0), np.geomspace(3.0, 0.05, 20)]
    jps = [oracle.sqa_coupling(x, y, 8, 10) for x, y in zip(b, g)]
    assert sum((1 << 23) <= j < (1 << 24) for j in jps) >= 10 and max(jps) == 1 << 24
    Pr = spv.Problem.from_instance(inst)
    _say(f"[sqa] Jp up to 2^24: n={inst.n} P=8 reads=12 sweeps={b.size}")
    sp, E = spv.spv_sqa_sample(ctx, Pr, b, g, 8, 12, 45)
    osp, oE, _ = oracle.sqa_sample(inst, b, g, 8, reads=12, seed=45, threads=6)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


def test_sqa_chimera8_config_size_sampled_reads(spv, ctx):
    """Chimera 8x8 (N = 512), 16 slices, 400 reads x 300 sweeps on the device; 24 reads
    recomputed by the oracle, every energy equal to its state's."""
    inst = si.chimera(8, seed=8)
    b, g = _sched(300, 0.1, 5.0, 3.0, 0.01)
    _say("[sqa] chimera8 P=16 400 reads x 300 sweeps")
    sp, E = spv.spv_sqa_sample(ctx, spv.Problem.from_instance(inst), b, g, 16, 400, 43)
    sp, E = sp.cpu().numpy(), E.cpu().numpy()
    rows = np.r_[0:8, 190:198, 392:400]
    osp, oE, _ = oracle.sqa_sample(inst, b, g, 16, seed=43, r_begin=0, r_end=8, threads=8)
    assert np.array_equal(sp[0:8], osp) and np.array_equal(E[0:8], oE)
    for lo in (190, 392):
        osp, oE, _ = oracle.sqa_sample(inst, b, g, 16, seed=43, r_begin=lo, r_end=lo + 8, threads=8)
        assert np.array_equal(sp[lo:lo + 8], osp) and np.array_equal(E[lo:lo + 8], oE)
    assert np.array_equal(E, oracle.energy(inst, sp))
    assert rows.size == 24


def test_sqa_workload_size_sampled_reads(spv, ctx):
    """The chimera8_sqa workload as the benchmark launches it (Chimera 8x8 instance of the SA
    workload, 16 slices, 1000 reads x 2000 sweeps, beta 0.1 -> 5.0, Gamma 3.0 -> 0.01): reads 0,
    499 and 999 recomputed by the oracle, every energy equal to its state's."""
    from spvar_inputs import configs as cf

    inst = cf.instance(cf.CHIMERA8_SA)
    b, g = si.linear_betas(0.1, 5.0, 2000), np.geomspace(3.0, 0.01, 2000)
    _say("[sqa] workload size: chimera8 P=16 1000 reads x 2000 sweeps")
    sp, E = spv.spv_sqa_sample(ctx, spv.Problem.from_instance(inst), b, g, 16, 1000, 11)
    sp, E = sp.cpu().numpy(), E.cpu().numpy()
    for r in (0, 499, 999):
        osp, oE, _ = oracle.sqa_sample(inst, b, g, 16, seed=11, r_begin=r, r_end=r + 1)
        assert np.array_equal(sp[r], osp[0]) and E[r] == oE[0], r
    assert np.array_equal(E, oracle.energy(inst, sp))


def test_sqa_cubic10_gauss_sampled_reads(spv, ctx):
    """The L = 10 Gaussian cube (N = 1000, couplers at scale 2^10, two digits), 16 slices,
    96 reads x 120 sweeps; 8 reads recomputed by the oracle, every energy equal to its state's."""
    inst = si.cubic_lattice(10, "gauss", seed=12, scale_log2=10)
    b, g = _sched(120, 0.2, 3.0, 3.0, 0.05)
    _say("[sqa] cubic10 gauss P=16 96 reads x 120 sweeps")
    sp, E = spv.spv_sqa_sample(ctx, spv.Problem.from_instance(inst), b, g, 16, 96, 44)
    sp, E = sp.cpu().numpy(), E.cpu().numpy()
    osp, oE, _ = oracle.sqa_sample(inst, b, g, 16, seed=44, r_begin=88, r_end=96, threads=8)
    assert np.array_equal(sp[88:], osp) and np.array_equal(E[88:], oE)
    assert np.array_equal(E, oracle.energy(inst, sp))


def test_sqa_rejects_bad_arguments(spv, ctx):
    import paper_1706_07826_amd as m

    inst = si.chimera(2, seed=9)
    Pr = spv.Problem.from_instance(inst)
    b, g = _sched(10)
    for P in (4, 12, 0, 264):
        with pytest.raises(m.SpvError) as ei:
            spv.spv_sqa_sample(ctx, Pr, b, g, P, 4, 1)
        assert ei.value.code == -1
    g0 = g.copy()
    g0[3] = 0.0
    with pytest.raises(m.SpvError) as ei:
        spv.spv_sqa_sample(ctx, Pr, b, g0, 8, 4, 1)
    assert ei.value.code == -1
    with pytest.raises(m.SpvError) as ei:  # Jp at 2^24 and beyond
        gi = si.cubic_lattice(4, "gauss", seed=10, scale_log2=10)
        spv.spv_sqa_sample(ctx, spv.Problem.from_instance(gi), np.full(3, 0.01), np.full(3, 1e-300), 8, 4, 1)
    assert ei.value.code == -4
    # the context stays usable
    sp, E = spv.spv_sqa_sample(ctx, Pr, b, g, 8, 4, 1)
    osp, oE, _ = oracle.sqa_sample(inst, b, g, 8, reads=4, seed=1)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


def test_sqa_empty_problem_zero_reads_and_capacity(spv, ctx):
    import paper_1706_07826_amd as m
    import torch

    b, g = _sched(5)
    empty = si.from_edges(0, [], [], [], [], [], 1)
    sp, E = spv.spv_sqa_sample(ctx, spv.Problem.from_instance(empty), b, g, 8, 3, 1)
    assert tuple(sp.shape) == (3, 0) and np.array_equal(E.cpu().numpy(), np.zeros(3, np.int64))
    inst = si.chimera(2, seed=31)
    sp, E = spv.spv_sqa_sample(ctx, spv.Problem.from_instance(inst), b, g, 8, 0, 1)
    assert tuple(sp.shape) == (0, inst.n) and E.numel() == 0
    # 256 slices of an 800-variable instance: 64 words per variable (200 KiB) exceed a workgroup's LDS
    big = si.chimera(10, seed=32)
    with pytest.raises(m.SpvError) as ei:
        spv.spv_sqa_sample(ctx, spv.Problem.from_instance(big), b, g, 256, 2, 1)
    assert ei.value.code == -5
    torch.cuda.synchronize()


def _with_env(env, fn):
    import os
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return fn()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("name,make,P,reads,sweeps", [CASES[i] for i in (0, 3, 4)], ids=[CASES[i][0] for i in (0, 3, 4)])
def test_sqa_global_instance_forced_small(spv, ctx, name, make, P, reads, sweeps):
    """The instance read from the global image (slices and rows in LDS), forced on small cases."""
    inst = make()
    b, g = _sched(sweeps)
    _say(f"[sqa] global instance forced: {name}")
    Pr = spv.Problem.from_instance(inst)
    sp, E = _with_env({"SPVAR_SQA_BIG": 1}, lambda: spv.spv_sqa_sample(ctx, Pr, b, g, P, reads, 45))
    osp, oE, _ = oracle.sqa_sample(inst, b, g, P, reads=reads, seed=45, threads=8)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


def test_sqa_beyond_lds_cubic20(spv, ctx):
    """The L = 20 Gaussian cube (N = 8000): its records do not fit beside 8 slices, so the
    instance stays in global memory; 6 reads x 20 sweeps against the oracle."""
    inst = si.cubic_lattice(20, "gauss", seed=13, scale_log2=10)
    b, g = _sched(20, 0.2, 3.0, 3.0, 0.05)
    _say("[sqa] beyond LDS: cubic20 gauss P=8")
    sp, E = spv.spv_sqa_sample(ctx, spv.Problem.from_instance(inst), b, g, 8, 6, 46)
    osp, oE, _ = oracle.sqa_sample(inst, b, g, 8, reads=6, seed=46, threads=6)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)
