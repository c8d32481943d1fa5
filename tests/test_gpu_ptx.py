"""GPU parity of tempering with the ladder split over several workgroups
(boundary replica exchange through L2, instance in LDS or read from global
memory), bit for bit against the CPU oracle; plus the single-workgroup kernel
forced on ladders the split would otherwise take."""
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


def _check(got, want):
    for key in ("final_spins", "final_E", "top_E", "top_count", "top_spins"):
        assert np.array_equal(got[key].cpu().numpy(), want[key]), key


CASES = [
    # name, instance, K, runs, chains, sweeps, icm, groups, big, sweep_offset
    ("cubic4_K8_G2", lambda: si.cubic_lattice(4, "gauss", seed=1, scale_log2=10), 8, 3, 1, 100, None, 2, 0, 0),
    ("cubic4_K8_G2_icm", lambda: si.cubic_lattice(4, "gauss", seed=2, scale_log2=10), 8, 2, 2, 90, (0, 8), 2, 0, 0),
    ("cubic4_K12_G3_icm_window_big", lambda: si.cubic_lattice(4, "gauss", seed=3, scale_log2=10), 12, 2, 2, 75,
     (2, 10), 3, 1, 0),
    ("chimera2_K12_G2_uneven", lambda: si.chimera(2, seed=4), 12, 3, 1, 61, None, 2, 0, 0),
    ("sparse40_K16_G4_odd_offset", lambda: si.random_sparse(40, 3.0, seed=5), 16, 2, 2, 51, (0, 16), 4, 0, 7),
    ("cubic6_pm1_K8_G2_big", lambda: si.cubic_lattice(6, "pm1", seed=6), 8, 4, 2, 80, (0, 8), 2, 1, 0),
    ("zero_sweeps_G2", lambda: si.chimera(2, seed=7), 8, 2, 1, 0, None, 2, 0, 0),
    ("one_sweep_G2", lambda: si.chimera(2, seed=8), 8, 2, 1, 1, None, 2, 0, 1),
    ("K4_G1_forced_split", lambda: si.chimera(2, seed=9), 4, 3, 2, 40, (0, 4), 1, 0, 0),
    # 8 slots per group with the cluster moves from slot 1: a batch of pairs spans two quad words
    ("sparse40_K16_G2_icm_straddling_batch", lambda: si.random_sparse(40, 3.0, seed=12), 16, 2, 2, 60, (1, 15), 2,
     0, 0),
    # n not a multiple of 4: the top-10 states copied and compared byte by byte
    ("sparse42_K8_G2_icm_ragged_n", lambda: si.random_sparse(42, 3.0, seed=14), 8, 2, 2, 70, (0, 8), 2, 0, 0),
    ("cubic4_K16_G2_icm_straddling_batch_big", lambda: si.cubic_lattice(4, "gauss", seed=13, scale_log2=10), 16, 1,
     2, 45, (3, 14), 2, 1, 0),
    # groups of 2 slots (more groups than quads, cluster moves on): each group owns half of
    # every quad word it holds, the upper half when its first slot is 2 mod 4
    ("cubic4_K8_G4_icm_half_quads", lambda: si.cubic_lattice(4, "gauss", seed=15, scale_log2=10), 8, 2, 2, 80,
     (0, 8), 4, 0, 0),
    ("sparse40_K16_G8_icm_half_quads_window_offset", lambda: si.random_sparse(40, 3.0, seed=16), 16, 2, 2, 61,
     (3, 13), 8, 0, 5),
    ("cubic4_K12_G6_icm_half_quads_big", lambda: si.cubic_lattice(4, "gauss", seed=17, scale_log2=10), 12, 1, 2,
     50, (0, 12), 6, 1, 0),
    ("sparse42_K8_G4_icm_half_quads_ragged_n", lambda: si.random_sparse(42, 3.0, seed=18), 8, 2, 2, 40, (0, 8), 4,
     0, 0),
    ("chimera2_K8_G4_icm_half_quads_one_digit", lambda: si.chimera(2, seed=19), 8, 2, 2, 45, (0, 8), 4, 0, 1),
    ("zero_sweeps_G4_half_quads", lambda: si.chimera(2, seed=20), 8, 2, 2, 0, (0, 8), 4, 0, 0),
    ("cubic10_K8_G4_icm_half_quads_wide", lambda: si.cubic_lattice(10, "gauss", seed=21, scale_log2=10), 8, 1, 2,
     30, (0, 8), 4, 0, 0),
    # groups of 1 slot (a quarter of each quad word; the lower and upper boundary pairs on
    # alternate sweeps)
    ("cubic4_K8_G8_icm_single_slots", lambda: si.cubic_lattice(4, "gauss", seed=22, scale_log2=10), 8, 2, 2, 80,
     (0, 8), 8, 0, 0),
    ("sparse40_K16_G16_icm_single_slots_window_offset", lambda: si.random_sparse(40, 3.0, seed=23), 16, 2, 2, 63,
     (3, 13), 16, 0, 3),
    ("cubic4_K12_G12_icm_single_slots_big", lambda: si.cubic_lattice(4, "gauss", seed=24, scale_log2=10), 12, 1, 2,
     50, (0, 12), 12, 1, 0),
    ("sparse42_K8_G8_icm_single_slots_ragged_n", lambda: si.random_sparse(42, 3.0, seed=25), 8, 2, 2, 40, (0, 8),
     8, 0, 1),
    ("chimera2_K12_G7_icm_single_slots_one_digit", lambda: si.chimera(2, seed=26), 12, 2, 2, 51, (0, 12), 7, 0, 0),
    ("zero_sweeps_G8_single_slots", lambda: si.chimera(2, seed=27), 8, 2, 2, 0, (0, 8), 8, 0, 0),
    ("one_sweep_G8_single_slots_odd_offset", lambda: si.chimera(2, seed=28), 8, 2, 2, 1, (0, 8), 8, 0, 1),
    ("cubic10_K8_G8_icm_single_slots_wide", lambda: si.cubic_lattice(10, "gauss", seed=29, scale_log2=10), 8, 1, 2,
     30, (0, 8), 8, 0, 0),
    # many waves per workgroup on the cluster moves (1024 threads)
    ("cubic10_K8_G2_icm_wide", lambda: si.cubic_lattice(10, "gauss", seed=10, scale_log2=10), 8, 2, 2, 30,
     (0, 8), 2, 0, 0),
    ("cubic10_K8_G2_icm_wide_big", lambda: si.cubic_lattice(10, "gauss", seed=11, scale_log2=10), 8, 1, 2, 30,
     (0, 8), 2, 1, 1),
]


@pytest.mark.parametrize("name,make,K,runs,chains,sweeps,icm,groups,big,off", CASES, ids=[c[0] for c in CASES])
def test_split_pt_parity(spv, ctx, monkeypatch, name, make, K, runs, chains, sweeps, icm, groups, big, off):
    inst = make()
    print(f"[ptx] {name} n={inst.n} K={K} runs={runs} chains={chains} G={groups} big={big}", flush=True)
    monkeypatch.setenv("SPVAR_PT_SPLIT", "1")
    monkeypatch.setenv("SPVAR_PT_GROUPS", str(groups))
    monkeypatch.setenv("SPVAR_PT_BIG", str(big))
    P = spv.Problem.from_instance(inst)
    betas = si.geometric_betas(0.2, 5.0 if inst.scale_log2 else 3.0, K)
    got = spv.spv_pt_sample(ctx, P, betas, runs, chains, sweeps, seed=90 + K, sweep_offset=off, icm=icm)
    want = oracle.pt_sample(inst, betas, runs, chains, sweeps, seed=90 + K, sweep_offset=off, icm=icm, threads=8)
    _check(got, want)


@pytest.mark.parametrize("esum", ["0", "1"])
def test_single_slot_groups_with_and_without_gathered_cluster_terms(spv, ctx, monkeypatch, esum):
    """Groups of one slot pair either gather each disagreeing site's cluster energy term in the
    join scan (the default) or run the separate energy pass over the records: both bit for bit
    against the oracle."""
    inst = si.cubic_lattice(5, "gauss", seed=31, scale_log2=10)
    monkeypatch.setenv("SPVAR_PT_SPLIT", "1")
    monkeypatch.setenv("SPVAR_PT_GROUPS", "12")
    monkeypatch.setenv("SPVAR_PT_ESUM", esum)
    P = spv.Problem.from_instance(inst)
    betas = si.geometric_betas(0.2, 5.0, 12)
    got = spv.spv_pt_sample(ctx, P, betas, 2, 2, 60, seed=77, icm=(0, 12))
    want = oracle.pt_sample(inst, betas, 2, 2, 60, seed=77, icm=(0, 12), threads=4)
    _check(got, want)


@pytest.mark.parametrize("K,chains,icm", [(8, 1, None), (8, 2, (0, 8)), (12, 2, (3, 9))])
def test_single_workgroup_kernel_forced(spv, ctx, monkeypatch, K, chains, icm):
    monkeypatch.setenv("SPVAR_PT_SPLIT", "0")
    inst = si.cubic_lattice(4, "gauss", seed=20 + K, scale_log2=10)
    P = spv.Problem.from_instance(inst)
    betas = si.geometric_betas(0.2, 5.0, K)
    got = spv.spv_pt_sample(ctx, P, betas, 3, chains, 70, seed=K, icm=icm)
    want = oracle.pt_sample(inst, betas, 3, chains, 70, seed=K, icm=icm, threads=3)
    _check(got, want)


def test_cubic20_pticm_config_shape(spv, ctx):
    """The N=8000 PT-ICM shape (40 slots x 2 chains, Houdayer at every slot,
    one run) on the default plan (instance in global memory, one workgroup per
    slot), a short schedule against the oracle."""
    cfg = cf.CUBIC20_PTICM
    inst = cf.instance(cfg)
    betas = cf.betas(cfg)
    K = betas.size
    print(f"[ptx] cubic20 n={inst.n} K={K}", flush=True)
    P = spv.Problem.from_instance(inst)
    got = spv.spv_pt_sample(ctx, P, betas, 1, cfg["chains"], 40, seed=cfg["seed"], icm=(0, K))
    want = oracle.pt_sample(inst, betas, 1, cfg["chains"], 40, seed=cfg["seed"], icm=(0, K), threads=1)
    _check(got, want)
    assert np.array_equal(got["final_E"].cpu().numpy().reshape(-1),
                          oracle.energy(inst, got["final_spins"].cpu().numpy().reshape(-1, inst.n)))


def test_cubic20_pticm_full_sweeps_properties(spv, ctx):
    """The full N=8000 PT-ICM launch (10^4 sweeps, the bench's plan): every final energy and
    every top-10 energy equals the recomputed energy of its state, each list is full, sorted
    and free of repeated states (the oracle replays the short schedule above bit for bit)."""
    cfg = cf.CUBIC20_PTICM
    inst = cf.instance(cfg)
    betas = cf.betas(cfg)
    K = betas.size
    print(f"[ptx] cubic20 full {cfg['sweeps']} sweeps", flush=True)
    P = spv.Problem.from_instance(inst)
    got = spv.spv_pt_sample(ctx, P, betas, 1, cfg["chains"], cfg["sweeps"], seed=cfg["seed"], icm=(0, K))
    fs, fe = got["final_spins"].cpu().numpy(), got["final_E"].cpu().numpy()
    assert np.array_equal(fe.reshape(-1), oracle.energy(inst, fs.reshape(-1, inst.n)))
    te, ts, tc = (got[k].cpu().numpy() for k in ("top_E", "top_spins", "top_count"))
    assert np.all(tc == 10)
    assert np.all(np.diff(te, axis=-1) >= 0)
    assert np.array_equal(te.reshape(-1), oracle.energy(inst, ts.reshape(-1, inst.n)))
    lists = ts.reshape(-1, 10, inst.n)
    for L in lists:
        assert len({row.tobytes() for row in L}) == 10


def test_bounded_neighbour_wait_reports_and_recovers(spv, ctx, monkeypatch):
    """Failure handling forced from the host: with a spin limit of 0 a workgroup
    whose neighbour has not yet published gives up at once instead of waiting.
    The call must return, every list of a workgroup that stopped reads
    top_count = -1 (and sample assembly refuses it), the others stay valid, and
    the next call with the normal limit is exact again."""
    inst = si.cubic_lattice(6, "gauss", seed=41, scale_log2=10)
    P = spv.Problem.from_instance(inst)
    betas = si.geometric_betas(0.2, 5.0, 16)
    monkeypatch.setenv("SPVAR_PT_SPLIT", "1")
    monkeypatch.setenv("SPVAR_PT_GROUPS", "4")
    monkeypatch.setenv("SPVAR_PT_SPIN", "0")
    got = spv.spv_pt_sample(ctx, P, betas, 3, 2, 200, seed=5, icm=(0, 16))
    tc = got["top_count"].cpu().numpy()
    assert set(np.unique(tc)).issubset(set(range(-1, 11)))
    if (tc < 0).any():
        with pytest.raises(spv.SpvError, match="EINVAL"):
            spv.spv_top_sample(ctx, got)
    monkeypatch.setenv("SPVAR_PT_SPIN", str(1 << 24))
    got = spv.spv_pt_sample(ctx, P, betas, 3, 2, 200, seed=5, icm=(0, 16))
    want = oracle.pt_sample(inst, betas, 3, 2, 200, seed=5, icm=(0, 16), threads=3)
    _check(got, want)
