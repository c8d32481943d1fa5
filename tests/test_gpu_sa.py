"""GPU parity: simulated annealing, energies and iterated SPVAR through the C ABI,
bit for bit against the CPU oracle on the same seeded inputs."""
import sys

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


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _no_edges(n):
    inst = si.from_edges(n, [], [], [], np.arange(1, n + 1) * (-1) ** np.arange(n), np.zeros(n), 1)
    return inst


SMALL = [
    ("chimera3", lambda: si.chimera(3, seed=1), 64, 50, (0.1, 3.0)),
    ("cubic4_ragged_reads", lambda: si.cubic_lattice(4, "pm1", seed=2), 37, 100, (0.1, 3.0)),
    ("sparse50_3colours", lambda: si.random_sparse(50, 3.0, seed=3), 21, 80, (0.1, 4.0)),
    ("cubic4_gauss_two_digits", lambda: si.cubic_lattice(4, "gauss", seed=4, scale_log2=10), 16, 60,
     (0.2, 5.0)),
    ("sparse30_three_digits", lambda: si.random_sparse(30, 10.0, seed=5, scale_log2=14,
                                                       dist=("uniform_nonzero", 32767)), 12, 40,
     (0.05, 2.0)),
    ("cubic5_odd_greedy", lambda: si.cubic_lattice(5, "pm1", seed=6), 9, 30, (0.1, 3.0)),
    ("no_edges", lambda: _no_edges(7), 10, 20, (0.1, 3.0)),
    ("single_spin", lambda: _no_edges(1), 5, 10, (0.5, 1.0)),
    ("zero_sweeps", lambda: si.chimera(2, seed=7), 8, 0, (0.1, 3.0)),
    ("residual", lambda: si.residual_batch(1, parent_M=6, n_min=60, n_max=90, seed=8)[0], 33, 70,
     (0.1, 5.0)),
]


@pytest.mark.parametrize("name,make,reads,sweeps,br", SMALL, ids=[c[0] for c in SMALL])
def test_sa_parity_small(spv, ctx, name, make, reads, sweeps, br):
    inst = make()
    _say(f"[sa] {name} n={inst.n} reads={reads} sweeps={sweeps}")
    P = spv.Problem.from_instance(inst)
    spv.spv_problem_check(ctx, P)
    betas = si.linear_betas(br[0], br[1], sweeps) if sweeps else np.zeros(0)
    seed = 1000 + len(name)
    sp, E = spv.spv_sample(ctx, P, betas, reads, seed)
    osp, oE = oracle.sa_sample(inst, betas, reads=reads, seed=seed, threads=8)
    assert np.array_equal(sp.cpu().numpy(), osp)
    assert np.array_equal(E.cpu().numpy(), oE)


def test_sa_resume_from_state(spv, ctx):
    inst = si.chimera(3, seed=11)
    P = spv.Problem.from_instance(inst)
    betas = si.linear_betas(0.1, 4.0, 60)
    init = si.random_spins(23, inst.n, seed=12)
    import torch
    sp, E = spv.spv_sample(ctx, P, betas[20:], 23, 77, sweep_offset=20,
                           init_spins=torch.as_tensor(init).cuda())
    osp, oE = oracle.sa_sample(inst, betas[20:], reads=23, seed=77, sweep_offset=20, init=init)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


def test_energy_parity(spv, ctx):
    import torch
    for inst in (si.chimera(4, seed=2), si.cubic_lattice(6, "gauss", seed=3, scale_log2=10),
                 si.random_sparse(77, 3.0, seed=4)):
        S = si.random_spins(131, inst.n, seed=inst.n)
        P = spv.Problem.from_instance(inst)
        E = spv.spv_energy(ctx, P, torch.as_tensor(S).cuda())
        assert np.array_equal(E.cpu().numpy(), oracle.energy(inst, S))


def test_sa_parity_chimera8_full_size_sampled_reads(spv, ctx):
    """The full 10,000 reads x 2,000 sweeps launch; the oracle recomputes a sample of reads."""
    cfg = cf.CHIMERA8_SA
    inst = cf.instance(cfg)
    betas = cf.betas(cfg)
    P = spv.Problem.from_instance(inst)
    _say(f"[sa] chimera8 full size: {cfg['reads']} reads x {cfg['sweeps']} sweeps")
    sp, E = spv.spv_sample(ctx, P, betas, cfg["reads"], cfg["seed"])
    sp, E = sp.cpu().numpy(), E.cpu().numpy()
    rng = np.random.default_rng(0)
    picks = sorted(set([0, 1, 2, 3, 4, 4999, 5000, 9995, 9998, 9999] +
                       rng.integers(0, cfg["reads"], 14).tolist()))
    for r in picks:
        osp, oE = oracle.sa_sample(inst, betas, seed=cfg["seed"], r_begin=r, r_end=r + 1)
        assert np.array_equal(sp[r], osp[0]), r
        assert E[r] == oE[0], r
    # every energy equals the recomputed energy of its state
    assert np.array_equal(E, oracle.energy(inst, sp))


def test_ispvar_parity_cubic4_config(spv, ctx):
    cfg = cf.CUBIC4_SA
    inst = cf.instance(cfg)
    betas = cf.betas(cfg)
    P = spv.Problem.from_instance(inst)
    res = spv.spv_ispvar(ctx, P, betas, cfg["reads"], cfg["seed"], cfg["rounds"], cfg["elite"],
                         cfg["theta"], cfg["gauge"])
    ores = oracle.ispvar(inst, betas, cfg["reads"], cfg["seed"], cfg["rounds"], cfg["elite"],
                         cfg["theta"], cfg["gauge"])
    assert res["rounds_run"] == ores["rounds_run"]
    assert np.array_equal(res["round_info"], ores["round_info"])
    assert np.array_equal(res["fixed_mask"].cpu().numpy(), ores["fixed_mask"])
    assert np.array_equal(res["fixed_val"].cpu().numpy(), ores["fixed_val"])
