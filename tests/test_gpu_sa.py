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


@pytest.mark.parametrize("shape", [{}, {"SPVAR_SA_WPL": 1, "SPVAR_SA_THREADS": 512}], ids=["w2", "w1"])
def test_sa_streamed_launch_equals_plain(spv, ctx, shape):
    """Chimera N=512, 10,000 reads (more workgroups than stay resident): the streamed launch
    (chunks of sweeps through global memory) and the plain launch give identical samples."""
    cfg = cf.CHIMERA8_SA
    inst = cf.instance(cfg)
    betas = cf.betas(cfg)[::7]  # 286 sweeps: several chunks, the last one shorter
    P = spv.Problem.from_instance(inst)
    _say(f"[sa] streamed vs plain {shape}: {cfg['reads']} reads x {len(betas)} sweeps")
    run = lambda: [t.cpu().numpy() for t in spv.spv_sample(ctx, P, betas, cfg["reads"], 99)]
    s1, e1 = _with_env(dict(shape), run)
    s0, e0 = _with_env(dict(shape, SPVAR_SA_STREAM=0), run)
    assert np.array_equal(s1, s0) and np.array_equal(e1, e0)
    osp, oE = oracle.sa_sample(inst, betas, seed=99, r_begin=9990, r_end=10000)
    assert np.array_equal(s1[9990:], osp) and np.array_equal(e1[9990:], oE)


def test_sa_streamed_launch_waits_for_earlier_chunks(spv, ctx):
    """A grid larger than the task front: tasks wait for their group's previous chunk
    (release/acquire flags); the sample equals the oracle's, ragged reads included."""
    inst = si.cubic_lattice(4, "pm1", seed=5)
    betas = si.linear_betas(0.1, 3.0, 200)
    P = spv.Problem.from_instance(inst)
    _say("[sa] streamed launch with dependent chunks: 30 reads, grid 16")
    S, E = _with_env({"SPVAR_SA_STREAM": 16}, lambda: spv.spv_sample(ctx, P, betas, 30, 1234))
    osp, oE = oracle.sa_sample(inst, betas, reads=30, seed=1234)
    assert np.array_equal(S.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


def test_sa_streamed_launch_abandoned_wait_is_marked(spv, ctx):
    """With a wait limit of one poll, a task that finds its group's previous chunk unfinished
    gives up; the kernel still ends and every read of such a group reports INT64_MIN."""
    inst = si.cubic_lattice(4, "pm1", seed=5)
    betas = si.linear_betas(0.1, 3.0, 200)
    P = spv.Problem.from_instance(inst)
    _say("[sa] streamed launch, wait limit 1")
    S, E = _with_env({"SPVAR_SA_STREAM": 16, "SPVAR_SA_SPIN": 1},
                     lambda: spv.spv_sample(ctx, P, betas, 30, 1234))
    osp, oE = oracle.sa_sample(inst, betas, reads=30, seed=1234)
    En = E.cpu().numpy()
    marked = En == np.iinfo(np.int64).min
    assert np.all(marked | (En == oE))
    assert set(np.unique(S.cpu().numpy())).issubset({-1, 1})
    # Persistence refuses a sample holding marked reads (it would fix from abandoned states).
    fx = spv.spv_persist_fix(ctx, P, S, E, 0.1, 1.0, 2)
    if marked.any():
        with pytest.raises(spv.SpvError) as ei:
            fx.info()
        assert ei.value.code == -1
    else:
        want = oracle.persist_fix(inst, osp, oE, 0.1, 1.0, 2)
        assert fx.info()["n_free"] == want["n_free"]
    # ISPVAR under the same wait limit: the oracle's fixes, or an error, never a silent fix.
    def ispvar():
        return spv.spv_ispvar(ctx, P, betas, 30, 1234, 2, 0.1, 1.0, 2)
    try:
        fm, fv, info = _with_env({"SPVAR_SA_STREAM": 16, "SPVAR_SA_SPIN": 1}, ispvar)
    except spv.SpvError as e:
        assert e.code == -1
    else:
        want = oracle.ispvar(inst, betas, 30, 1234, 2, 0.1, 1.0, 2)
        assert np.array_equal(fv.cpu().numpy()[:inst.n], want["fixed_val"])


def test_persist_fix_rejects_marked_energy(spv, ctx):
    """A sample whose energies hold INT64_MIN (the mark of an abandoned streamed read) is
    refused by persistence with SPV_EINVAL in info[7], on the device as in the oracle."""
    inst = si.chimera(2, seed=21)
    betas = si.linear_betas(0.1, 3.0, 50)
    P = spv.Problem.from_instance(inst)
    S, E = spv.spv_sample(ctx, P, betas, 40, 5)
    E[17] = np.iinfo(np.int64).min
    _say("[sa] persistence on a planted INT64_MIN energy")
    with pytest.raises(spv.SpvError) as ei:
        spv.spv_persist_fix(ctx, P, S, E, 0.25, 1.0, 0).info()
    assert ei.value.code == -1
    with pytest.raises(oracle.OracleError):
        oracle.persist_fix(inst, S.cpu().numpy(), E.cpu().numpy(), 0.25, 1.0, 0)
    # the context stays usable
    E2 = spv.spv_energy(ctx, P, S)
    fx = spv.spv_persist_fix(ctx, P, S, E2, 0.25, 1.0, 0)
    want = oracle.persist_fix(inst, S.cpu().numpy(), E2.cpu().numpy(), 0.25, 1.0, 0)
    assert fx.info()["offset"] == want["offset"]


@pytest.mark.parametrize("name,make,reads,sweeps,br", SMALL[:6], ids=[c[0] for c in SMALL[:6]])
def test_sa_parity_small_two_words_per_lane(spv, ctx, name, make, reads, sweeps, br):
    """The byte-parallel body with both quad words of a site in one lane (the shape used when
    the workgroups outnumber the CUs), forced on small cases, against the oracle."""
    inst = make()
    betas = si.linear_betas(br[0], br[1], sweeps)
    P = spv.Problem.from_instance(inst)
    seed = 4242
    _say(f"[sa] {name} two words per lane")
    sp, E = _with_env({"SPVAR_SA_WPL": 2, "SPVAR_SA_THREADS": 256}, lambda: spv.spv_sample(ctx, P, betas, reads, seed))
    osp, oE = oracle.sa_sample(inst, betas, reads=reads, seed=seed, threads=8)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


def test_sa_streamed_launch_resumes_from_states(spv, ctx):
    """A streamed launch that starts from caller states at a sweep offset (resume) gives the
    oracle's sample."""
    import torch

    inst = si.chimera(3, seed=21)
    betas = si.linear_betas(0.1, 3.0, 300)
    P = spv.Problem.from_instance(inst)
    reads = 50
    init = si.random_spins(reads, inst.n, seed=22)
    _say("[sa] streamed resume: 50 reads from caller states, sweep offset 40, grid 8")
    S, E = _with_env({"SPVAR_SA_STREAM": 8},
                     lambda: spv.spv_sample(ctx, P, betas[40:], reads, 555, sweep_offset=40,
                                            init_spins=torch.as_tensor(init).cuda()))
    osp, oE = oracle.sa_sample(inst, betas[40:], reads=reads, seed=555, sweep_offset=40, init=init)
    assert np.array_equal(S.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


@pytest.mark.parametrize("name,make,reads,sweeps,br", [c for c in SMALL[:3]] + [SMALL[5], SMALL[9]],
                         ids=[c[0] for c in SMALL[:3]] + [SMALL[5][0], SMALL[9][0]])
@pytest.mark.parametrize("shape", [{}, {"SPVAR_SA_WPL": 2, "SPVAR_SA_THREADS": 256}], ids=["default", "w2"])
def test_sa_global_instance_forced_small(spv, ctx, name, make, reads, sweeps, br, shape):
    """The byte-parallel body with its instance in global memory (records read through L2,
    spins in LDS), forced on small cases, against the oracle."""
    inst = make()
    betas = si.linear_betas(br[0], br[1], sweeps)
    P = spv.Problem.from_instance(inst)
    _say(f"[sa] {name} global instance {shape}")
    sp, E = _with_env(dict(shape, SPVAR_SA_BIG=1), lambda: spv.spv_sample(ctx, P, betas, reads, 31))
    osp, oE = oracle.sa_sample(inst, betas, reads=reads, seed=31, threads=8)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


@pytest.mark.parametrize("M,reads,sweeps", [(20, 40, 60), (32, 16, 30)], ids=["chimera20_n3200", "chimera32_n8192"])
def test_sa_beyond_lds_matches_oracle(spv, ctx, M, reads, sweeps):
    """Chimera instances whose records do not fit the LDS (N = 3200 and 8192) take the
    global-instance body automatically; the sample equals the oracle's."""
    inst = si.chimera(M, seed=40 + M)
    betas = si.linear_betas(0.1, 5.0, sweeps)
    P = spv.Problem.from_instance(inst)
    _say(f"[sa] beyond LDS: chimera{M} n={inst.n}")
    sp, E = spv.spv_sample(ctx, P, betas, reads, 77)
    osp, oE = oracle.sa_sample(inst, betas, reads=reads, seed=77, threads=8)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


def test_sa_beyond_lds_streamed_sampled_reads(spv, ctx):
    """N = 3200 with 10,000 reads x 200 sweeps: the streamed launch over the global instance;
    sampled reads recomputed by the oracle, every energy equal to its state's."""
    inst = si.chimera(20, seed=61)
    betas = si.linear_betas(0.1, 5.0, 200)
    P = spv.Problem.from_instance(inst)
    _say("[sa] beyond LDS, streamed: chimera20 10000 reads x 200 sweeps")
    sp, E = spv.spv_sample(ctx, P, betas, 10000, 5)
    shape = spv.spv_sample_last_shape(ctx)
    assert shape["chunks"] > 1
    sp, E = sp.cpu().numpy(), E.cpu().numpy()
    for r in (0, 1, 4097, 9999):
        osp, oE = oracle.sa_sample(inst, betas, seed=5, r_begin=r, r_end=r + 1)
        assert np.array_equal(sp[r], osp[0]) and E[r] == oE[0], r
    assert np.array_equal(E, oracle.energy(inst, sp))


def _x_bound(inst):
    a, b, w = inst.edges()
    xb = np.abs(np.asarray(inst.h, np.int64)).copy()
    np.add.at(xb, a, np.abs(w))
    np.add.at(xb, b, np.abs(w))
    return int(xb.max())


GENERAL = [
    ("cubic4_one_digit_wide_table", lambda: si.cubic_lattice(4, "gauss", seed=4, scale_log2=5), 20, 50, (0.1, 3.0)),
    SMALL[3],
    SMALL[4],
]


@pytest.mark.parametrize("name,make,reads,sweeps,br", GENERAL, ids=[c[0] for c in GENERAL])
def test_sa_general_body_global_instance_forced_small(spv, ctx, name, make, reads, sweeps, br):
    """The general body (tables wider than one byte-parallel row) reading its instance
    from global memory, forced on small cases, against the oracle."""
    inst = make()
    if name.startswith("cubic4_one"):
        assert 256 <= _x_bound(inst) < 512  # one digit, but too wide for the byte-parallel body
    betas = si.linear_betas(br[0], br[1], sweeps)
    P = spv.Problem.from_instance(inst)
    _say(f"[sa] general body, global instance: {name} n={inst.n}")
    sp, E = _with_env({"SPVAR_SA_BIG": 1}, lambda: spv.spv_sample(ctx, P, betas, reads, 32))
    assert spv.spv_sample_last_shape(ctx)["global_instance"] == 1
    osp, oE = oracle.sa_sample(inst, betas, reads=reads, seed=32, threads=8)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


def test_sa_general_body_global_instance_ragged_reads_and_resume(spv, ctx):
    """The global-instance general body with a read count that leaves the last quad partly
    empty, from caller states at a sweep offset, against the oracle."""
    import torch

    inst = si.cubic_lattice(5, "gauss", seed=12, scale_log2=10)
    betas = si.linear_betas(0.1, 3.0, 70)
    P = spv.Problem.from_instance(inst)
    reads = 13
    init = si.random_spins(reads, inst.n, seed=23)
    _say("[sa] general body, global instance: 13 reads from caller states, sweep offset 30")
    sp, E = _with_env({"SPVAR_SA_BIG": 1},
                      lambda: spv.spv_sample(ctx, P, betas[30:], reads, 556, sweep_offset=30,
                                             init_spins=torch.as_tensor(init).cuda()))
    assert spv.spv_sample_last_shape(ctx)["global_instance"] == 1
    osp, oE = oracle.sa_sample(inst, betas[30:], reads=reads, seed=556, sweep_offset=30, init=init)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


GENERAL_BIG = [
    ("cubic20_gauss_n8000", lambda: si.cubic_lattice(20, "gauss", seed=9, scale_log2=10), 12, 30),
    ("sparse12000_three_digits", lambda: si.random_sparse(12000, 10.0, seed=5, scale_log2=14,
                                                          dist=("uniform_nonzero", 32767)), 8, 10),
]


@pytest.mark.parametrize("name,make,reads,sweeps", GENERAL_BIG, ids=[c[0] for c in GENERAL_BIG])
def test_sa_general_body_beyond_lds_matches_oracle(spv, ctx, name, make, reads, sweeps):
    """Instances with multi-digit tables whose records do not fit the LDS (the L = 20
    Gaussian cube, N = 8000; a sparse N = 12,000 graph of degree up to 24) take the
    global-instance general body automatically; the sample equals the oracle's."""
    inst = make()
    betas = si.linear_betas(0.1, 3.0, sweeps)
    P = spv.Problem.from_instance(inst)
    _say(f"[sa] general body beyond LDS: {name} n={inst.n}")
    sp, E = spv.spv_sample(ctx, P, betas, reads, 78)
    assert spv.spv_sample_last_shape(ctx)["global_instance"] == 1
    osp, oE = oracle.sa_sample(inst, betas, reads=reads, seed=78, threads=8)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


def test_zero_sweeps_on_a_fresh_context_reads_no_table(spv):
    """Regression: with no sweeps no acceptance table is uploaded, so the general body (and SQA)
    must not read one; on a fresh context the table pointer is not even allocated."""
    ctx2 = spv.Context(0)
    inst = si.cubic_lattice(4, "gauss", seed=4, scale_log2=10)  # multi-digit: the general body
    P = spv.Problem.from_instance(inst)
    sp, E = spv.spv_sample(ctx2, P, np.zeros(0), 9, 3)
    osp, oE = oracle.sa_sample(inst, np.zeros(0), reads=9, seed=3)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)
    ctx3 = spv.Context(0)
    sp, E = spv.spv_sqa_sample(ctx3, P, np.zeros(0), np.zeros(0), 8, 5, 4)
    osp, oE, _ = oracle.sqa_sample(inst, np.zeros(0), np.zeros(0), 8, reads=5, seed=4)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)
