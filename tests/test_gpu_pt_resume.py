"""GPU parity of the tempering checkpoint through the C ABI (Sec. III.D.1 runs continued from
their final states and top-10 lists), on the single-workgroup kernel and on ladders split over
workgroups (instance in LDS or in global memory):

* N sweeps, then M sweeps resumed from the first call's outputs with sweep_offset = N, equal
  one (N + M)-sweep call on the device and the oracle's uninterrupted run, also when continued
  in place (the outputs written over the checkpoint) and across a change of layout;
* an arbitrary checkpoint (lists with fewer entries, a count of -1 and of 11, spin bytes other
  than +-1) resumes exactly as the oracle resumes it."""
import numpy as np
import pytest
import torch

import oracle
import spvar_inputs as si

pytestmark = pytest.mark.gpu

KEYS = ("final_spins", "final_E", "top_spins", "top_E", "top_count")


@pytest.fixture(scope="module")
def spv():
    import paper_1706_07826_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(spv):
    return spv.Context(0)


def _layout(monkeypatch, split, groups=1, big=0):
    monkeypatch.setenv("SPVAR_PT_SPLIT", "1" if split else "0")
    monkeypatch.setenv("SPVAR_PT_GROUPS", str(groups))
    monkeypatch.setenv("SPVAR_PT_BIG", str(big))


def _host(res):
    return {k: res[k].cpu().numpy() for k in KEYS}


def _check(got, want):
    for key in KEYS:
        assert np.array_equal(got[key], want[key]), key


CASES = [
    # name, instance, K, runs, chains, icm, split, groups, big
    ("single_K6_chains1", lambda: si.cubic_lattice(4, "gauss", seed=1, scale_log2=10), 6, 2, 1, None, 0, 1, 0),
    ("single_K5_straddling_quads", lambda: si.chimera(2, seed=2), 5, 3, 1, None, 0, 1, 0),
    ("single_K8_icm", lambda: si.cubic_lattice(4, "gauss", seed=3, scale_log2=10, h_dist="gauss"), 8, 2, 2,
     (0, 8), 0, 1, 0),
    ("split_K8_G2_icm", lambda: si.cubic_lattice(4, "gauss", seed=4, scale_log2=10), 8, 2, 2, (0, 8), 1, 2, 0),
    ("split_K12_G3_big_window", lambda: si.random_sparse(40, 3.0, seed=5), 12, 2, 2, (2, 10), 1, 3, 1),
    ("split_K8_G4_icm_half_quads", lambda: si.cubic_lattice(4, "gauss", seed=6, scale_log2=10), 8, 2, 2, (0, 8), 1,
     4, 0),
    ("split_K8_G8_icm_single_slots", lambda: si.cubic_lattice(4, "gauss", seed=7, scale_log2=10), 8, 2, 2, (0, 8),
     1, 8, 0),
]


@pytest.mark.parametrize("name,make,K,runs,chains,icm,split,groups,big", CASES, ids=[c[0] for c in CASES])
def test_split_run_equals_one_run(spv, ctx, monkeypatch, name, make, K, runs, chains, icm, split, groups, big):
    inst = make()
    _layout(monkeypatch, split, groups, big)
    P = spv.Problem.from_instance(inst)
    betas = si.geometric_betas(0.2, 5.0 if inst.scale_log2 else 3.0, K)
    N, M, seed = 23, 41, 70 + K
    print(f"[pt-resume] {name} n={inst.n} K={K} runs={runs} chains={chains} N={N} M={M}", flush=True)
    whole = spv.spv_pt_sample(ctx, P, betas, runs, chains, N + M, seed, icm=icm)
    first = spv.spv_pt_sample(ctx, P, betas, runs, chains, N, seed, icm=icm)
    rest = spv.spv_pt_sample(ctx, P, betas, runs, chains, M, seed, sweep_offset=N, icm=icm, resume=first)
    want = oracle.pt_sample(inst, betas, runs, chains, N + M, seed=seed, icm=icm, threads=4)
    _check(_host(whole), want)
    _check(_host(rest), want)
    # continued in place: the outputs overwrite the checkpoint tensors
    ck = {k: first[k].clone() for k in KEYS}
    again = spv.spv_pt_sample(ctx, P, betas, runs, chains, M, seed, sweep_offset=N, icm=icm, resume=ck,
                              in_place=True)
    assert all(again[k] is ck[k] for k in KEYS)
    _check(_host(ck), want)


def test_checkpoint_moves_between_layouts(spv, ctx, monkeypatch):
    inst = si.cubic_lattice(4, "gauss", seed=6, scale_log2=10)
    P = spv.Problem.from_instance(inst)
    K, runs, chains, icm = 8, 2, 2, (0, 8)
    betas = si.geometric_betas(0.2, 5.0, K)
    print("[pt-resume] split G=2 checkpoint resumed on one workgroup, then split G=2 big", flush=True)
    _layout(monkeypatch, 1, 2, 0)
    a = spv.spv_pt_sample(ctx, P, betas, runs, chains, 30, 5, icm=icm)
    _layout(monkeypatch, 0)
    b = spv.spv_pt_sample(ctx, P, betas, runs, chains, 30, 5, sweep_offset=30, icm=icm, resume=a)
    _layout(monkeypatch, 1, 2, 1)
    c = spv.spv_pt_sample(ctx, P, betas, runs, chains, 20, 5, sweep_offset=60, icm=icm, resume=b)
    _check(_host(c), oracle.pt_sample(inst, betas, runs, chains, 80, seed=5, icm=icm, threads=4))


@pytest.mark.parametrize("split,groups,big", [(0, 1, 0), (1, 2, 0), (1, 2, 1)])
def test_arbitrary_checkpoint_matches_oracle(spv, ctx, monkeypatch, split, groups, big):
    inst = si.cubic_lattice(4, "gauss", seed=7, scale_log2=10)
    n, K, runs, chains, icm = inst.n, 8, 2, 2, (1, 7)
    half = K // 2
    betas = si.geometric_betas(0.2, 5.0, K)
    ck = oracle.pt_sample(inst, betas, runs, chains, 40, seed=8, icm=icm)
    rng = np.random.default_rng(3)
    ck["top_count"][0, 0, 1] = 4
    ck["top_count"][0, 1, 0] = -1
    ck["top_count"][1, 0, 3] = 11
    ck["top_count"][1, 1, 2] = 0
    ts = ck["top_spins"]
    ck["top_spins"] = np.where(ts > 0, rng.integers(1, 128, ts.shape), np.where(ts < 0, -3, 0)).astype(np.int8)
    fs = ck["final_spins"]
    ck["final_spins"] = np.where(fs > 0, 9, rng.integers(-128, 1, fs.shape)).astype(np.int8)
    want = oracle.pt_sample(inst, betas, runs, chains, 35, seed=8, sweep_offset=40, icm=icm, resume=ck)
    assert want["top_count"][0, 1, 0] == -1 and want["top_count"][1, 0, 3] == -1
    _layout(monkeypatch, split, groups, big)
    P = spv.Problem.from_instance(inst)
    dck = {k: torch.from_numpy(np.ascontiguousarray(ck[k])).to(ctx.device) for k in KEYS}
    print(f"[pt-resume] arbitrary checkpoint split={split} G={groups} big={big}", flush=True)
    got = spv.spv_pt_sample(ctx, P, betas, runs, chains, 35, 8, sweep_offset=40, icm=icm, resume=dck)
    _check(_host(got), want)
    with pytest.raises(spv.SpvError):
        spv.spv_pt_sample(ctx, P, betas, runs, chains, 5, 8, icm=icm,
                          resume={"final_spins": dck["final_spins"], "top_count": dck["top_count"]})
