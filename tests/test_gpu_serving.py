"""Serving loop (continuous batching over execution slots): every request's
outputs are bit-identical to the same call made alone, whatever else is in
flight, and a subset is checked against the oracle.  Admission honours the
LDS budget (FIFO, one at a time when only one fits) and rejects requests that
can never fit."""
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


def _mix():
    """A mixed stream of SA and PT requests of different sizes, some with persistence."""
    reqs = []
    for k in range(10):
        inst = si.chimera(2 + k % 3, seed=100 + k)
        sweeps = 30 + 17 * k
        reqs.append(dict(kind="sa", inst=inst, betas=si.linear_betas(0.1, 3.0, sweeps), reads=24 + 13 * k,
                         seed=500 + k, fix=(0.2, 0.9, k % 3) if k % 2 == 0 else None))
    for k in range(5):
        inst = si.cubic_lattice(3 + k % 2, "gauss", seed=200 + k, scale_log2=10)
        K = 6 + 2 * (k % 2)
        reqs.append(dict(kind="pt", inst=inst, betas=si.geometric_betas(0.2, 5.0, K), runs=2 + k % 3,
                         chains=2 if k % 2 else 1, sweeps=60 + 10 * k, seed=700 + k,
                         icm=(0, K) if k % 2 else None, fix=(0.2, 1.0, 2) if k != 2 else None))
    return reqs


def _alone(spv, ctx, r, P):
    import torch
    if r["kind"] == "sa":
        S, E = spv.spv_sample(ctx, P, r["betas"], r["reads"], r["seed"])
        out = dict(spins=S, energies=E)
    elif r["kind"] == "sqa":
        S, E = spv.spv_sqa_sample(ctx, P, r["betas"], r["gammas"], r["trotter"], r["reads"], r["seed"])
        out = dict(spins=S, energies=E)
    else:
        out = spv.spv_pt_sample(ctx, P, r["betas"], r["runs"], r["chains"], r["sweeps"], r["seed"], icm=r["icm"])
        S, E = spv.spv_top_sample(ctx, out)
    if r["fix"]:
        out["fix"] = spv.spv_persist_fix(ctx, P, S, E, *r["fix"])
    torch.cuda.synchronize()
    return out


def _submit(srv, r, P):
    kw = {} if not r["fix"] else dict(elite_frac=r["fix"][0], threshold=r["fix"][1], gauge=r["fix"][2])
    if r["kind"] == "sa":
        return srv.submit_sa(P, r["betas"], r["reads"], r["seed"], **kw)
    if r["kind"] == "sqa":
        return srv.submit_sqa(P, r["betas"], r["gammas"], r["trotter"], r["reads"], r["seed"], **kw)
    return srv.submit_pt(P, r["betas"], r["runs"], r["chains"], r["sweeps"], r["seed"], icm=r["icm"], **kw)


def _same(a, b):
    return np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def _check_against_alone(r, got, want):
    if r["kind"] in ("sa", "sqa"):
        assert _same(got["spins"], want["spins"]) and _same(got["energies"], want["energies"])
    else:
        for key in ("final_spins", "final_E", "top_spins", "top_E", "top_count"):
            assert _same(got[key], want[key]), key
    if r["fix"]:
        wf = want["fix"]
        gf = got["fix"]
        assert np.array_equal(gf["info"][:7].cpu().numpy(),
                              np.array([wf.info()[k] for k in ("n_free", "nnz_free", "offset", "n_fixed",
                                                                 "pivot", "m", "k_min")]))
        n = r["inst"].n
        assert _same(gf["fixed_mask"][:n], wf.fixed_mask) and _same(gf["fixed_val"][:n], wf.fixed_val)
        nf = wf.info()["n_free"]
        assert _same(gf["orig_index"][:nf], wf.orig_index)
        nz = wf.info()["nnz_free"]
        red = wf.reduced()
        assert _same(gf["row_ptr"][:nf + 1], red.row_ptr) and _same(gf["J"][:nz], red.J[:nz])
        assert _same(gf["h"][:nf], red.h[:nf]) and _same(gf["col"][:nz], red.col[:nz])


def test_mixed_stream_matches_alone_and_oracle(spv, ctx):
    reqs = _mix()
    Ps = [spv.Problem.from_instance(r["inst"]) for r in reqs]
    print(f"[serving] {len(reqs)} requests, alone", flush=True)
    alone = [_alone(spv, ctx, r, P) for r, P in zip(reqs, Ps)]
    print("[serving] mixed on 4 slots", flush=True)
    srv = spv.Server(ctx, slots=4)
    tickets = [_submit(srv, r, P) for r, P in zip(reqs, Ps)]
    results = [srv.wait(t) for t in tickets]
    srv.drain()
    slots_used = set()
    for r, (res, keep), want in zip(reqs, results, alone):
        assert res.status == 0 and res.submit_ns <= res.start_ns <= res.done_ns
        slots_used.add(res.slot)
        _check_against_alone(r, keep, want)
    assert len(slots_used) > 1
    srv.close()
    # oracle: the first SA request with persistence and the first PT request with persistence
    r0, (_, k0) = reqs[0], results[0]
    osp, oE = oracle.sa_sample(r0["inst"], r0["betas"], reads=r0["reads"], seed=r0["seed"], threads=8)
    assert np.array_equal(k0["spins"].cpu().numpy(), osp) and np.array_equal(k0["energies"].cpu().numpy(), oE)
    w = oracle.persist_fix(r0["inst"], osp, oE, *r0["fix"])
    assert np.array_equal(k0["fix"]["fixed_val"][:r0["inst"].n].cpu().numpy(), w["fixed_val"])
    assert int(k0["fix"]["info"][2]) == w["offset"]
    ip = next(i for i, r in enumerate(reqs) if r["kind"] == "pt" and r["fix"])
    r1, (_, k1) = reqs[ip], results[ip]
    want = oracle.pt_sample(r1["inst"], r1["betas"], r1["runs"], r1["chains"], r1["sweeps"], seed=r1["seed"],
                            icm=r1["icm"], threads=4)
    assert np.array_equal(k1["top_E"].cpu().numpy(), want["top_E"])
    S, E = oracle.top_sample(want)
    w = oracle.persist_fix(r1["inst"], S, E, *r1["fix"])
    assert np.array_equal(k1["fix"]["fixed_mask"][:r1["inst"].n].cpu().numpy(), w["fixed_mask"])
    assert np.array_equal(k1["fix"]["fixed_val"][:r1["inst"].n].cpu().numpy(), w["fixed_val"])
    assert int(k1["fix"]["info"][2]) == w["offset"] and int(k1["fix"]["info"][5]) == w["m"]


def test_budget_admits_one_at_a_time_in_fifo_order(spv, ctx):
    reqs = [r for r in _mix() if r["kind"] == "sa"][:5]
    Ps = [spv.Problem.from_instance(r["inst"]) for r in reqs]
    alone = [_alone(spv, ctx, r, P) for r, P in zip(reqs, Ps)]
    srv = spv.Server(ctx, slots=4, lds_budget=1)
    with pytest.raises(spv.SpvError, match="EBUDGET"):
        _submit(srv, reqs[0], Ps[0])
    srv.close()
    # learn the footprints, then serve under a budget that holds the largest request alone
    srv = spv.Server(ctx, slots=4)
    lds = [srv.wait(_submit(srv, r, P))[0].lds_bytes for r, P in zip(reqs, Ps)]
    srv.close()
    budget = max(lds)
    srv = spv.Server(ctx, slots=4, lds_budget=budget)
    tickets = [_submit(srv, r, P) for r, P in zip(reqs, Ps)]
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for r, (res, keep), want in zip(reqs, results, alone):
        _check_against_alone(r, keep, want)
    starts = [res.start_ns for res, _ in results]
    assert starts == sorted(starts)
    for res, _ in results:
        inflight = sum(o.lds_bytes for o, _ in results if o.start_ns <= res.start_ns < o.done_ns)
        assert inflight <= budget


def test_mixed_stream_with_split_tempering(spv, ctx):
    """Requests on the split tempering paths (N=1000 with the instance in LDS, N=8000
    PT-ICM with it in global memory) in flight together with SA requests: each
    result equals the same calls made alone."""
    from spvar_inputs import configs as cf
    c3, c5 = cf.CUBIC10_PT, cf.CUBIC20_PTICM
    i3, i5 = cf.instance(c3), cf.instance(c5)
    b3, b5 = cf.betas(c3), cf.betas(c5)
    reqs = [
        dict(kind="pt", inst=i5, betas=b5, runs=1, chains=2, sweeps=30, seed=11, icm=(0, b5.size),
             fix=(0.2, 1.0, 2)),
        dict(kind="sa", inst=si.chimera(4, seed=12), betas=si.linear_betas(0.1, 3.0, 200), reads=400, seed=13,
             fix=(0.1, 0.95, 0)),
        dict(kind="pt", inst=i3, betas=b3, runs=4, chains=1, sweeps=120, seed=14, icm=None, fix=(0.2, 1.0, 2)),
        dict(kind="sa", inst=si.chimera(3, seed=15), betas=si.linear_betas(0.1, 3.0, 300), reads=256, seed=16,
             fix=None),
        dict(kind="pt", inst=i3, betas=b3, runs=2, chains=1, sweeps=90, seed=17, icm=None, fix=None),
    ]
    Ps = [spv.Problem.from_instance(r["inst"]) for r in reqs]
    print(f"[serving] split tempering mix, {len(reqs)} requests", flush=True)
    alone = [_alone(spv, ctx, r, P) for r, P in zip(reqs, Ps)]
    srv = spv.Server(ctx, slots=4)
    tickets = [_submit(srv, r, P) for r, P in zip(reqs, Ps)]
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for r, (res, keep), want in zip(reqs, results, alone):
        assert res.status == 0
        _check_against_alone(r, keep, want)


def test_top_sample_matches_oracle_formation(spv, ctx):
    inst = si.cubic_lattice(4, "gauss", seed=31, scale_log2=10)
    P = spv.Problem.from_instance(inst)
    betas = si.geometric_betas(0.2, 5.0, 7)
    got = spv.spv_pt_sample(ctx, P, betas, 3, 2, 40, seed=9, icm=(0, 7))
    S, E = spv.spv_top_sample(ctx, got)
    want = oracle.pt_sample(inst, betas, 3, 2, 40, seed=9, icm=(0, 7), threads=3)
    wS, wE = oracle.top_sample(want)
    assert np.array_equal(S.cpu().numpy(), wS) and np.array_equal(E.cpu().numpy(), wE)


def test_mixed_stream_with_sqa_requests(spv, ctx):
    """SQA requests (with and without persistence) served among SA and PT requests: every
    result equals the same call made alone; one SQA request is recomputed by the oracle."""
    reqs = []
    for k in range(4):
        sw = 25 + 10 * k
        reqs.append(dict(kind="sqa", inst=si.chimera(2 + k % 2, seed=300 + k), betas=si.linear_betas(0.2, 3.0, sw),
                         gammas=np.geomspace(3.0, 0.05, sw), trotter=8 * (1 + k % 2), reads=9 + 7 * k, seed=900 + k,
                         fix=(0.25, 0.9, 0) if k % 2 == 0 else None))
    reqs += _mix()[:4] + _mix()[10:12]
    Ps = [spv.Problem.from_instance(r["inst"]) for r in reqs]
    print(f"[serving] {len(reqs)} requests with SQA, alone", flush=True)
    alone = [_alone(spv, ctx, r, P) for r, P in zip(reqs, Ps)]
    print("[serving] mixed with SQA on 3 slots", flush=True)
    srv = spv.Server(ctx, slots=3)
    tickets = [_submit(srv, r, P) for r, P in zip(reqs, Ps)]
    results = [srv.wait(t) for t in tickets]
    srv.drain()
    for r, (res, keep), want in zip(reqs, results, alone):
        assert res.status == 0
        _check_against_alone(r, keep, want)
    srv.close()
    r0, (_, k0) = reqs[0], results[0]
    osp, oE, _ = oracle.sqa_sample(r0["inst"], r0["betas"], r0["gammas"], r0["trotter"], reads=r0["reads"],
                                   seed=r0["seed"], threads=8)
    assert np.array_equal(k0["spins"].cpu().numpy(), osp) and np.array_equal(k0["energies"].cpu().numpy(), oE)
    w = oracle.persist_fix(r0["inst"], osp, oE, *r0["fix"])
    assert np.array_equal(k0["fix"]["fixed_val"][:r0["inst"].n].cpu().numpy(), w["fixed_val"])
    assert int(k0["fix"]["info"][2]) == w["offset"]
