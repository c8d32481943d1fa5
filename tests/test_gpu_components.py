"""GPU parity of the connected-component split and the sorted-merge recombination
(Sec. II.C) through the C ABI, bit for bit against the oracle: component labels,
merged rows, merged energies and each component's sorted partial energies."""
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


def _check(spv, ctx, inst, S):
    import torch
    P = spv.Problem.from_instance(inst)
    comp, nc = spv.spv_components(ctx, P)
    wcomp, wnc = oracle.components(inst)
    assert nc == wnc and np.array_equal(comp.cpu().numpy(), wcomp)
    merged, mE, pe = spv.spv_merge_components(ctx, P, comp, nc, torch.as_tensor(S).cuda(), part=True)
    wm, wE, wpe = oracle.merge_sorted(inst, wcomp, wnc, S)
    assert np.array_equal(merged.cpu().numpy(), wm)
    assert np.array_equal(mE.cpu().numpy(), wE)
    assert np.array_equal(pe.cpu().numpy(), wpe)
    return nc


CASES = [
    ("union4_shuffled", lambda: si.disjoint_union([si.chimera(2, seed=1), si.random_sparse(40, 2.5, seed=2),
                                                    si.chimera(1, seed=3), si.random_sparse(9, 1.0, seed=4)],
                                                   perm_seed=5), 301),
    ("connected_chimera3", lambda: si.chimera(3, seed=6), 97),
    ("sparse_many_components", lambda: si.random_sparse(700, 0.9, seed=7), 1029),
    ("isolated_only", lambda: si.disjoint_union([si.weak_strong_toy(-50)] * 3), 64),
    ("one_row", lambda: si.disjoint_union([si.chimera(1, seed=8), si.chimera(1, seed=9)], perm_seed=1), 1),
    ("cubic_gauss_two_blocks", lambda: si.disjoint_union([si.cubic_lattice(4, "gauss", seed=10, scale_log2=10),
                                                          si.cubic_lattice(3, "gauss", seed=11, scale_log2=10)],
                                                         perm_seed=2), 500),
]


@pytest.mark.parametrize("name,make,R", CASES, ids=[c[0] for c in CASES])
def test_components_and_merge_match_oracle(spv, ctx, name, make, R):
    inst = make()
    S = si.random_spins(R, inst.n, seed=R)
    print(f"[components] {name} n={inst.n} R={R}", flush=True)
    _check(spv, ctx, inst, S)


def test_merge_on_a_residual_after_fixing(spv, ctx):
    """The situation of Sec. II.C: SA on the Chimera N=512 workload, persistence, then a
    sample of the (disconnected) residual recombined per component."""
    import torch
    cfg = cf.CHIMERA8_SA
    inst = cf.instance(cfg)
    P = spv.Problem.from_instance(inst)
    betas = si.linear_betas(0.1, 5.0, 300)
    S, E = spv.spv_sample(ctx, P, betas, 2000, seed=3)
    fx = spv.spv_persist_fix(ctx, P, S, E, 0.05, 0.95, 0)
    red = fx.reduced()
    h = red.to_host()
    rinst = si.Instance(n=h["n"], row_ptr=h["row_ptr"], col=h["col"], J=h["J"], h=h["h"], colour=h["colour"],
                        n_colours=h["n_colours"], scale_log2=h["scale_log2"])
    Rs, Re = spv.spv_sample(ctx, red, betas, 3000, seed=4)
    nc = _check(spv, ctx, rinst, Rs.cpu().numpy())
    assert nc >= 1
    print(f"[components] residual n={rinst.n} components={nc}", flush=True)
