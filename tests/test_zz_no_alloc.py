"""The allocation-free persistence entry point (spv_persist_fix_noalloc, scratch in the library's
static device array) through the C ABI: bit-identical to spv_persist_fix on two calls in a row,
the second with a smaller input (the array keeps the first call's contents), with and without the
zero-bias gauge; and a call needing more scratch than the array holds is refused before any
launch."""
import numpy as np
import pytest

import oracle
import spvar_inputs as si

pytestmark = pytest.mark.gpu

ECAPACITY = -5


@pytest.fixture(scope="module")
def spv():
    import paper_1706_07826_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(spv):
    return spv.Context(0)


def _outputs(fx):
    i = fx.info()
    k = fx._keep
    nf, nz = i["n_free"], i["nnz_free"]
    return dict(info=i, fixed_mask=fx.fixed_mask.cpu().numpy(), fixed_val=fx.fixed_val.cpu().numpy(),
                row_ptr=k["row_ptr"][:nf + 1].cpu().numpy(), col=k["col"][:nz].cpu().numpy(),
                J=k["J"][:nz].cpu().numpy(), h=k["h"][:nf].cpu().numpy(), colour=k["colour"][:nf].cpu().numpy(),
                orig_index=k["orig_index"][:nf].cpu().numpy())


def _same(a, b):
    assert a["info"] == b["info"]
    for key in ("fixed_mask", "fixed_val", "row_ptr", "col", "J", "h", "colour", "orig_index"):
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("gauge", [0, 2])
def test_noalloc_matches_persist_fix_on_two_calls(spv, ctx, gauge):
    big = si.chimera(8, seed=51, h_zero=gauge == 2)        # N = 512
    small = si.cubic_lattice(4, "pm1", seed=52)             # N = 64, h = 0
    for k, (inst, reads, sweeps, elite, theta) in enumerate(((big, 2000, 200, 0.05, 0.95),
                                                             (small, 300, 100, 0.1, 1.0))):
        print(f"[noalloc] gauge={gauge} call {k}: n={inst.n} reads={reads}", flush=True)
        P = spv.Problem.from_instance(inst)
        S, E = spv.spv_sample(ctx, P, si.linear_betas(0.1, 3.0, sweeps), reads, 600 + k)
        want = _outputs(spv.spv_persist_fix(ctx, P, S, E, elite, theta, gauge))
        got = _outputs(spv.spv_persist_fix(ctx, P, S, E, elite, theta, gauge, noalloc=True))
        _same(got, want)
        ref = oracle.persist_fix(inst, S.cpu().numpy(), E.cpu().numpy(), elite, theta, gauge)
        assert got["info"]["offset"] == ref["offset"] and got["info"]["n_free"] == ref["n_free"]
        assert np.array_equal(got["fixed_val"], ref["fixed_val"])


def test_noalloc_refuses_scratch_beyond_its_array(spv, ctx):
    import torch
    inst = si.chimera(8, seed=53)
    P = spv.Problem.from_instance(inst)
    R = 300000  # elite 1.0: column bitmaps alone take 512 * ceil(R / 64) * 8 B = 19.2 MB > 16 MiB
    S = torch.ones((R, inst.n), dtype=torch.int8, device="cuda")
    E = torch.zeros(R, dtype=torch.int64, device="cuda")
    with pytest.raises(spv.SpvError) as e:
        spv.spv_persist_fix(ctx, P, S, E, 1.0, 1.0, 0, noalloc=True)
    assert e.value.code == ECAPACITY
    # the context stays usable: a call within the array's size (unanimous rows fix everything)
    fx = spv.spv_persist_fix(ctx, P, S[:1000], E[:1000], 1.0, 1.0, 0, noalloc=True)
    assert fx.info()["n_free"] == 0 and bool((fx.fixed_val == 1).all())
