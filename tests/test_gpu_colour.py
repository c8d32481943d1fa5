"""GPU parity of the colour classes (Jones-Plassmann rounds with Philox priorities) through
the C ABI: the device colouring equals the oracle's byte for byte, and a problem coloured on
the device samples bit-identically to the oracle sampling it with the same classes."""
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


def _complete(n):
    a, b = np.triu_indices(n, 1)
    return si.from_edges(n, a, b, np.ones(a.size, np.int64), np.zeros(n), np.zeros(n), 1)


CASES = [
    ("sparse200", lambda: si.random_sparse(200, 4.0, seed=1), 0),
    ("chimera8", lambda: si.chimera(8, seed=2), 7),
    ("cubic10", lambda: si.cubic_lattice(10, "gauss", seed=3, scale_log2=10), 2**40 + 9),
    ("cubic20", lambda: si.cubic_lattice(20, "gauss", seed=4, scale_log2=10), 5),
    ("sparse20000", lambda: si.random_sparse(20000, 5.0, seed=5), 11),
    ("sparse_dense", lambda: si.random_sparse(300, 12.0, seed=6), 3),
    ("complete12", lambda: _complete(12), 4),
    ("edgeless", lambda: si.from_edges(100, [], [], [], np.zeros(100), np.zeros(100), 1), 1),
    ("single", lambda: si.from_edges(1, [], [], [], np.zeros(1), np.zeros(1), 1), 1),
]


@pytest.mark.parametrize("name,make,seed", CASES, ids=[c[0] for c in CASES])
def test_colour_matches_oracle(spv, ctx, name, make, seed):
    inst = make()
    P = spv.Problem.from_instance(inst)
    colour, nc = spv.spv_colour(ctx, P, seed)
    want, wnc = oracle.colour_jp(inst, seed)
    assert nc == wnc
    assert np.array_equal(colour.cpu().numpy(), want)


def test_colour_past_the_cap_is_an_error(spv, ctx):
    P = spv.Problem.from_instance(_complete(20))
    with pytest.raises(spv.SpvError):
        spv.spv_colour(ctx, P, 3)


def test_device_coloured_problem_samples_like_the_oracle(spv, ctx):
    """Colour a random graph on the device, then sample it with those classes: the SA
    sample equals the oracle's on the same classes."""
    base = si.random_sparse(150, 3.5, seed=8)
    P0 = spv.Problem.from_instance(base)
    colour, nc = spv.spv_colour(ctx, P0, 21)
    a, b, w = base.edges()
    inst = si.from_edges(base.n, a, b, w, base.h, colour.cpu().numpy(), nc)
    P = spv.Problem.from_instance(inst)
    spv.spv_problem_check(ctx, P)
    betas = si.linear_betas(0.1, 3.0, 60)
    S, E = spv.spv_sample(ctx, P, betas, 40, 99)
    osp, oE = oracle.sa_sample(inst, betas, reads=40, seed=99)
    assert np.array_equal(S.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)
