"""GPU parity of the tree / degree-1 pre-processing (Sec. II.C) through the C ABI, bit for
bit against the oracle: per-variable kind, value, parent and round, the reduced problem
(CSR, biases, colours, index map), the offset and counts, a removal order consistent with
the rounds, and the completion of reduced states."""
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


def _coloured(inst):
    colour, nc = si.greedy_colouring(inst)
    a, b, w = inst.edges()
    return si.from_edges(inst.n, a, b, w, inst.h, colour, nc)


def _random_tree(n, seed):
    rng = np.random.default_rng(seed)
    ei = np.array([rng.integers(0, i) for i in range(1, n)], np.int64)
    ej = np.arange(1, n, dtype=np.int64)
    w = rng.integers(1, 7, size=n - 1) * rng.choice([-1, 1], size=n - 1)
    h = rng.integers(-6, 7, size=n)
    h[rng.random(n) < 0.3] = 0
    return _coloured(si.from_edges(n, ei, ej, w, h, np.zeros(n), 1))


def _path(n, seed):
    """A chain: about n / 2 rounds, one removal from each end per round."""
    rng = np.random.default_rng(seed)
    w = rng.integers(1, 7, size=n - 1) * rng.choice([-1, 1], size=n - 1)
    h = rng.integers(-3, 4, size=n)
    return _coloured(si.from_edges(n, np.arange(n - 1), np.arange(1, n), w, h, np.zeros(n), 1))


def _with_zero_couplers(inst, seed, frac=0.2):
    """The same graph with a fraction of its couplers stored as explicit zeros."""
    a, b, w = inst.edges()
    rng = np.random.default_rng(seed)
    w = w.copy()
    w[rng.random(w.size) < frac] = 0
    return si.from_edges(inst.n, a, b, w, inst.h, inst.colour, inst.n_colours, inst.scale_log2)


def _pendants(M, per_site, seed):
    """A Chimera graph with random trees hanging off a fraction of its sites."""
    base = si.chimera(M, seed=seed)
    rng = np.random.default_rng(seed + 1)
    a, b, w = base.edges()
    ei, ej, ww = list(a), list(b), list(w)
    n = base.n
    h = list(base.h)
    for v in range(base.n):
        if rng.random() < per_site:
            for _ in range(int(rng.integers(1, 4))):
                par = v if rng.random() < 0.5 or n == base.n else int(rng.integers(base.n, n))
                ei.append(par)
                ej.append(n)
                ww.append(int(rng.integers(1, 7)) * int(rng.choice([-1, 1])))
                h.append(int(rng.integers(-6, 7)))
                n += 1
    return _coloured(si.from_edges(n, np.array(ei), np.array(ej), np.array(ww), np.array(h), np.zeros(n), 1))


CASES = [
    ("tree13", lambda: _random_tree(13, 1)),
    ("tree5000", lambda: _random_tree(5000, 2)),
    ("path3001", lambda: _path(3001, 3)),
    ("pair_by_hand", lambda: si.from_edges(2, [0], [1], [-3], [1, -1], [0, 1], 2)),
    ("sparse300", lambda: si.random_sparse(300, 1.3, seed=4)),
    ("sparse20000", lambda: si.random_sparse(20000, 1.5, seed=5)),
    ("sparse_zero_J", lambda: _with_zero_couplers(si.random_sparse(2000, 2.5, seed=6), 7)),
    ("chimera_pendants", lambda: _pendants(8, 0.3, 8)),
    ("chimera_no_leaves", lambda: si.chimera(4, seed=9)),
    ("cubic_no_leaves", lambda: si.cubic_lattice(6, "gauss", seed=10, scale_log2=10)),
    ("isolated", lambda: si.from_edges(1500, [], [], [], np.random.default_rng(11).integers(-3, 4, 1500),
                                       np.zeros(1500), 1)),
]


def _check(spv, ctx, inst):
    P = spv.Problem.from_instance(inst)
    want = oracle.tree_peel(inst)
    got = spv.spv_tree_reduce(ctx, P)
    info = got.info()
    for key in ("n_free", "nnz_free", "offset", "n_fixed", "n_inferred", "rounds"):
        assert info[key] == want[key], key
    assert info["n_removed"] == inst.n - want["n_free"]
    for key in ("kind", "value", "parent", "round"):
        assert np.array_equal(getattr(got, key).cpu().numpy(), want[key]), key
    # the removal order: every removed variable once, rounds non-decreasing
    order = got.order.cpu().numpy()
    removed = np.flatnonzero(want["kind"] != 0)
    assert np.array_equal(np.sort(order), removed)
    assert np.all(np.diff(want["round"][order]) >= 0)
    red, wr = got.reduced().to_host(), want["reduced"]
    assert np.array_equal(red["row_ptr"], wr.row_ptr)
    for key in ("col", "J", "h", "colour"):
        assert np.array_equal(red[key], getattr(wr, key)), key
    assert np.array_equal(got.orig_index.cpu().numpy(), want["orig_index"])
    return P, got, want


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_tree_reduce_matches_oracle(spv, ctx, name, make):
    _check(spv, ctx, make())


@pytest.mark.parametrize("name,make", [CASES[i] for i in (1, 4, 5, 6, 7)], ids=[CASES[i][0] for i in (1, 4, 5, 6, 7)])
def test_tree_complete_matches_oracle(spv, ctx, name, make):
    import torch

    inst = make()
    P, got, want = _check(spv, ctx, inst)
    R, nf = 300, want["n_free"]
    rs = si.random_spins(R, nf, seed=12) if nf else np.zeros((R, 0), np.int8)
    full = spv.spv_tree_complete(ctx, got, torch.as_tensor(rs).to(ctx.device))
    expect = oracle.tree_expand(inst, want, rs)
    assert np.array_equal(full.cpu().numpy(), expect)
    # E(s) = E'(s') + offset on the device
    E = spv.spv_energy(ctx, P, full).cpu().numpy()
    Ered = spv.spv_energy(ctx, got.reduced(), torch.as_tensor(rs).to(ctx.device)).cpu().numpy() if nf else \
        np.zeros(R, np.int64)
    assert np.array_equal(E, Ered + want["offset"])


def test_tree_repeated_calls_reuse_scratch(spv, ctx):
    """A large call, then a small one on the same context: the scratch is re-initialised."""
    _check(spv, ctx, si.random_sparse(30000, 1.4, seed=13))
    _check(spv, ctx, _random_tree(40, 14))


def test_tree_empty_problem(spv, ctx):
    import torch

    inst = si.from_edges(0, [], [], [], [], [], 1)
    P = spv.Problem.from_instance(inst)
    got = spv.spv_tree_reduce(ctx, P)
    assert got.info() == dict(n_free=0, nnz_free=0, offset=0, n_fixed=0, n_inferred=0, rounds=0, n_removed=0)
    full = spv.spv_tree_complete(ctx, got, torch.zeros((4, 0), dtype=torch.int8, device=ctx.device))
    assert tuple(full.shape) == (4, 0)


def test_tree_complete_rejects_bad_sizes(spv, ctx):
    import paper_1706_07826_amd as m

    inst = _random_tree(20, 15)
    P = spv.Problem.from_instance(inst)
    got = spv.spv_tree_reduce(ctx, P)
    got.info()
    rc = m._lib.spv_tree_complete(ctx.handle, inst.n, m.C.byref(got.out), 5, 5, None, 1, None, None)
    assert rc == -1  # n_free + n_removed != n
