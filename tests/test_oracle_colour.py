"""Pins of the oracle's colour classes (Jones-Plassmann rounds with Philox priorities):
every class is an independent set, the result equals first-fit greedy colouring in
decreasing priority order (a different, sequential algorithm with the same unique
result), a complete graph gets its colours in priority order, an edgeless graph one
colour, and the colour count stays within max degree + 1 (ERANGE past the cap)."""
import numpy as np
import pytest

import oracle
import spvar_inputs as si


def _priorities(n, seed):
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n, dtype=np.uint32)
    ctr[:, 3] = 5 << 24
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32)
    return oracle.philox_batch(ctr, key)[:, 0].astype(np.int64)


def _greedy_by_priority(inst, seed):
    pr = _priorities(inst.n, seed)
    order = sorted(range(inst.n), key=lambda v: (pr[v], v), reverse=True)
    col = -np.ones(inst.n, np.int64)
    for v in order:
        taken = {int(col[j]) for j in inst.col[inst.row_ptr[v]:inst.row_ptr[v + 1]] if col[j] >= 0}
        c = 0
        while c in taken:
            c += 1
        col[v] = c
    return col


def _proper(inst, colour):
    rows = np.repeat(np.arange(inst.n), np.diff(inst.row_ptr))
    return bool(np.all(colour[rows] != colour[inst.col]))


def _complete(n):
    a, b = np.triu_indices(n, 1)
    return si.from_edges(n, a, b, np.ones(a.size, np.int64), np.zeros(n), np.zeros(n), 1)


GRAPHS = [
    ("sparse200", lambda: si.random_sparse(200, 4.0, seed=1)),
    ("chimera4", lambda: si.chimera(4, seed=2)),
    ("cubic5", lambda: si.cubic_lattice(5, "pm1", seed=3)),
    ("residual", lambda: si.residual_batch(1, parent_M=6, n_min=80, n_max=120, seed=4)[0]),
    ("sparse_dense", lambda: si.random_sparse(60, 9.0, seed=5)),
]


@pytest.mark.parametrize("name,make", GRAPHS, ids=[g[0] for g in GRAPHS])
@pytest.mark.parametrize("seed", [0, 77, 2**40 + 3])
def test_jp_equals_greedy_in_priority_order(name, make, seed):
    inst = make()
    colour, nc = oracle.colour_jp(inst, seed)
    assert _proper(inst, colour)
    assert np.array_equal(colour.astype(np.int64), _greedy_by_priority(inst, seed))
    assert nc == int(colour.max()) + 1
    assert nc <= int(np.diff(inst.row_ptr).max()) + 1


def test_complete_graph_colours_in_priority_order():
    inst = _complete(9)
    colour, nc = oracle.colour_jp(inst, 5)
    pr = _priorities(9, 5)
    order = sorted(range(9), key=lambda v: (pr[v], v), reverse=True)
    assert nc == 9 and [int(colour[v]) for v in order] == list(range(9))


def test_edgeless_graph_one_colour():
    inst = si.from_edges(30, [], [], [], np.zeros(30), np.zeros(30), 1)
    colour, nc = oracle.colour_jp(inst, 1)
    assert nc == 1 and not colour.any()


def test_too_many_colours_is_an_error():
    with pytest.raises(oracle.OracleError):
        oracle.colour_jp(_complete(20), 3, max_colours=16)
