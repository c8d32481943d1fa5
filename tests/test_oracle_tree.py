"""Pins of the oracle's tree / degree-1 pre-processing (Sec. II.C): trees are solved
exactly (the offset equals the brute-force ground energy and the completed state
reaches it), attached trees leave the minimum unchanged, every completion of a
reduced state satisfies E(s) = E'(s') + offset, a graph without leaves is
untouched, and a two-variable case worked by hand."""
import itertools

import numpy as np
import pytest

import oracle
import spvar_inputs as si


def _brute_min(inst):
    if inst.n == 0:
        return 0
    best = None
    for bits in itertools.product((-1, 1), repeat=inst.n):
        e = int(oracle.energy(inst, np.array(bits, np.int8)[None])[0])
        best = e if best is None or e < best else best
    return best


def _coloured(inst):
    colour, nc = si.greedy_colouring(inst)
    a, b, w = inst.edges()
    return si.from_edges(inst.n, a, b, w, inst.h, colour, nc)


def _random_tree(n, seed, j_max=6, h_max=6, h_zero_frac=0.3):
    rng = np.random.default_rng(seed)
    ei = np.array([rng.integers(0, i) for i in range(1, n)], np.int64)
    ej = np.arange(1, n, dtype=np.int64)
    w = rng.integers(1, j_max + 1, size=n - 1) * rng.choice([-1, 1], size=n - 1)
    h = rng.integers(-h_max, h_max + 1, size=n)
    h[rng.random(n) < h_zero_frac] = 0
    return _coloured(si.from_edges(n, ei, ej, w, h, np.zeros(n), 1))


def _tree_plus_cycle(n_cycle, n_tree, seed):
    """A cycle (the 2-core) with a random forest hanging off it."""
    rng = np.random.default_rng(seed)
    n = n_cycle + n_tree
    ei = list(range(n_cycle))
    ej = [(i + 1) % n_cycle for i in range(n_cycle)]
    for v in range(n_cycle, n):
        ei.append(int(rng.integers(0, v)))
        ej.append(v)
    m = len(ei)
    w = rng.integers(1, 7, size=m) * rng.choice([-1, 1], size=m)
    h = rng.integers(-6, 7, size=n)
    return _coloured(si.from_edges(n, np.array(ei), np.array(ej), w, h, np.zeros(n), 1))


@pytest.mark.parametrize("seed", range(8))
def test_trees_are_solved_exactly(seed):
    inst = _random_tree(13, seed)
    pe = oracle.tree_peel(inst)
    assert pe["n_free"] == 0 and pe["n_fixed"] + pe["n_inferred"] == inst.n
    ground = _brute_min(inst)
    assert pe["offset"] == ground
    s = oracle.tree_expand(inst, pe, np.zeros((1, 0), np.int8))
    assert int(oracle.energy(inst, s)[0]) == ground


@pytest.mark.parametrize("seed", range(6))
def test_attached_trees_keep_the_minimum(seed):
    inst = _tree_plus_cycle(5, 10, seed)
    pe = oracle.tree_peel(inst)
    assert pe["n_free"] == 5  # the cycle is the 2-core
    assert _brute_min(pe["reduced"]) + pe["offset"] == _brute_min(inst)


@pytest.mark.parametrize("seed", range(4))
def test_every_completion_matches_reduced_energy(seed):
    inst = si.random_sparse(300, 1.3, seed=seed)   # many trees and a small core
    pe = oracle.tree_peel(inst)
    R = 50
    rs = si.random_spins(R, pe["n_free"], seed=seed) if pe["n_free"] else np.zeros((R, 0), np.int8)
    full = oracle.tree_expand(inst, pe, rs)
    assert set(np.unique(full)).issubset({-1, 1})
    Ered = oracle.energy(pe["reduced"], rs) if pe["n_free"] else np.zeros(R, np.int64)
    assert np.array_equal(oracle.energy(inst, full), Ered + pe["offset"])
    # the remaining variables keep their couplers among themselves
    assert np.all(pe["kind"][pe["orig_index"]] == 0)


def test_graph_without_leaves_is_untouched():
    inst = si.cubic_lattice(4, "gauss", seed=3, scale_log2=10)
    pe = oracle.tree_peel(inst)
    assert pe["n_free"] == inst.n and pe["offset"] == 0 and pe["rounds"] == 0
    r = pe["reduced"]
    assert np.array_equal(r.row_ptr, inst.row_ptr) and np.array_equal(r.J, inst.J) and np.array_equal(r.h, inst.h)


def test_two_variables_by_hand():
    """J = -3, h = (1, -1): round 0 peels variable 1 (the larger index of the pair) as
    inferred, s1 = +s0, folding -sign(J) h1 = -1 into h0 (now 0) and -|J| into the
    offset; round 1 fixes variable 0 to +1 (h0 = 0).  Offset -3 = the ground energy."""
    inst = si.from_edges(2, [0], [1], [-3], [1, -1], [0, 1], 2)
    pe = oracle.tree_peel(inst)
    assert list(pe["kind"]) == [1, 2] and list(pe["round"]) == [1, 0] and pe["parent"][1] == 0
    assert list(pe["value"]) == [1, 1] and pe["offset"] == -3 and pe["rounds"] == 2
    s = oracle.tree_expand(inst, pe, np.zeros((1, 0), np.int8))
    assert list(s[0]) == [1, 1] and int(oracle.energy(inst, s)[0]) == -3 == _brute_min(inst)
