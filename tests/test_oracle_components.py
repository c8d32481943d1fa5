"""Pins of the oracle's connected-component split and sorted-merge recombination
(Sec. II.C, special considerations) against what the definition fixes: the
component partition of a library graph routine, partial energies that add up to
the full energy recomputed independently, the best merged row equal to the sum
of the per-component minima, and the single-component case reducing to a
stable sort of the sample by energy."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle
import spvar_inputs as si


def _with_zero_couplers(inst, frac, seed):
    """The same graph with some couplers set to 0 (they no longer connect)."""
    rng = np.random.default_rng(seed)
    a, b, w = inst.edges()
    w = np.where(rng.random(w.size) < frac, 0, w)
    return si.from_edges(inst.n, a, b, w, inst.h, inst.colour, inst.n_colours, inst.scale_log2)


def _scipy_labels(inst):
    a, b, w = inst.edges()
    keep = w != 0
    g = sp.coo_matrix((np.ones(int(keep.sum())), (a[keep], b[keep])), shape=(inst.n, inst.n))
    return connected_components(g, directed=False)


def _canonical(labels):
    """Relabel components in order of their smallest member."""
    first = {}
    out = np.empty_like(labels)
    for i, l in enumerate(labels):
        if l not in first:
            first[l] = len(first)
        out[i] = first[l]
    return out


@pytest.mark.parametrize("seed", range(6))
def test_components_match_library_partition(seed):
    base = si.random_sparse(120, 1.6, seed=seed)
    inst = _with_zero_couplers(base, 0.3, seed)
    comp, nc = oracle.components(inst)
    n_ref, lab = _scipy_labels(inst)
    assert nc == n_ref
    assert np.array_equal(comp, _canonical(lab))
    # numbering: component c's smallest member precedes component c+1's
    firsts = [int(np.flatnonzero(comp == c)[0]) for c in range(nc)]
    assert firsts == sorted(firsts)


def test_components_of_a_union_with_isolated_variables():
    parts = [si.chimera(1, seed=1), si.cubic_lattice(3, "pm1", seed=2), si.weak_strong_toy(-0.5 * 100)]
    inst = si.disjoint_union(parts, perm_seed=7)
    comp, nc = oracle.components(inst)
    assert nc == 3
    sizes = sorted(np.bincount(comp).tolist())
    assert sizes == sorted(p.n for p in parts)


def _partial_energies(inst, comp, nc, S):
    """Independent numpy evaluation of E_c(r) = sum of couplers inside c + biases in c."""
    a, b, w = inst.edges()
    S = S.astype(np.int64)
    pe = np.zeros((S.shape[0], nc), np.int64)
    for c in range(nc):
        inside = comp[a] == c
        pe[:, c] = (S[:, a[inside]] * S[:, b[inside]] * w[inside]).sum(axis=1)
        vs = np.flatnonzero(comp == c)
        pe[:, c] += (S[:, vs] * inst.h[vs].astype(np.int64)).sum(axis=1)
    return pe


@pytest.mark.parametrize("seed", range(4))
def test_merge_sorted_properties(seed):
    parts = [si.chimera(2, seed=10 + seed), si.random_sparse(40, 2.5, seed=20 + seed),
             si.chimera(1, seed=30 + seed), si.random_sparse(9, 1.0, seed=40 + seed)]
    inst = si.disjoint_union(parts, perm_seed=seed)
    comp, nc = oracle.components(inst)
    S = si.random_spins(57, inst.n, seed=seed)
    merged, mE, part = oracle.merge_sorted(inst, comp, nc, S)
    pe = _partial_energies(inst, comp, nc, S)
    # partial energies add up to the full energy
    assert np.array_equal(pe.sum(axis=1), oracle.energy(inst, S))
    # each component's column of partial energies, sorted
    for c in range(nc):
        assert np.array_equal(part[c], np.sort(pe[:, c], kind="stable"))
    # merged energies are the sums of the k-th partial energies, recompute from spins
    assert np.array_equal(mE, part.sum(axis=0))
    assert np.array_equal(mE, oracle.energy(inst, merged))
    assert np.all(np.diff(mE) >= 0)
    # the best merged row holds every component's best partial solution
    assert mE[0] == pe.min(axis=0).sum()
    # every component block of a merged row is that component's block of some sample row
    for c in range(nc):
        vs = np.flatnonzero(comp == c)
        order = np.argsort(pe[:, c], kind="stable")
        assert np.array_equal(merged[:, vs], S[order][:, vs])


def test_single_component_reduces_to_stable_sort():
    inst = si.chimera(3, seed=5)
    comp, nc = oracle.components(inst)
    assert nc == 1 and not comp.any()
    S = si.random_spins(40, inst.n, seed=3)
    S[7] = S[3]  # a tie: the lower row comes first
    E = oracle.energy(inst, S)
    merged, mE, _ = oracle.merge_sorted(inst, comp, nc, S)
    order = np.argsort(E, kind="stable")
    assert np.array_equal(merged, S[order]) and np.array_equal(mE, E[order])


def test_two_blocks_solved_in_different_rows_merge_to_the_ground_state():
    """The motivating case: row 0 solves block A only, row 1 block B only; the best
    merged row is a ground state of the whole problem (brute force on each block)."""
    import itertools
    A, B = si.random_sparse(8, 2.0, seed=1), si.random_sparse(7, 2.0, seed=2)
    inst = si.disjoint_union([A, B])

    def ground(p):
        best = None
        for bits in itertools.product((-1, 1), repeat=p.n):
            s = np.array(bits, np.int8)
            e = int(oracle.energy(p, s[None])[0])
            if best is None or e < best[0]:
                best = (e, s)
        return best

    (ea, sa), (eb, sb) = ground(A), ground(B)
    bad_a, bad_b = -sa, -sb
    if oracle.energy(A, bad_a[None])[0] == ea:
        bad_a = np.ones(A.n, np.int8)
    S = np.stack([np.concatenate([sa, bad_b]), np.concatenate([bad_a, sb])])
    comp, nc = oracle.components(inst)
    merged, mE, _ = oracle.merge_sorted(inst, comp, nc, S)
    assert mE[0] == ea + eb
    assert np.array_equal(merged[0], np.concatenate([sa, sb]))
