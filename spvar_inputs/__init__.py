"""Seeded synthetic inputs for the sample-persistence hot path.

This module only *builds inputs*: Ising instances in symmetric CSR form, their
graph colourings, inverse-temperature schedules and the workload descriptors.
It holds none of the method's arithmetic (no energies, acceptance tests,
random streams of the sampler, persistence or reduction), so both the CPU
oracle and the HIP library can consume its output without sharing code.

Problem statement followed (Sec. I): minimise s^T J s + h^T s over
s in {-1,+1}^N.  Couplers and biases are integers; the real value of an
integer quantity q is q / 2**scale_log2.

None of the paper's instance pools ship here; every instance is drawn from a
numpy PCG64 stream seeded by the caller.
"""
from __future__ import annotations

import dataclasses
import math
from collections import deque

import numpy as np

__all__ = [
    "Instance", "from_edges", "cubic_lattice", "chimera", "weak_strong_toy",
    "random_sparse", "greedy_colouring", "residual_batch", "linear_betas",
    "geometric_betas", "random_spins",
]


@dataclasses.dataclass
class Instance:
    """Symmetric CSR Ising instance plus a proper colouring of its graph.

    row_ptr[n+1], col[nnz] (sorted per row, no self loops, no duplicates),
    J[nnz] int32 (J(i,j) == J(j,i); each undirected coupler is stored twice
    and counted once in the objective), h[n] int32, colour[n] uint8 with no
    edge inside a colour class.
    """
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    J: np.ndarray
    h: np.ndarray
    colour: np.ndarray
    n_colours: int
    scale_log2: int = 0
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def edges(self):
        """Undirected edges (i<j) and their couplings, in CSR order."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        sel = rows < self.col
        return rows[sel], self.col[sel].astype(np.int64), self.J[sel].astype(np.int64)


def from_edges(n, ei, ej, w, h, colour, n_colours, scale_log2=0, name=""):
    """Build the symmetric CSR of an undirected edge list (i != j, no repeats)."""
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    w = np.asarray(w, dtype=np.int64)
    if np.any(ei == ej):
        raise ValueError("self loop in edge list")
    a = np.concatenate([ei, ej])
    b = np.concatenate([ej, ei])
    v = np.concatenate([w, w])
    order = np.lexsort((b, a))
    a, b, v = a[order], b[order], v[order]
    if a.size and np.any((a[1:] == a[:-1]) & (b[1:] == b[:-1])):
        raise ValueError("duplicate edge in edge list")
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(row_ptr, a + 1, 1)
    row_ptr = np.cumsum(row_ptr, dtype=np.int64).astype(np.int32)
    return Instance(
        n=int(n), row_ptr=row_ptr, col=b.astype(np.int32), J=v.astype(np.int32),
        h=np.asarray(h, dtype=np.int32).copy(), colour=np.asarray(colour, dtype=np.uint8).copy(),
        n_colours=int(n_colours), scale_log2=int(scale_log2), name=name)


def _round_half_away(x):
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def _draw_couplings(rng, m, dist, scale_log2):
    if dist == "pm1":
        return rng.choice(np.array([-1, 1], dtype=np.int64), size=m)
    if dist == "gauss":
        z = rng.standard_normal(m) * float(2 ** scale_log2)
        return np.clip(_round_half_away(z), -32767, 32767).astype(np.int64)
    if isinstance(dist, tuple) and dist[0] == "uniform_nonzero":
        k = int(dist[1])
        vals = np.concatenate([np.arange(-k, 0), np.arange(1, k + 1)]).astype(np.int64)
        return rng.choice(vals, size=m)
    raise ValueError(f"unknown coupling distribution {dist!r}")


def cubic_lattice(L, dist="pm1", seed=0, scale_log2=0, h_dist=None):
    """Periodic L x L x L cubic lattice, site i = x + L*(y + L*z).

    Couplers are drawn for the +x, +y, +z bond of every site in site order.
    Colouring: (x+y+z) & 1, a proper 2-colouring for even L; odd L falls back
    to greedy first-fit in index order.
    """
    if L < 3:
        raise ValueError("L >= 3 required (L=2 would duplicate periodic bonds)")
    rng = np.random.Generator(np.random.PCG64(seed))
    n = L ** 3
    idx = np.arange(n, dtype=np.int64)
    x, y, z = idx % L, (idx // L) % L, idx // (L * L)
    nbrs = [((x + 1) % L) + L * (y + L * z), x + L * (((y + 1) % L) + L * z),
            x + L * (y + L * ((z + 1) % L))]
    ei = np.repeat(idx, 3)
    ej = np.stack(nbrs, axis=1).reshape(-1)
    w = _draw_couplings(rng, ei.size, dist, scale_log2)
    if h_dist is None:
        h = np.zeros(n, dtype=np.int64)
    else:
        h = _draw_couplings(rng, n, h_dist, scale_log2)
    if L % 2 == 0:
        colour = ((x + y + z) & 1).astype(np.uint8)
        inst = from_edges(n, ei, ej, w, h, colour, 2, scale_log2, name=f"cubic{L}")
    else:
        inst = from_edges(n, ei, ej, w, h, np.zeros(n, np.uint8), 1, scale_log2, name=f"cubic{L}")
        inst.colour, inst.n_colours = greedy_colouring(inst)
    return inst


def chimera(M, j_max=6, h_max=6, seed=0, h_zero=False):
    """M x M Chimera graph of K4,4 unit cells (full yield).

    Site i = 8*(r*M + c) + u, shore = u >> 2.  Shore-0 sites couple to the
    same site of the cell below (r+1), shore-1 sites to the cell on the right
    (c+1).  Couplers and biases are uniform on {-k..-1, 1..k}.
    Colouring: shore xor ((r + c) & 1).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 8 * M * M
    ei, ej = [], []
    for cell in range(M * M):
        base = 8 * cell
        for a in range(4):
            for b in range(4):
                ei.append(base + a)
                ej.append(base + 4 + b)
    for r in range(M - 1):
        for c in range(M):
            for k in range(4):
                ei.append(8 * (r * M + c) + k)
                ej.append(8 * ((r + 1) * M + c) + k)
    for r in range(M):
        for c in range(M - 1):
            for k in range(4):
                ei.append(8 * (r * M + c) + 4 + k)
                ej.append(8 * (r * M + c + 1) + 4 + k)
    ei = np.array(ei, dtype=np.int64)
    ej = np.array(ej, dtype=np.int64)
    w = _draw_couplings(rng, ei.size, ("uniform_nonzero", j_max), 0)
    if h_zero:
        h = np.zeros(n, dtype=np.int64)
    else:
        h = _draw_couplings(rng, n, ("uniform_nonzero", h_max), 0)
    i = np.arange(n)
    cell = i // 8
    r, c, shore = cell // M, cell % M, (i % 8) >> 2
    colour = (shore ^ ((r + c) & 1)).astype(np.uint8)
    return from_edges(n, ei, ej, w, h, colour, 2, 0, name=f"chimera{M}")


def weak_strong_toy(h_weak, j=-100, h_strong=100):
    """Two horizontally adjacent Chimera cells: a 'strong' cluster (sites 0-7,
    bias h_strong) and a 'weak' one (sites 8-15, bias h_weak), every coupler
    ferromagnetic (j < 0): 16 intra-cell couplers per cell and the 4
    inter-cell couplers between the shore-1 sites (Sec. III.B setting, in
    integer units of 1/100)."""
    ei, ej = [], []
    for base in (0, 8):
        for a in range(4):
            for b in range(4):
                ei.append(base + a)
                ej.append(base + 4 + b)
    for k in range(4):
        ei.append(4 + k)
        ej.append(12 + k)
    w = np.full(len(ei), j, dtype=np.int64)
    h = np.array([h_strong] * 8 + [h_weak] * 8, dtype=np.int64)
    u = np.arange(16) % 8
    colour = ((u >> 2) ^ (np.arange(16) // 8)).astype(np.uint8)
    return from_edges(16, ei, ej, w, h, colour, 2, 0, name="weak_strong_toy")


def greedy_colouring(inst):
    """First-fit colouring in index order; returns (colour uint8[n], n_colours)."""
    colour = np.full(inst.n, -1, dtype=np.int64)
    for i in range(inst.n):
        used = set(int(colour[j]) for j in inst.col[inst.row_ptr[i]:inst.row_ptr[i + 1]] if colour[j] >= 0)
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    nc = int(colour.max()) + 1 if inst.n else 1
    if nc > 255:
        raise ValueError("too many colours")
    return colour.astype(np.uint8), nc


def random_sparse(n, avg_degree=3.0, j_max=6, h_max=6, seed=0, h_zero=False, scale_log2=0,
                  dist=None):
    """Erdos-Renyi style sparse instance with greedy colouring (test workloads)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m_target = int(round(avg_degree * n / 2))
    pairs = set()
    tries = 0
    while len(pairs) < m_target and tries < 50 * max(1, m_target):
        a, b = rng.integers(0, n, size=2)
        tries += 1
        if a == b:
            continue
        pairs.add((int(min(a, b)), int(max(a, b))))
    pairs = sorted(pairs)
    ei = np.array([p[0] for p in pairs], dtype=np.int64)
    ej = np.array([p[1] for p in pairs], dtype=np.int64)
    d = dist if dist is not None else ("uniform_nonzero", j_max)
    w = _draw_couplings(rng, ei.size, d, scale_log2)
    if h_zero:
        h = np.zeros(n, dtype=np.int64)
    else:
        h = _draw_couplings(rng, n, d if dist is not None else ("uniform_nonzero", h_max), scale_log2)
    inst = from_edges(n, ei, ej, w, h, np.zeros(n, np.uint8), 1, scale_log2, name=f"sparse{n}")
    inst.colour, inst.n_colours = greedy_colouring(inst)
    return inst


def residual_batch(B, parent_M=16, n_min=50, n_max=1000, seed=0, j_max=6, h_max=6):
    """Residual-shaped instances of uneven size (stand-in for the subproblems
    left after fixing, Sec. II.C and Sec. III.C).

    Parent: an M x M Chimera with couplers and biases uniform on
    {-6..-1, 1..6}.  Each instance keeps a BFS ball of n vertices (n
    log-uniform on [n_min, n_max]) around a random start vertex; the other
    parent vertices are frozen at a random +-1 state and their couplings to
    the ball are folded into the ball's biases.  The induced colouring is the
    parent's.
    """
    parent = chimera(parent_M, j_max, h_max, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    out = []
    for _ in range(B):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        n = max(1, min(n, parent.n))
        start = int(rng.integers(0, parent.n))
        seen = np.zeros(parent.n, dtype=bool)
        seen[start] = True
        q = deque([start])
        ball = []
        while q and len(ball) < n:
            v = q.popleft()
            ball.append(v)
            for u in parent.col[parent.row_ptr[v]:parent.row_ptr[v + 1]]:
                if not seen[u]:
                    seen[u] = True
                    q.append(int(u))
        keep = np.zeros(parent.n, dtype=bool)
        keep[np.array(ball, dtype=np.int64)] = True
        frozen = rng.choice(np.array([-1, 1], dtype=np.int64), size=parent.n)
        ids = np.nonzero(keep)[0]
        new_id = -np.ones(parent.n, dtype=np.int64)
        new_id[ids] = np.arange(ids.size)
        rows = np.repeat(np.arange(parent.n), np.diff(parent.row_ptr))
        cols = parent.col.astype(np.int64)
        vals = parent.J.astype(np.int64)
        inside = keep[rows] & keep[cols]
        boundary = keep[rows] & ~keep[cols]
        hb = parent.h.astype(np.int64).copy()
        np.add.at(hb, rows[boundary], vals[boundary] * frozen[cols[boundary]])
        sel = inside & (rows < cols)
        inst = from_edges(ids.size, new_id[rows[sel]], new_id[cols[sel]], vals[sel], hb[ids],
                          parent.colour[ids], parent.n_colours, 0, name=f"residual{ids.size}")
        out.append(inst)
    return out


def disjoint_union(parts, perm_seed=None, name="union"):
    """Block-diagonal union of instances (a disconnected problem, as left by fixing),
    optionally with the variables shuffled by a seeded permutation so that components
    interleave in index order.  All parts must share scale_log2."""
    scale = parts[0].scale_log2
    if any(p.scale_log2 != scale for p in parts):
        raise ValueError("parts with different scale_log2")
    ei, ej, w, h, colour = [], [], [], [], []
    off = 0
    for p in parts:
        a, b, v = p.edges()
        ei.append(a + off)
        ej.append(b + off)
        w.append(v)
        h.append(np.asarray(p.h, np.int64))
        colour.append(np.asarray(p.colour, np.int64))
        off += p.n
    ei, ej, w = np.concatenate(ei), np.concatenate(ej), np.concatenate(w)
    h, colour = np.concatenate(h), np.concatenate(colour)
    n = off
    if perm_seed is not None:
        perm = np.random.default_rng(perm_seed).permutation(n)  # old index -> new index
        ei, ej = perm[ei], perm[ej]
        h2, c2 = np.empty_like(h), np.empty_like(colour)
        h2[perm], c2[perm] = h, colour
        h, colour = h2, c2
    return from_edges(n, ei, ej, w, h, colour, max(p.n_colours for p in parts), scale, name)


def linear_betas(beta0, beta1, sweeps):
    """beta_t = beta0 + (beta1 - beta0) * t / (sweeps - 1), t = 0..sweeps-1."""
    if sweeps == 1:
        return np.array([beta1], dtype=np.float64)
    t = np.arange(sweeps, dtype=np.float64)
    return beta0 + (beta1 - beta0) * t / float(sweeps - 1)


def geometric_betas(beta_min, beta_max, K):
    """beta_k = beta_min * (beta_max / beta_min) ** (k / (K - 1)), ascending."""
    if K == 1:
        return np.array([beta_min], dtype=np.float64)
    k = np.arange(K, dtype=np.float64)
    return beta_min * (beta_max / beta_min) ** (k / float(K - 1))


def random_spins(R, n, seed=0):
    """Uniform +-1 int8 spin matrix [R][n] (test samples / initial states)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.integers(0, 2, size=(R, n), dtype=np.int8) * 2 - 1).astype(np.int8)
