"""Brute-force helpers for tiny instances (independent of the oracle's loops).

The objective is evaluated with dense numpy linear algebra over the full
state table: E(s) = sum_{i<j} J_ij s_i s_j + sum_i h_i s_i (Sec. I), using the
strictly upper triangle of the dense coupling matrix so every coupler counts
once.
"""
import numpy as np


def dense(inst):
    Jd = np.zeros((inst.n, inst.n), dtype=np.int64)
    rows = np.repeat(np.arange(inst.n), np.diff(inst.row_ptr))
    Jd[rows, inst.col] = inst.J
    return Jd


def all_states(n):
    codes = np.arange(2 ** n, dtype=np.int64)
    bits = (codes[:, None] >> np.arange(n)[None, :]) & 1
    return (2 * bits - 1).astype(np.int8)


def energies(inst, S):
    S = np.asarray(S, dtype=np.int64).reshape(-1, inst.n)
    Ju = np.triu(dense(inst), 1)
    return np.einsum("ri,ij,rj->r", S, Ju, S) + S @ inst.h.astype(np.int64)


def ground(inst):
    S = all_states(inst.n)
    E = energies(inst, S)
    return S, E
