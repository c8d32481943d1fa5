"""Workload descriptors (sizes, schedules, seeds) for the five measured workloads.

Each stands in for a paper workload whose instances are not available:
  cubic4_sa     -- 3D spin glass L=4 (Sec. III.D), SA + iterated persistence
  chimera8_sa   -- Chimera U-set problems (Sec. III.C), SA + persistence
  cubic10_pt    -- 3D spin glass L=10 with parallel tempering (Sec. III.D.1)
  residual_batch-- residual problems left after fixing (Sec. II.C)
  cubic20_pticm -- 3D spin glass L=20 with PT + isoenergetic cluster moves
"""
from __future__ import annotations

from . import (chimera, cubic_lattice, geometric_betas, linear_betas, residual_batch)

CUBIC4_SA = dict(
    name="cubic4_sa", kind="sa", L=4, dist="pm1", inst_seed=1001, seed=2001,
    reads=100, sweeps=1000, beta0=0.1, beta1=3.0, elite=0.1, theta=1.0, gauge=2, rounds=5)

CHIMERA8_SA = dict(
    name="chimera8_sa", kind="sa", M=8, j_max=6, h_max=6, inst_seed=1002, seed=2002,
    reads=10000, sweeps=2000, beta0=0.1, beta1=5.0, elite=0.05, theta=0.95, gauge=0)

CUBIC10_PT = dict(
    name="cubic10_pt", kind="pt", L=10, dist="gauss", scale_log2=10, inst_seed=1003, seed=2003,
    K=32, beta_min=0.2, beta_max=5.0, runs=64, chains=1, sweeps=10000, icm=False,
    elite=0.2, theta=1.0, gauge=2)

RESIDUAL_BATCH = dict(
    name="residual_batch", kind="batch", B=512, parent_M=16, n_min=50, n_max=1000,
    inst_seed=1004, seed=2004, reads=1000, sweeps=1000, beta0=0.1, beta1=5.0)

CUBIC20_PTICM = dict(
    name="cubic20_pticm", kind="pt", L=20, dist="gauss", scale_log2=10, inst_seed=1005,
    seed=2005, K=40, beta_min=0.2, beta_max=5.0, runs=1, chains=2, sweeps=10000, icm=True,
    elite=0.2, theta=1.0, gauge=2)

ALL = [CUBIC4_SA, CHIMERA8_SA, CUBIC10_PT, RESIDUAL_BATCH, CUBIC20_PTICM]


def instance(cfg):
    """Instance(s) of a workload descriptor."""
    if cfg["kind"] == "batch":
        return residual_batch(cfg["B"], cfg["parent_M"], cfg["n_min"], cfg["n_max"],
                              seed=cfg["inst_seed"])
    if "M" in cfg:
        return chimera(cfg["M"], cfg["j_max"], cfg["h_max"], seed=cfg["inst_seed"])
    return cubic_lattice(cfg["L"], cfg["dist"], seed=cfg["inst_seed"],
                         scale_log2=cfg.get("scale_log2", 0))


def betas(cfg, sweeps=None):
    if cfg["kind"] == "pt":
        return geometric_betas(cfg["beta_min"], cfg["beta_max"], cfg["K"])
    return linear_betas(cfg["beta0"], cfg["beta1"], sweeps if sweeps is not None else cfg["sweeps"])
