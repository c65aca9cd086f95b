"""Shared helpers of the GPU parity tests: one oracle problem and one HIP
solver built from the same seeded workload description."""
import functools

import numpy as np

import oracle
import workloads


def oracle_problem(cfg, **over):
    opts = dict(sigma=cfg["sigma"], conforming=cfg["conforming"], smoother=cfg["smoother"],
                tau=cfg["tau"], delta=cfg["delta"])
    opts.update(over)
    return oracle.setup(cfg["corners"], cfg["elems"], cfg["p"], **opts)


def gpu_solver(cfg, **over):
    from paper_1902_01818_amd import igamg
    opts = dict(conforming=cfg["conforming"], smoother=cfg["smoother"], tau=cfg["tau"],
                delta=cfg["delta"])
    opts.update(over)
    sigma = opts.pop("sigma", cfg["sigma"])
    return igamg.Solver(cfg["corners"], cfg["elems"], cfg["p"], sigma, **opts)


@functools.lru_cache(maxsize=8)
def cached_oracle(name, scale, gs_tile=None, coarse_min=None):
    cfg = workloads.config(name, scale)
    over = {} if gs_tile is None else dict(gs_tile=gs_tile)
    if coarse_min is not None:
        over["coarse_min"] = coarse_min
    return cfg, oracle_problem(cfg, **over)


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
