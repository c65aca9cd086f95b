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


def max_abs_rel(a, b):
    """Element-wise bar: max_i |a_i - b_i| / max_i |b_i|."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def oracle_iterate(ob, f, k, its, iterates, outer="pcg"):
    """The oracle's k-th iterate of the same outer iteration (k may exceed the
    oracle's own iteration count by one when the library's recurrence
    residual crosses the tolerance one step later)."""
    if k <= its:
        return iterates[k - 1]
    if outer == "mg":
        return ob.mg_iteration(f, tol=0.0, maxit=k)[0]
    return ob.pcg(f, tol=0.0, maxit=k)[3][k - 1]
