"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (float64 end to end, the two sides differ only in rounding
order, atomics and quadrature-node rounding):
  operator apply            1e-12 relative
  one cycle                 1e-10 relative (the library applies explicit
                            inverses of the coarse matrix and the interface
                            pieces, the oracle Cholesky solves: rounding
                            bounded by cond eps, cond(A_0) = 1.1e6 at the
                            benchmark size)
  PCG iterates k = 1..K     1e-10 relative
  final solution            1e-10 relative and element-wise against the
                            oracle's iterate at the library's iteration
                            count (equal counts up to one); true residual
                            with the oracle's matrix <= 1e-8
"""
import numpy as np
import pytest

import workloads
from tests.gpu_common import cached_oracle, gpu_solver, max_abs_rel, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (config, scale, Gauss-Seidel tile width; None = the default 2(p+1), the
# only width the library's Gauss-Seidel kernel takes, operator applies: "auto"
# = stored rows on the SIPG Gauss-Seidel levels, "sumfact" = matrix-free)
CASES = [("c1", 1, None, "auto"), ("c1", 2, None, "auto"), ("c2", 16, None, "auto"),
         ("c2", 8, None, "auto"), ("c2", 8, None, "sumfact")]


def _to_gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


@pytest.fixture(scope="module", params=CASES, ids=["%s/%d/T%s/%s" % c for c in CASES])
def pair(request):
    name, scale, gs_tile, apply = request.param
    cfg, ob = cached_oracle(name, scale, gs_tile)
    sv = gpu_solver(cfg, gs_tile=ob.gs_tile if not cfg["conforming"] else 0, operator_apply=apply)
    yield cfg, ob, sv
    sv.close()


def test_sizes(pair):
    cfg, ob, sv = pair
    assert sv.n_dofs == ob.N
    assert sv.n_levels == len(ob.levels)


def test_apply(pair):
    cfg, ob, sv = pair
    rng = np.random.default_rng(11)
    x = rng.standard_normal((2, ob.N))
    y = sv.apply(_to_gpu(x)).cpu().numpy()
    for j in range(2):
        assert rel_err(y[j], ob.apply(x[j])) < 1e-12


def test_load_manufactured(pair):
    cfg, ob, sv = pair
    f = sv.load_manufactured().cpu().numpy()
    assert rel_err(f, ob.load_manufactured()) < 1e-12


def test_one_cycle(pair):
    cfg, ob, sv = pair
    rng = np.random.default_rng(12)
    f = rng.standard_normal(ob.N)
    u0 = rng.standard_normal(ob.N) * 0.1
    ug = sv.vcycle(_to_gpu(f), _to_gpu(u0)).cpu().numpy()
    uo = ob.mg(ob.L, f, u0.copy())
    assert rel_err(ug, uo) < 1e-10
    assert max_abs_rel(ug, uo) < 1e-10


def test_pcg_iterates(pair):
    cfg, ob, sv = pair
    f = workloads.normal_rhs(ob.N, 2002)
    _, its, hist, iterates = ob.pcg(f)
    fg = _to_gpu(f)
    for k in range(1, min(its, 6) + 1):
        u, info = sv.solve(fg, tol=1e-8, maxit=k)
        assert rel_err(u.cpu().numpy(), iterates[k - 1]) < 1e-10, k
        assert max_abs_rel(u.cpu().numpy(), iterates[k - 1]) < 1e-10, k


def test_solve_final(pair):
    cfg, ob, sv = pair
    f = ob.load_manufactured() if cfg["rhs"] == "manufactured" else workloads.normal_rhs(ob.N, 2002)
    uo, its, hist, iterates = ob.pcg(f)
    u, info = sv.solve(_to_gpu(f), tol=1e-8, maxit=200, history=True)
    ug = u.cpu().numpy()
    kg = info[0]["iterations"]
    assert abs(kg - its) <= 1
    assert info[0]["converged"]
    if kg > its:
        _, _, _, iterates = ob.pcg(f, tol=0.0, maxit=kg)
    assert rel_err(ug, iterates[kg - 1]) < 1e-10
    assert max_abs_rel(ug, iterates[kg - 1]) < 1e-10
    # true residual with the oracle's matrix
    A = ob.A[-1]
    assert np.linalg.norm(f - A @ ug) / np.linalg.norm(f) <= 1e-8
    assert abs(info[0]["true_rel_residual"] - np.linalg.norm(f - A @ ug) / np.linalg.norm(f)) < 1e-12
    np.testing.assert_allclose(info[0]["history"][:len(hist)], hist[:len(info[0]["history"])],
                               rtol=1e-6, atol=1e-14)


def test_l2_error(pair):
    """L2 error against the manufactured solution (p+3 Gauss points) of the
    oracle's solution and of a perturbed copy: the library's fixed-order sum
    equals the oracle's quadrature up to rounding (the error is the
    difference of two O(1) functions: 1e-8 relative)."""
    cfg, ob, sv = pair
    f = ob.load_manufactured()
    uo, _, _, _ = ob.pcg(f)
    rng = np.random.default_rng(13)
    for u in (uo, uo + 1e-3 * rng.standard_normal(ob.N)):
        eg = sv.l2_error(_to_gpu(u))
        eo = ob.l2_error(u)
        assert abs(eg - eo) <= 1e-8 * eo, (eg, eo)
