"""Cycle variants against the oracle: Gauss-Seidel alone and the subspace
corrected mass smoother alone (Algorithm 1 in the SIPG space), the W-cycle
(mu = 2, Algorithm 1's recursion taken twice below the second-coarsest
level), two smoothing steps (nu = 2), and the cycle used directly as the
solver.  Bars as in the parity tests: one cycle 1e-10, final solution 1e-10
(norm-wise and element-wise) against the oracle's iterate at the library's
iteration count, counts equal up to one, true residual <= 1e-8.
"""
import numpy as np
import pytest

import workloads
from tests.gpu_common import gpu_solver, max_abs_rel, oracle_iterate, oracle_problem, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

VARIANTS = {
    "gs_only": dict(smoother="gs"),
    "scms_only": dict(smoother="scms"),
    "w_cycle": dict(mu=2),
    "two_steps": dict(nu=2),
}


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


@pytest.fixture(scope="module", params=sorted(VARIANTS))
def variant(request):
    cfg = workloads.config("c2", 8)
    over = VARIANTS[request.param]
    ob = oracle_problem(cfg, **over)
    sv = gpu_solver(cfg, **over)
    yield cfg, ob, sv
    sv.close()


def test_variant_cycle_and_solve(variant):
    cfg, ob, sv = variant
    f = workloads.normal_rhs(ob.N, 2002)
    z = sv.vcycle(_gpu(f), torch.zeros(ob.N, dtype=torch.float64).cuda()).cpu().numpy()
    zo = ob.vcycle(f)
    assert rel_err(z, zo) < 1e-10
    assert max_abs_rel(z, zo) < 1e-10
    uo, its, _, iterates = ob.pcg(f, maxit=300)
    u, info = sv.solve(_gpu(f), tol=1e-8, maxit=300)
    kg = info[0]["iterations"]
    assert info[0]["converged"] and abs(kg - its) <= 1, (info, its)
    ui = oracle_iterate(ob, f, kg, its, iterates)
    ug = u.cpu().numpy()
    print("%d iterations, error vs oracle iterate %.3e" % (kg, rel_err(ug, ui)))
    assert rel_err(ug, ui) < 1e-10
    assert max_abs_rel(ug, ui) < 1e-10
    assert np.linalg.norm(f - ob.A[-1] @ ug) / np.linalg.norm(f) <= 1e-8


def test_multigrid_iteration_as_solver():
    """The cycle as the iteration itself (u <- MG(u)), stopped on the float64
    residual, against the oracle's MG iteration."""
    cfg = workloads.config("c2", 8)
    ob = oracle_problem(cfg)
    sv = gpu_solver(cfg, outer="mg")
    f = workloads.normal_rhs(ob.N, 2002)
    uo, its, _ = ob.mg_iteration(f)
    u, info = sv.solve(_gpu(f), tol=1e-8, maxit=300)
    kg = info[0]["iterations"]
    assert info[0]["converged"] and abs(kg - its) <= 1, (info, its)
    ui = uo if kg == its else ob.mg_iteration(f, tol=0.0, maxit=kg)[0]
    assert rel_err(u.cpu().numpy(), ui) < 1e-10
    assert max_abs_rel(u.cpu().numpy(), ui) < 1e-10
    assert np.linalg.norm(f - ob.A[-1] @ u.cpu().numpy()) / np.linalg.norm(f) <= 1e-8
    sv.close()
