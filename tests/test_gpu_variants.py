"""Cycle variants against the oracle: Gauss-Seidel alone and the subspace
corrected mass smoother alone (Algorithm 1 in the SIPG space), the W-cycle
(mu = 2, Algorithm 1's recursion taken twice below the second-coarsest
level), two smoothing steps (nu = 2), and the cycle used directly as the
solver.  Bars as in the parity tests: one cycle 1e-10, PCG solution 1e-9
(1e-10 per iteration beyond ten) with iteration counts equal up to one.
"""
import numpy as np
import pytest

import workloads
from tests.gpu_common import gpu_solver, oracle_problem, rel_err

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
    assert rel_err(z, ob.vcycle(f)) < 1e-10
    uo, its, _, _ = ob.pcg(f)
    u, info = sv.solve(_gpu(f), tol=1e-8, maxit=300)
    assert info[0]["converged"] and abs(info[0]["iterations"] - its) <= 1, (info, its)
    # rounding differences of the two sides grow with the number of iterations
    # (Gauss-Seidel alone needs about a hundred at p = 4)
    assert rel_err(u.cpu().numpy(), uo) < max(1e-9, 1e-10 * its)


def test_multigrid_iteration_as_solver():
    """The cycle as the iteration itself (u <- MG(u)), stopped on the float64
    residual, against the oracle's MG iteration."""
    cfg = workloads.config("c2", 8)
    ob = oracle_problem(cfg)
    sv = gpu_solver(cfg, outer="mg")
    f = workloads.normal_rhs(ob.N, 2002)
    uo, its, _ = ob.mg_iteration(f)
    u, info = sv.solve(_gpu(f), tol=1e-8, maxit=300)
    assert info[0]["converged"] and abs(info[0]["iterations"] - its) <= 1, (info, its)
    assert rel_err(u.cpu().numpy(), uo) < 1e-9
    assert np.linalg.norm(f - ob.A[-1] @ u.cpu().numpy()) / np.linalg.norm(f) <= 1.01e-8
    sv.close()
