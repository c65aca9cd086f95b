"""Parity at the full size of the benchmark workload (2D SIPG, 4x4 bilinear
patches, 64/96 elements, p = 4, 115,652 unknowns), with the hierarchy the
halving rule gives (6 levels, coarsest 2/3 elements) and with the one the
benchmark times (4 levels, direct solve on 8/12 elements)."""
import numpy as np
import pytest

import workloads
from tests.gpu_common import cached_oracle, gpu_solver, max_abs_rel, oracle_iterate, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", params=[2, 8], ids=["coarse2", "coarse8"])
def full_pair(request):
    cm = request.param
    cfg, ob = cached_oracle("c2", 1, None, cm)
    sv = gpu_solver(cfg, coarse_min=cm)   # library defaults otherwise, as in bench.py
    assert ob.gs_tile == 2 * (cfg["p"] + 1)
    assert sv.n_levels == len(ob.levels) == (6 if cm == 2 else 4)
    yield cfg, ob, sv
    sv.close()


def test_full_apply_and_cycle(full_pair):
    cfg, ob, sv = full_pair
    assert sv.n_dofs == ob.N == 115652
    rng = np.random.default_rng(21)
    x = rng.standard_normal(ob.N)
    y = sv.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel_err(y, ob.apply(x)) < 1e-12
    f = workloads.normal_rhs(ob.N, 2002)
    z = sv.vcycle(torch.from_numpy(f).cuda(), torch.zeros(ob.N, dtype=torch.float64).cuda())
    # the coarse solve applies an explicit inverse (the oracle a Cholesky
    # solve): its relative rounding is bounded by cond(A_0) eps = 1.1e6 x 2.2e-16
    assert rel_err(z.cpu().numpy(), ob.vcycle(f)) < 1e-10


def test_full_solve(full_pair):
    cfg, ob, sv = full_pair
    f = workloads.normal_rhs(ob.N, 2002)
    uo, its, hist, iterates = ob.pcg(f)
    u, info = sv.solve(torch.from_numpy(f).cuda(), tol=1e-8, maxit=200)
    ug = u.cpu().numpy()
    kg = info[0]["iterations"]
    assert info[0]["converged"] and abs(kg - its) <= 1
    ui = oracle_iterate(ob, f, kg, its, iterates)
    assert rel_err(ug, ui) < 1e-10
    assert max_abs_rel(ug, ui) < 1e-10
    assert np.linalg.norm(f - ob.A[-1] @ ug) / np.linalg.norm(f) <= 1e-8


def test_full_batch_cycle_staged_smoother(full_pair):
    """64 right-hand sides at the full size: the patch-interior solves of the
    finest level take the four-stage batched form (64 x (66^2 x 5 + 98^2 x
    7) x 8 fused-form re-reads exceed its threshold); two columns of the
    batched cycle match the oracle's cycle at the float64 cycle bar."""
    cfg, ob, sv = full_pair
    nb = 64
    sb = gpu_solver(cfg, coarse_min=2 if sv.n_levels == 6 else 8, max_rhs=nb)
    F = np.stack([workloads.normal_rhs(ob.N, 3000 + j) for j in range(nb)])
    Z = sb.vcycle(torch.from_numpy(F).cuda(), torch.zeros(nb * ob.N, dtype=torch.float64).cuda())
    Z = Z.cpu().numpy().reshape(nb, ob.N)
    for j in (0, nb - 1):
        zo = ob.vcycle(F[j])
        assert rel_err(Z[j], zo) < 1e-10, j
        assert max_abs_rel(Z[j], zo) < 1e-10, j
    sb.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_full_batch_low_precision_staged_smoother(full_pair, precision):
    """64 right-hand sides at the full size in float32 (and with bf16 SCMS
    operands): the patch interiors go through the four-stage batched form in
    that arithmetic.  float32: two columns of one cycle match the oracle's
    float64 cycle at the float32 cycle bar (2e-5); both: every column of a
    flexible CG solve meets the float64 true residual 1e-8."""
    cfg, ob, sv = full_pair
    nb = 64
    sb = gpu_solver(cfg, coarse_min=2 if sv.n_levels == 6 else 8, max_rhs=nb,
                    precision=precision, outer="fcg")
    F = np.stack([workloads.normal_rhs(ob.N, 3000 + j) for j in range(nb)])
    if precision == "fp32":
        Z = sb.vcycle(torch.from_numpy(F).cuda(), torch.zeros(nb * ob.N, dtype=torch.float64).cuda())
        Z = Z.cpu().numpy().reshape(nb, ob.N)
        for j in (0, nb - 1):
            assert rel_err(Z[j], ob.vcycle(F[j])) < 2e-5, j
    U, info = sb.solve(torch.from_numpy(F).cuda(), tol=1e-8, maxit=200)
    U = U.cpu().numpy().reshape(nb, ob.N)
    assert all(i["converged"] for i in info)
    for j in (0, nb - 1):
        assert np.linalg.norm(F[j] - ob.A[-1] @ U[j]) / np.linalg.norm(F[j]) <= 1e-8, j
    sb.close()
