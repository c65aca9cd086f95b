"""Run-to-run determinism of the HIP path: the same inputs give bitwise the
same results, on one solver (two solves) and on a second solver built from
the same description.  Every sum on the path has a fixed order: the volume
operator's tiles are applied in colour classes with disjoint outputs, the
Gauss-Seidel and stored-row kernels add the cross-patch couplings of a row
from fixed slots in lane order, reductions (dot products, coarse solve, L2
error) combine fixed partials in a fixed order.

Cases cover each kernel family: the 2D volume operator (SIPG with the SCMS
smoother, conforming with Gauss-Seidel), stored rows with cross-patch
couplings and Gauss-Seidel in float64 and float32 (hybrid SIPG), the
lane-per-right-hand-side operator of float32 batches (the degree-6 workload
at 1/8 with 64 right-hand sides, iterative refinement), the 3D volume
operator and 3D stored rows.
"""
import numpy as np
import pytest

import workloads
from tests.gpu_common import gpu_solver

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "sipg_scms_vol2d": (("c2", 8), dict(smoother="scms", tau=0.25, delta=0.1), 1),
    "conforming_gs_vol2d": (("c1", 1), dict(smoother="gs"), 1),
    "sipg_hybrid_fp64": (("c2", 8), dict(), 3),
    "sipg_hybrid_fp32_fcg": (("c2", 8), dict(precision="fp32", outer="fcg"), 3),
    "c4_batch64_ir": (("c4", 8), dict(precision="fp32", outer="ir", max_rhs=64), 64),
    "sipg3d_scms_vol3d": (("c3", 8), dict(smoother="scms", precision="fp64", outer="pcg"), 1),
    "sipg3d_hybrid_fp64": (("c3", 8), dict(precision="fp64", outer="pcg"), 2),
}


def _rhs(n, ncol, seed):
    return torch.from_numpy(np.stack([workloads.normal_rhs(n, seed + j)
                                      for j in range(ncol)])).cuda()


@pytest.mark.parametrize("name", list(CASES))
def test_solve_twice_bitwise(name):
    (cfg_name, scale), over, ncol = CASES[name]
    cfg = workloads.config(cfg_name, scale)
    print("determinism case: %s (%s / %d, %d columns)" % (name, cfg_name, scale, ncol), flush=True)
    outs = []
    for build in range(2):
        sv = gpu_solver(cfg, **over)
        try:
            F = _rhs(sv.n_dofs, ncol, 7100)
            y1 = sv.apply(F)
            y2 = sv.apply(F)
            assert torch.equal(y1, y2)
            runs = 2 if build == 0 else 1
            for _ in range(runs):
                U, info = sv.solve(F, tol=1e-8, maxit=300)
                assert all(i["converged"] for i in info)
                outs.append((U.clone(), [i["iterations"] for i in info], y1.clone()))
        finally:
            sv.close()
    U0, it0, y0 = outs[0]
    for U, its, y in outs[1:]:
        assert its == it0
        assert torch.equal(U, U0), float((U - U0).abs().max())
        assert torch.equal(y, y0)
