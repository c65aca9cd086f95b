"""Preconditioner cycles replayed from captured HIP graphs (option graphs)
give bitwise the results of the same cycles launched kernel by kernel.

Every solve replays the graph once per outer iteration, with the outer
iteration's own kernels, copies and host waits between the replays; three
solves in a row (two right-hand sides, the first again at the end) check
that each replay reads the current vectors.  The launch sequence is the
same in both modes and every sum has a fixed order, so equality is exact.
Cases: float64 PCG (SIPG hybrid; conforming SCMS, whose cycle converts the
residual first), float32 cycle in flexible CG, the 64-column float32 batch
with iterative refinement (graph of the inner residual), 3D float64.
"""
import numpy as np
import pytest

import workloads
from tests.gpu_common import gpu_solver

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "sipg_hybrid_fp64": (("c2", 8), dict(), 1),
    "conforming_scms_fp64": (("c1", 1), dict(), 1),
    "sipg_hybrid_fp32_fcg": (("c2", 8), dict(precision="fp32", outer="fcg"), 2),
    "c4_batch64_ir": (("c4", 8), dict(precision="fp32", outer="ir", max_rhs=64), 64),
    "sipg3d_hybrid_fp64": (("c3", 8), dict(precision="fp64", outer="pcg"), 1),
}


def _rhs(n, ncol, seed):
    return torch.from_numpy(np.stack([workloads.normal_rhs(n, seed + j)
                                      for j in range(ncol)])).cuda()


def _solves(sv, rhs_list):
    out = []
    for F in rhs_list:
        U, info = sv.solve(F, tol=1e-8, maxit=300)
        torch.cuda.synchronize()
        assert all(i["converged"] and i["true_rel_residual"] <= 1e-8 for i in info)
        out.append((U.clone(), [i["iterations"] for i in info]))
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_graph_replays_equal_launches(name):
    (cfg_name, scale), over, ncol = CASES[name]
    cfg = workloads.config(cfg_name, scale)
    print("graph case: %s (%s / %d, %d columns)" % (name, cfg_name, scale, ncol), flush=True)
    res = {}
    for graphs in (False, True):
        sv = gpu_solver(cfg, graphs=graphs, **over)
        try:
            F1 = _rhs(sv.n_dofs, ncol, 7300)
            F2 = _rhs(sv.n_dofs, ncol, 7400)
            res[graphs] = _solves(sv, [F1, F2, F1])
        finally:
            sv.close()
    for (ue, ie), (ug, ig) in zip(res[False], res[True]):
        assert ie == ig
        assert torch.equal(ue, ug), float((ue - ug).abs().max())
    assert torch.equal(res[True][0][0], res[True][2][0])
