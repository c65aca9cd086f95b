"""Float32 cycles on batches of right-hand sides against the same columns
one at a time: batches of 32 and more take the lane-per-right-hand-side
stored-row operator (and the grouped Gauss-Seidel sweeps), single columns
the 16-lane row kernels.  Both compute the same float32 operator in a
different summation order, so one cycle agrees to float32 rounding
amplified through the levels: 1e-5 relative per column (the float32 cycle
bar against the float64 oracle is 2e-5)."""
import numpy as np
import pytest

import workloads
from tests.gpu_common import gpu_solver, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("name,nrhs", [("c2", 64), ("c4", 64), ("c4", 40)])
def test_fp32_cycle_batch_equals_single(name, nrhs):
    cfg = workloads.config(name, 8)
    print("float32 batch case: %s/8 nrhs=%d" % (name, nrhs), flush=True)
    sb = gpu_solver(cfg, precision="fp32", outer="fcg", max_rhs=nrhs)
    s1 = gpu_solver(cfg, precision="fp32", outer="fcg")
    try:
        n = sb.n_dofs
        rng = np.random.default_rng(31)
        F = torch.from_numpy(rng.standard_normal((nrhs, n))).cuda()
        U0 = torch.from_numpy(0.1 * rng.standard_normal((nrhs, n))).cuda()
        Ub = sb.vcycle(F, U0.clone())
        for j in (0, 1, nrhs // 2, nrhs - 1):
            u1 = s1.vcycle(F[j].contiguous(), U0[j].clone().contiguous())
            assert rel_err(Ub[j].cpu().numpy(), u1.cpu().numpy()) < 1e-5, j
        # and the solve: float64 true residual 1e-8 for every column
        U, info = sb.solve(F, tol=1e-8, maxit=200)
        assert all(i["converged"] and i["true_rel_residual"] <= 1e-8 for i in info)
    finally:
        sb.close()
        s1.close()
