"""Edge cases of the HIP path against the oracle: a single patch (no
interfaces, no interface pieces), degree 1 (a 3 x 3 stencil, one 16-lane
group per row), degree 8 (the largest built: a 17 x 17 stencil, 19 lane
groups), a strip of patches with ragged Gauss-Seidel tiles, a hierarchy of
one level (the cycle is the direct solve), both operator forms; and invalid
batch sizes rejected at the boundary.

Tolerances as in the parity tests: apply 1e-12, one cycle 1e-10 (explicit
inverses of the coarse matrix and pieces vs the oracle's Cholesky solves),
final solution 1e-10 (norm-wise and element-wise) against the oracle's
iterate at the library's iteration count, counts equal up to one.
"""
import ctypes

import numpy as np
import pytest

import workloads
from tests.gpu_common import gpu_solver, max_abs_rel, oracle_iterate, oracle_problem, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cfg(counts, p, n_even, n_odd, frac=0.1, seed=7):
    return dict(corners=workloads.grid_corners(counts, frac=frac, seed=seed),
                elems=workloads.checkerboard_elems(counts, n_even, n_odd), p=p, sigma=5.0,
                conforming=False, smoother="hybrid", tau=0.25, delta=0.1)


CASES = {
    "single_patch_p2": _cfg((1, 1), 2, 8, 8),
    "strip_p1": _cfg((3, 1), 1, 8, 12),
    "coarse_only_p3": _cfg((2, 1), 3, 5, 7),   # odd counts: one level, the direct solve
    "square_p6": _cfg((2, 2), 6, 8, 12),
    "pair_p8": _cfg((1, 2), 8, 8, 12),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    cfg = CASES[request.param]
    return cfg, oracle_problem(cfg)


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


@pytest.mark.parametrize("apply", ["auto", "sumfact"])
def test_edge_parity(case, apply):
    cfg, ob = case
    sv = gpu_solver(cfg, operator_apply=apply)
    assert sv.n_dofs == ob.N and sv.n_levels == len(ob.levels)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(ob.N)
    assert rel_err(sv.apply(_gpu(x)).cpu().numpy(), ob.apply(x)) < 1e-12
    f = workloads.normal_rhs(ob.N, 11)
    z = sv.vcycle(_gpu(f), torch.zeros(ob.N, dtype=torch.float64).cuda()).cpu().numpy()
    assert rel_err(z, ob.vcycle(f)) < 1e-10
    assert max_abs_rel(z, ob.vcycle(f)) < 1e-10
    uo, its, _, iterates = ob.pcg(f)
    u, info = sv.solve(_gpu(f), tol=1e-8, maxit=200)
    kg = info[0]["iterations"]
    assert info[0]["converged"] and abs(kg - its) <= 1, (info, its)
    ui = oracle_iterate(ob, f, kg, its, iterates) if kg > 0 else uo
    assert rel_err(u.cpu().numpy(), ui) < 1e-10
    assert max_abs_rel(u.cpu().numpy(), ui) < 1e-10
    assert np.linalg.norm(f - ob.A[-1] @ u.cpu().numpy()) / np.linalg.norm(f) <= 1e-8
    sv.close()


def test_invalid_batch_sizes_rejected():
    from paper_1902_01818_amd import igamg
    cfg = CASES["single_patch_p2"]
    sv = gpu_solver(cfg)
    x = torch.zeros(sv.n_dofs, dtype=torch.float64).cuda()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = ctypes.c_void_p(x.data_ptr())
    for nrhs in (0, -1):
        assert igamg._lib.igamg_apply(sv._h, p, p, nrhs, stream) == igamg.EINVAL
        assert igamg._lib.igamg_vcycle(sv._h, p, p, nrhs, stream) == igamg.EINVAL
    sv.close()
