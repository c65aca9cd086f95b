"""Batches of right-hand sides and the float32 cycle, through the C ABI.

Batches: each right-hand side of a batch goes through the same kernels, with
the same operation order, as in a one-vector call; only the atomic
accumulation order of the volume kernel differs between any two runs.  Batched
results are therefore compared with one-vector results at 1e-12 and with the
oracle at the float64 parity bars.

Float32 cycle inside the float64 outer iteration (an extension beyond the
paper): the outer residual and its stopping test are float64, so the final
true residual (recomputed with the oracle's matrix) must meet the tolerance
exactly as in float64.  One float32 cycle is compared with the oracle's
float64 cycle at 2e-5 relative: the cycle's kernels round every stored value
to float32 (unit roundoff 6e-8) and a cycle sums contributions of six levels
and smoothing steps whose partial results cancel by up to two orders of
magnitude.
"""
import numpy as np
import pytest

import workloads
from tests.gpu_common import cached_oracle, gpu_solver, max_abs_rel, oracle_iterate, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _rhs_batch(n, seeds):
    return np.stack([workloads.normal_rhs(n, s) for s in seeds])


@pytest.fixture(scope="module")
def c2_small():
    return cached_oracle("c2", 8)


def test_batch_apply_cycle_equal_single(c2_small):
    cfg, ob = c2_small
    s1 = gpu_solver(cfg)
    sb = gpu_solver(cfg, max_rhs=3)
    rng = np.random.default_rng(31)
    X = rng.standard_normal((5, ob.N))   # 5 > max_rhs: batches of 3 and 2
    Yb = sb.apply(_gpu(X)).cpu().numpy()
    Ub = sb.vcycle(_gpu(X), torch.zeros(5 * ob.N, dtype=torch.float64).cuda()).cpu().numpy()
    Ub = Ub.reshape(5, ob.N)
    for j in range(5):
        y1 = s1.apply(_gpu(X[j])).cpu().numpy()
        u1 = s1.vcycle(_gpu(X[j]), torch.zeros(ob.N, dtype=torch.float64).cuda()).cpu().numpy()
        assert rel_err(Yb[j], y1) < 1e-12
        assert rel_err(Ub[j], u1) < 1e-12
        assert rel_err(Yb[j], ob.apply(X[j])) < 1e-12
        assert rel_err(Ub[j], ob.vcycle(X[j])) < 1e-10
        assert max_abs_rel(Ub[j], ob.vcycle(X[j])) < 1e-10
    s1.close()
    sb.close()


@pytest.mark.parametrize("outer", ["pcg", "mg"])
def test_batch_solve(c2_small, outer):
    cfg, ob = c2_small
    sb = gpu_solver(cfg, max_rhs=4, outer=outer)
    F = _rhs_batch(ob.N, [2002, 2003, 2004])
    F = np.concatenate([F, np.zeros((1, ob.N))])          # a zero right-hand side
    U, info = sb.solve(_gpu(F), tol=1e-8, maxit=200)
    U = U.cpu().numpy().reshape(4, ob.N)
    for j in range(3):
        kg = info[j]["iterations"]
        if outer == "pcg":
            uo, its, _, iterates = ob.pcg(F[j])
            ui = oracle_iterate(ob, F[j], kg, its, iterates)
        else:
            uo, its, _ = ob.mg_iteration(F[j])
            ui = uo if kg == its else ob.mg_iteration(F[j], tol=0.0, maxit=kg)[0]
        assert info[j]["converged"] and abs(kg - its) <= 1, (j, info[j], its)
        assert rel_err(U[j], ui) < 1e-10
        assert max_abs_rel(U[j], ui) < 1e-10
        assert np.linalg.norm(F[j] - ob.A[-1] @ U[j]) / np.linalg.norm(F[j]) <= 1e-8
    assert info[3]["iterations"] == 0 and not np.any(U[3])
    sb.close()


def test_fp32_one_cycle(c2_small):
    cfg, ob = c2_small
    sv = gpu_solver(cfg, precision="fp32")
    f = workloads.normal_rhs(ob.N, 2002)
    u = sv.vcycle(_gpu(f), torch.zeros(ob.N, dtype=torch.float64).cuda()).cpu().numpy()
    assert rel_err(u, ob.vcycle(f)) < 2e-5
    sv.close()


@pytest.mark.parametrize("outer", ["fcg", "pcg"])
def test_fp32_cycle_fp64_outer_solve(c2_small, outer):
    cfg, ob = c2_small
    sv = gpu_solver(cfg, precision="fp32", outer=outer, max_rhs=2)
    F = _rhs_batch(ob.N, [2002, 2005])
    U, info = sv.solve(_gpu(F), tol=1e-8, maxit=200)
    U = U.cpu().numpy().reshape(2, ob.N)
    for j in range(2):
        uo, its, _, _ = ob.pcg(F[j])
        nf = np.linalg.norm(F[j])
        true_res = np.linalg.norm(F[j] - ob.A[-1] @ U[j]) / nf
        assert info[j]["converged"]
        assert true_res <= 1e-8, true_res
        assert abs(info[j]["true_rel_residual"] - true_res) < 1e-12
        assert info[j]["iterations"] <= its + 2
        err = rel_err(U[j], ob.pcg(F[j], tol=1e-13)[0])
        print("fp32 cycle, %s: column %d error vs oracle %.3e" % (outer, j, err))
        assert err < 1e-6
    sv.close()


def test_bf16_scms_solve(c2_small):
    """bfloat16 operands in the patch-interior contractions (float32
    accumulation) inside float64 flexible CG: the float64 stopping test still
    decides, so the true residual meets the tolerance; the coarser smoother
    may cost iterations, bounded here by twice the float64 count."""
    cfg, ob = c2_small
    sv = gpu_solver(cfg, precision="bf16", outer="fcg", max_rhs=2)
    F = _rhs_batch(ob.N, [2002, 2005])
    U, info = sv.solve(_gpu(F), tol=1e-8, maxit=200)
    U = U.cpu().numpy().reshape(2, ob.N)
    for j in range(2):
        _, its, _, _ = ob.pcg(F[j])
        true_res = np.linalg.norm(F[j] - ob.A[-1] @ U[j]) / np.linalg.norm(F[j])
        assert info[j]["converged"]
        assert true_res <= 1e-8, true_res
        assert info[j]["iterations"] <= 2 * its, (info[j]["iterations"], its)
        err = rel_err(U[j], ob.pcg(F[j], tol=1e-13)[0])
        print("bf16 SCMS: column %d error vs oracle %.3e" % (j, err))
        assert err < 1e-6
    sv.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_iterative_refinement(c2_small, precision):
    """Float64 iterative refinement around inner PCG solves in the cycle
    arithmetic (relative reduction 1e-4 per refinement step): the float64
    residual decides, so the true residual meets the tolerance; restarting
    the Krylov space at every step may cost iterations, bounded here by twice
    the float64 PCG count."""
    cfg, ob = c2_small
    sv = gpu_solver(cfg, precision=precision, outer="ir", max_rhs=2)
    F = _rhs_batch(ob.N, [2002, 2005])
    U, info = sv.solve(_gpu(F), tol=1e-8, maxit=200, history=True)
    U = U.cpu().numpy().reshape(2, ob.N)
    for j in range(2):
        _, its, _, _ = ob.pcg(F[j])
        true_res = np.linalg.norm(F[j] - ob.A[-1] @ U[j]) / np.linalg.norm(F[j])
        assert info[j]["converged"], info[j]
        assert true_res <= 1e-8, true_res
        assert abs(info[j]["true_rel_residual"] - true_res) < 1e-12
        assert info[j]["iterations"] <= 2 * its, (info[j]["iterations"], its)
        err = rel_err(U[j], ob.pcg(F[j], tol=1e-13)[0])
        print("refinement, %s: column %d error vs oracle %.3e" % (precision, j, err))
        assert err < 1e-6
    sv.close()


def test_fp32_fullsize_solve():
    cfg, ob = cached_oracle("c2", 1)
    sv = gpu_solver(cfg, precision="fp32", outer="fcg")
    f = workloads.normal_rhs(ob.N, 2002)
    u, info = sv.solve(_gpu(f), tol=1e-8, maxit=200)
    u = u.cpu().numpy()
    assert info[0]["converged"]
    assert np.linalg.norm(f - ob.A[-1] @ u) / np.linalg.norm(f) <= 1e-8
    sv.close()
