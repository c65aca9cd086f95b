"""Parity of the conforming-space Gauss-Seidel and hybrid cycles (Section 4,
Table GS1; Section 6, Table HYB3) with the FP64 oracle, through the C ABI.

The layouts are the paper's L-shaped domain (three unit squares around a
re-entrant corner, one element per patch on level 0), the 2 x 2 square
(four patches around an interior vertex) and the Fichera corner (seven unit
cubes around a vertex).  Glued unknowns couple every patch around their
vertex or edge; the library folds the rows of their copies into the first
copy and mirrors its updates to the others.  Both sides sweep in the same
multicolour order (keys at an unknown's first copy, patch colours of the
vertex-sharing graph).

Tolerances as in the SIPG parity tests: one cycle and PCG iterates 1e-10
relative, norm-wise and element-wise (max |diff| / max |u|); final solution
1e-10 against the oracle's iterate at the library's iteration count (equal
up to one), true residual <= 1e-8.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_common import max_abs_rel, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (layout, refinement level / element count, degree, smoother, damping)
CASES = [("lshape", 4, 2, "gs", 0.25), ("lshape", 4, 3, "gs", 0.25), ("lshape", 3, 4, "gs", 0.25),
         ("lshape", 4, 3, "hybrid", 0.5), ("lshape", 4, 2, "scms", 1.0),
         ("square", 16, 2, "gs", 0.25), ("square", 8, 3, "hybrid", 0.5),
         ("fichera", 2, 2, "gs", 0.25), ("fichera", 2, 2, "hybrid", 0.5),
         ("fichera", 2, 3, "gs", 0.25)]


def _layout(name, lev):
    if name == "lshape":
        return workloads.lshape_corners(), workloads.lshape_elems(lev)
    if name == "square":
        return workloads.grid_corners((2, 2)), np.full((4, 2), lev, dtype=np.int64)
    return workloads.fichera_corners(), workloads.fichera_elems(lev)


def _to_gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


@pytest.fixture(scope="module", params=CASES, ids=["%s/%d/p%d/%s" % c[:4] for c in CASES])
def pair(request):
    from paper_1902_01818_amd import igamg
    name, lev, p, smoother, tau = request.param
    corners, elems = _layout(name, lev)
    print("conforming parity case: %s %d p=%d %s tau=%g" % (name, lev, p, smoother, tau),
          flush=True)
    ob = oracle.setup(corners, elems, p, conforming=True, smoother=smoother, tau=tau,
                      delta=0.12, coarse_min=1)
    sv = igamg.Solver(corners, elems, p, 5.0, conforming=True, smoother=smoother, tau=tau,
                      delta=0.12, coarse_min=1)
    yield ob, sv
    sv.close()


def test_sizes(pair):
    ob, sv = pair
    assert sv.n_dofs == ob.N and sv.n_levels == len(ob.levels)


def test_one_cycle(pair):
    ob, sv = pair
    rng = np.random.default_rng(21)
    f = rng.standard_normal(ob.N)
    u0 = 0.1 * rng.standard_normal(ob.N)
    ug = sv.vcycle(_to_gpu(f), _to_gpu(u0)).cpu().numpy()
    uo = ob.mg(ob.L, f, u0.copy())
    assert rel_err(ug, uo) < 1e-10
    assert max_abs_rel(ug, uo) < 1e-10


def test_pcg_iterates_and_final(pair):
    ob, sv = pair
    f = ob.load_manufactured()
    uo, its, hist, iterates = ob.pcg(f)
    fg = _to_gpu(f)
    for k in range(1, min(its, 5) + 1):
        u, _ = sv.solve(fg, tol=1e-8, maxit=k)
        assert rel_err(u.cpu().numpy(), iterates[k - 1]) < 1e-10, k
        assert max_abs_rel(u.cpu().numpy(), iterates[k - 1]) < 1e-10, k
    u, info = sv.solve(fg, tol=1e-8, maxit=300)
    kg = info[0]["iterations"]
    assert info[0]["converged"] and abs(kg - its) <= 1, (kg, its)
    if kg > its:
        iterates = ob.pcg(f, tol=0.0, maxit=kg)[3]
    ug = u.cpu().numpy()
    assert rel_err(ug, iterates[kg - 1]) < 1e-10
    assert max_abs_rel(ug, iterates[kg - 1]) < 1e-10
    assert np.linalg.norm(f - ob.A[-1] @ ug) / np.linalg.norm(f) <= 1e-8


def test_multigrid_iteration_lshape():
    """Column (a) of Table GS1: the Gauss-Seidel V-cycle used directly as the
    solver; the library's iterate after k cycles equals the oracle's."""
    from paper_1902_01818_amd import igamg
    corners, elems = _layout("lshape", 4)
    ob = oracle.setup(corners, elems, 3, conforming=True, smoother="gs", coarse_min=1)
    sv = igamg.Solver(corners, elems, 3, 5.0, conforming=True, smoother="gs", coarse_min=1,
                      outer="mg")
    try:
        f = ob.load_manufactured()
        _, its, _ = ob.mg_iteration(f, maxit=200)
        u, info = sv.solve(_to_gpu(f), tol=1e-8, maxit=200)
        assert abs(info[0]["iterations"] - its) <= 1
        uo, _, _ = ob.mg_iteration(f, tol=0.0, maxit=5)
        u5, _ = sv.solve(_to_gpu(f), tol=1e-30, maxit=5)
        assert rel_err(u5.cpu().numpy(), uo) < 1e-10
    finally:
        sv.close()


@pytest.mark.parametrize("outer", ["fcg", "ir"])
def test_float32_cycle_lshape(outer):
    """Float32 Gauss-Seidel cycle inside float64 flexible CG, or float64
    iterative refinement around a float32 inner PCG (whose cycle input is
    the weighted float32 residual of the glued space), on the L-shape:
    reaches the float64 true residual 1e-8 (flexible CG within two
    iterations of the float64 count, refinement within twice it) and agrees
    with the float64 solution to 1e-6."""
    from paper_1902_01818_amd import igamg
    corners, elems = _layout("lshape", 5)
    s64 = igamg.Solver(corners, elems, 3, 5.0, conforming=True, smoother="gs", coarse_min=1)
    s32 = igamg.Solver(corners, elems, 3, 5.0, conforming=True, smoother="gs", coarse_min=1,
                       precision="fp32", outer=outer)
    try:
        f = s64.load_manufactured()
        u64, i64 = s64.solve(f, tol=1e-8, maxit=200)
        u32, i32 = s32.solve(f, tol=1e-8, maxit=200)
        assert i32[0]["converged"] and i32[0]["true_rel_residual"] <= 1e-8
        bound = i64[0]["iterations"] + 2 if outer == "fcg" else 2 * i64[0]["iterations"]
        assert i32[0]["iterations"] <= bound, (i32[0]["iterations"], i64[0]["iterations"])
        assert float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64)) < 1e-6
    finally:
        s64.close()
        s32.close()


@pytest.mark.parametrize("case", [("square", 8, 3, "hybrid", 0.5), ("lshape", 4, 2, "scms", 1.0)],
                         ids=["square/8/p3/hybrid", "lshape/4/p2/scms"])
def test_float32_batch_cycle(case):
    """A float32 cycle on 16 right-hand sides at once in the glued space (at
    this size the interface pieces run inside the fused SCMS launch and add
    each row into every copy of its unknown) against the oracle's float64
    cycle, column by column, to the float32 bar 2e-5."""
    from paper_1902_01818_amd import igamg
    name, lev, p, smoother, tau = case
    corners, elems = _layout(name, lev)
    print("conforming float32 batch case: %s %d p=%d %s" % (name, lev, p, smoother), flush=True)
    ob = oracle.setup(corners, elems, p, conforming=True, smoother=smoother, tau=tau, delta=0.12,
                      coarse_min=1)
    sv = igamg.Solver(corners, elems, p, 5.0, conforming=True, smoother=smoother, tau=tau,
                      delta=0.12, coarse_min=1, precision="fp32", max_rhs=16)
    try:
        rng = np.random.default_rng(23)
        F = rng.standard_normal((16, ob.N))
        U0 = 0.1 * rng.standard_normal((16, ob.N))
        Ug = sv.vcycle(_to_gpu(F), _to_gpu(U0)).cpu().numpy().reshape(16, ob.N)
        for j in range(16):
            uo = ob.mg(ob.L, F[j], U0[j].copy())
            assert rel_err(Ug[j], uo) < 2e-5, j
            assert max_abs_rel(Ug[j], uo) < 2e-5, j
    finally:
        sv.close()
