"""Parity of the 3D SIPG cycle with a degree per patch (the non-matching
spaces of Section 5 on the Fichera corner of Table HYB3 (b), and a perturbed
2x1x1 layout with degrees 3 / 2) with the FP64 oracle, through the C ABI.

Stored rows take the largest degree's (2p_max+1)^3 layout on every patch,
the Gauss-Seidel order the largest degree's tiles and positions.  Bars as in
the 2D test: apply 1e-12, one cycle and PCG iterates 1e-10 (norm-wise and
element-wise), final solution 1e-10 against the oracle's iterate at the
library's iteration count, load 1e-12, L2 error 1e-8 relative.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_common import max_abs_rel, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = [("fichera", 3, 2, "hybrid", 0.5), ("fichera", 2, 2, "gs", 0.25),
         ("fichera", 2, 2, "scms", 0.5), ("2x1x1", 0, 0, "hybrid", 0.25)]


def _problem(name, lev, p):
    if name == "fichera":
        elems, deg = workloads.nonmatching_spaces(workloads.fichera_elems(lev), p)
        return workloads.fichera_corners(), elems, deg
    corners = workloads.grid_corners((2, 1, 1), frac=0.05, seed=35)
    return corners, np.array([[6, 6, 6], [4, 4, 4]]), np.array([3, 2])


def _to_gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


@pytest.fixture(scope="module", params=CASES, ids=["%s/%d/p%d/%s" % c[:4] for c in CASES])
def pair(request):
    from paper_1902_01818_amd import igamg
    name, lev, p, smoother, tau = request.param
    corners, elems, deg = _problem(name, lev, p)
    print("3D non-matching case: %s %d degrees %s %s tau %g" % (name, lev, list(deg), smoother,
                                                                 tau), flush=True)
    ob = oracle.setup(corners, elems, deg, smoother=smoother, tau=tau, delta=0.12, coarse_min=1)
    sv = igamg.Solver(corners, elems, deg, 5.0, smoother=smoother, tau=tau, delta=0.12,
                      coarse_min=1)
    yield ob, sv
    sv.close()


def test_sizes(pair):
    ob, sv = pair
    assert sv.n_dofs == ob.N and sv.n_levels == len(ob.levels)


def test_apply(pair):
    ob, sv = pair
    x = np.random.default_rng(51).standard_normal((2, ob.N))
    y = sv.apply(_to_gpu(x)).cpu().numpy()
    for j in range(2):
        yo = ob.apply(x[j])
        assert rel_err(y[j], yo) < 1e-12
        assert max_abs_rel(y[j], yo) < 1e-12


def test_load_and_l2(pair):
    ob, sv = pair
    f = sv.load_manufactured().cpu().numpy()
    fo = ob.load_manufactured()
    assert rel_err(f, fo) < 1e-12
    uo = ob.pcg(fo, tol=1e-12)[0]
    eg, eo = sv.l2_error(_to_gpu(uo)), ob.l2_error(uo)
    assert abs(eg - eo) <= 1e-8 * eo, (eg, eo)


def test_one_cycle(pair):
    ob, sv = pair
    rng = np.random.default_rng(52)
    f = rng.standard_normal(ob.N)
    u0 = 0.1 * rng.standard_normal(ob.N)
    ug = sv.vcycle(_to_gpu(f), _to_gpu(u0)).cpu().numpy()
    uo = ob.mg(ob.L, f, u0.copy())
    assert rel_err(ug, uo) < 1e-10
    assert max_abs_rel(ug, uo) < 1e-10


def test_pcg_iterates_and_final(pair):
    ob, sv = pair
    f = ob.load_manufactured()
    _, its, _, iterates = ob.pcg(f)
    fg = _to_gpu(f)
    for k in range(1, min(its, 5) + 1):
        u, _ = sv.solve(fg, tol=1e-8, maxit=k)
        assert rel_err(u.cpu().numpy(), iterates[k - 1]) < 1e-10, k
    u, info = sv.solve(fg, tol=1e-8, maxit=300)
    kg = info[0]["iterations"]
    assert info[0]["converged"] and abs(kg - its) <= 1, (kg, its)
    if kg > its:
        iterates = ob.pcg(f, tol=0.0, maxit=kg)[3]
    ug = u.cpu().numpy()
    assert rel_err(ug, iterates[kg - 1]) < 1e-10
    assert max_abs_rel(ug, iterates[kg - 1]) < 1e-10
