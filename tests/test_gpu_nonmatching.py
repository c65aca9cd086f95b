"""Parity of the SIPG cycle with a degree per patch (the non-matching spaces
of Section 5, Table SCMS2: one third of the patches S_{p,h}, one third
S_{p+1,2h}, one third S_{p,2h}) with the FP64 oracle, through the C ABI.

Layouts: the paper's L-shape (three unit squares) and a perturbed 3 x 2
layout, degrees p and p+1 side by side, interfaces non-matching in degree
and element count.  Smoothers: SCMS (Algorithm 1 with eq. Ldef), the hybrid
smoother (Algorithm 2) and Gauss-Seidel, whose stored rows and multicolour
order take the largest degree's layout on every patch.  Bars as in the
other parity tests: operator apply 1e-12, one cycle and PCG iterates 1e-10
(norm-wise and element-wise), final solution 1e-10 against the oracle's
iterate at the library's iteration count; load and L2 error of the
manufactured solution 1e-12 / 1e-8 relative; a float32 cycle over a batch
of 32 columns (the lane-per-right-hand-side operator) 2e-5.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_common import max_abs_rel, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = [("lshape", 4, 2, "scms", 0.5), ("lshape", 6, 3, "scms", 0.5),
         ("lshape", 3, 5, "scms", 0.9), ("grid3x2", 16, 4, "scms", 0.5),
         ("lshape", 5, 2, "hybrid", 0.25), ("grid3x2", 16, 3, "hybrid", 0.25),
         ("grid3x2", 8, 3, "gs", 0.25)]


def _problem(name, lev, p):
    if name == "lshape":
        corners = workloads.lshape_corners()
        base = workloads.lshape_elems(lev)
    else:
        corners = workloads.grid_corners((3, 2), frac=0.08, seed=77)
        base = np.full((6, 2), lev, dtype=np.int64)
    elems, deg = workloads.nonmatching_spaces(base, p)
    return corners, elems, deg


def _to_gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


@pytest.fixture(scope="module", params=CASES, ids=["%s/%d/p%d/%s" % c[:4] for c in CASES])
def pair(request):
    from paper_1902_01818_amd import igamg
    name, lev, p, smoother, tau = request.param
    corners, elems, deg = _problem(name, lev, p)
    print("non-matching case: %s %d degrees %s %s tau %g" % (name, lev, list(deg), smoother, tau),
          flush=True)
    ob = oracle.setup(corners, elems, deg, smoother=smoother, tau=tau, delta=0.12, coarse_min=1)
    sv = igamg.Solver(corners, elems, deg, 5.0, smoother=smoother, tau=tau, delta=0.12,
                      coarse_min=1)
    sv.case = (corners, elems, deg, smoother, tau)
    yield ob, sv
    sv.close()


def test_sizes(pair):
    ob, sv = pair
    assert sv.n_dofs == ob.N and sv.n_levels == len(ob.levels)


def test_apply(pair):
    ob, sv = pair
    x = np.random.default_rng(41).standard_normal((2, ob.N))
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
    rng = np.random.default_rng(42)
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
    assert np.linalg.norm(f - ob.A[-1] @ ug) / np.linalg.norm(f) <= 1e-8


def test_float32_batch_cycle(pair):
    """32 columns through the float32 cycle (lane-per-right-hand-side rows on
    Gauss-Seidel levels) against the float64 oracle's cycle, sampled columns."""
    from paper_1902_01818_amd import igamg
    ob, sv = pair
    corners, elems, deg, smoother, tau = sv.case
    if smoother == "scms":
        pytest.skip("no stored rows with the SCMS smoother alone (its float32 cycle is covered "
                    "by the batch tests of the single-degree workloads)")
    nb = 32
    s32 = igamg.Solver(corners, elems, deg, 5.0, smoother=smoother, tau=tau, delta=0.12,
                       coarse_min=1, precision="fp32", max_rhs=nb)
    try:
        F = np.random.default_rng(43).standard_normal((nb, ob.N))
        Z = s32.vcycle(_to_gpu(F), torch.zeros(nb * ob.N, dtype=torch.float64).cuda())
        Z = Z.cpu().numpy().reshape(nb, ob.N)
        for j in (0, 13, nb - 1):
            zo = ob.vcycle(F[j])
            assert rel_err(Z[j], zo) < 2e-5, j
            assert max_abs_rel(Z[j], zo) < 2e-5, j
    finally:
        s32.close()
