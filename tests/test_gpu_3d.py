"""Parity of the 3D path with the FP64 oracle, through the C ABI: SIPG with
the Gauss-Seidel, hybrid and SCMS smoothers (SCMS patch interiors by six
mode-product stages, face / edge / vertex pieces by dense inverses), the
conforming space with SCMS, the operator from the stored rows or by sum
factorization, and a one-level hierarchy.

Inputs: trilinear 2 x 2 x 2 patch layouts with 5 % corner perturbation and
checkerboard element counts (the C3 structure at reduced size), a 2 x 1 x 1
layout with three levels, and the C3 layout itself divided by 8.
Tolerances as in the 2D parity tests (float64 end to end, rounding order
only): apply 1e-12, one cycle and PCG iterates 1e-10, final solution
1e-10 per iteration, equal iteration counts (+-1).
"""
import functools

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_common import gpu_solver, max_abs_rel, oracle_iterate, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _case(name, smoother="gs"):
    if name == "c3/8":
        cfg = workloads.config("c3", 8)
    elif name == "2x2x2/p2":
        cfg = dict(workloads.config("c3", 8))
        cfg.update(corners=workloads.grid_corners((2, 2, 2), frac=0.05, seed=31),
                   elems=workloads.checkerboard_elems((2, 2, 2), 4, 6), p=2)
    elif name == "2x1x1/p3":
        cfg = dict(workloads.config("c3", 8))
        cfg.update(corners=workloads.grid_corners((2, 1, 1), frac=0.05, seed=32),
                   elems=np.array([[8, 8, 8], [8, 8, 8]]), p=3)
    elif name == "conforming/p2":
        # matching interfaces (Assumption 2), glued unknowns
        cfg = dict(workloads.config("c3", 8))
        cfg.update(corners=workloads.grid_corners((2, 2, 2), frac=0.05, seed=33),
                   elems=np.full((8, 3), 4), p=2, conforming=True)
    elif name == "one-level/p3":
        # 2 elements per direction: the direct solve is the whole hierarchy
        cfg = dict(workloads.config("c3", 8))
        cfg.update(corners=workloads.grid_corners((2, 1, 1), frac=0.05, seed=34),
                   elems=np.full((2, 3), 2), p=3)
    else:
        raise KeyError(name)
    cfg = dict(cfg)
    cfg["smoother"] = smoother
    return cfg


@functools.lru_cache(maxsize=2)
def _oracle(name, smoother):
    cfg = _case(name, smoother)
    return cfg, oracle.setup(cfg["corners"], cfg["elems"], cfg["p"], sigma=cfg["sigma"],
                             conforming=cfg["conforming"], smoother=smoother, tau=cfg["tau"],
                             delta=cfg["delta"])


# (layout, smoother, operator form: "auto" = stored rows on Gauss-Seidel
# levels, "sumfact" = matrix-free sum factorization everywhere)
CASES = [("2x2x2/p2", "gs", "auto"), ("2x1x1/p3", "gs", "auto"), ("c3/8", "gs", "auto"),
         ("2x2x2/p2", "hybrid", "auto"), ("2x1x1/p3", "hybrid", "auto"),
         ("c3/8", "hybrid", "auto"), ("2x2x2/p2", "hybrid", "sumfact"),
         ("c3/8", "scms", "auto"), ("conforming/p2", "scms", "auto"),
         ("one-level/p3", "hybrid", "auto")]


def _to_gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


@pytest.fixture(scope="module", params=CASES, ids=["%s/%s/%s" % c for c in CASES])
def pair(request):
    print("3d case", request.param, flush=True)
    name, smoother, apply = request.param
    cfg, ob = _oracle(name, smoother)
    cfg = dict(cfg, operator_apply=apply)
    sv = gpu_solver(cfg, operator_apply=apply)
    yield cfg, ob, sv
    sv.close()


def test_sizes(pair):
    cfg, ob, sv = pair
    assert sv.n_dofs == ob.N
    assert sv.n_levels == len(ob.levels)


def test_apply(pair):
    cfg, ob, sv = pair
    rng = np.random.default_rng(11)
    x = rng.standard_normal((2, ob.N))
    y = sv.apply(_to_gpu(x)).cpu().numpy()
    for j in range(2):
        assert rel_err(y[j], ob.apply(x[j])) < 1e-12


def test_load_manufactured(pair):
    cfg, ob, sv = pair
    f = sv.load_manufactured().cpu().numpy()
    assert rel_err(f, ob.load_manufactured()) < 1e-12


def test_one_cycle(pair):
    cfg, ob, sv = pair
    rng = np.random.default_rng(12)
    f = rng.standard_normal(ob.N)
    u0 = rng.standard_normal(ob.N) * 0.1
    ug = sv.vcycle(_to_gpu(f), _to_gpu(u0)).cpu().numpy()
    uo = ob.mg(ob.L, f, u0.copy())
    assert rel_err(ug, uo) < 1e-10
    assert max_abs_rel(ug, uo) < 1e-10


def test_pcg_iterates(pair):
    cfg, ob, sv = pair
    f = workloads.normal_rhs(ob.N, 2002)
    _, its, hist, iterates = ob.pcg(f)
    fg = _to_gpu(f)
    for k in range(1, min(its, 4) + 1):
        u, info = sv.solve(fg, tol=1e-8, maxit=k)
        assert rel_err(u.cpu().numpy(), iterates[k - 1]) < 1e-10, k
        assert max_abs_rel(u.cpu().numpy(), iterates[k - 1]) < 1e-10, k


def test_solve_final(pair):
    cfg, ob, sv = pair
    f = ob.load_manufactured()
    uo, its, hist, iterates = ob.pcg(f)
    u, info = sv.solve(_to_gpu(f), tol=1e-8, maxit=200)
    ug = u.cpu().numpy()
    kg = info[0]["iterations"]
    assert abs(kg - its) <= 1
    assert info[0]["converged"]
    ui = oracle_iterate(ob, f, kg, its, iterates) if kg > 0 else uo
    assert rel_err(ug, ui) < 1e-10
    assert max_abs_rel(ug, ui) < 1e-10
    A = ob.A[-1]
    assert np.linalg.norm(f - A @ ug) / np.linalg.norm(f) <= 1e-8


def test_l2_error(pair):
    """L2 error against the manufactured solution in 3D: same vector, library
    and oracle quadrature agree to 1e-8 relative."""
    cfg, ob, sv = pair
    uo, _, _, _ = ob.pcg(ob.load_manufactured())
    eg = sv.l2_error(_to_gpu(uo))
    eo = ob.l2_error(uo)
    assert abs(eg - eo) <= 1e-8 * eo, (eg, eo)


def test_batch_matches_single(pair):
    cfg, ob, sv = pair
    F = np.stack([workloads.normal_rhs(ob.N, 70 + j) for j in range(3)])
    sb = gpu_solver(cfg, max_rhs=3, operator_apply=cfg["operator_apply"])
    try:
        U, infos = sb.solve(_to_gpu(F), tol=1e-8, maxit=200)
        U = U.cpu().numpy()
        for j in range(3):
            u1, i1 = sv.solve(_to_gpu(F[j]), tol=1e-8, maxit=200)
            assert infos[j]["iterations"] == i1[0]["iterations"]
            assert rel_err(U[j], u1.cpu().numpy()) < 1e-12
    finally:
        sb.close()


@pytest.mark.parametrize("outer", ["fcg", "pcg"])
def test_float32_cycle(pair, outer):
    """Float32 cycle (Gauss-Seidel, transfers, stored rows rounded once) inside
    the float64 outer iteration: converged to the same tolerance, solution
    within the discretization's conditioning of the oracle's."""
    cfg, ob, sv = pair
    f = ob.load_manufactured()
    uo, its, _, _ = ob.pcg(f)
    s32 = gpu_solver(cfg, precision="fp32", outer=outer, operator_apply=cfg["operator_apply"])
    try:
        u, info = s32.solve(_to_gpu(f), tol=1e-8, maxit=200)
        ug = u.cpu().numpy()
        assert info[0]["converged"]
        assert info[0]["iterations"] <= its + 3
        A = ob.A[-1]
        assert np.linalg.norm(f - A @ ug) / np.linalg.norm(f) <= 1e-8
        assert rel_err(ug, uo) < 1e-6
    finally:
        s32.close()


def test_bf16_scms(pair):
    """bfloat16 operands in the mode-product stages of the patch interiors
    (float32 accumulation, float32 cycle) inside float64 flexible CG: the
    float64 stopping test decides; iterations bounded by twice the float64
    count."""
    cfg, ob, sv = pair
    if cfg["smoother"] == "gs":
        pytest.skip("bfloat16 applies to the SCMS stages")
    f = ob.load_manufactured()
    _, its, _, _ = ob.pcg(f)
    sb = gpu_solver(cfg, precision="bf16", outer="fcg", operator_apply=cfg["operator_apply"])
    try:
        u, info = sb.solve(_to_gpu(f), tol=1e-8, maxit=200)
        ug = u.cpu().numpy()
        assert info[0]["converged"]
        assert np.linalg.norm(f - ob.A[-1] @ ug) / np.linalg.norm(f) <= 1e-8
        assert info[0]["iterations"] <= 2 * its, (info[0]["iterations"], its)
    finally:
        sb.close()


def test_unsupported_3d_options():
    """Stored operator rows without a Gauss-Seidel smoother and degrees above
    4 are refused; the conforming space on non-matching faces is an invalid
    argument (its interfaces must match)."""
    from paper_1902_01818_amd import igamg
    cfg = _case("2x2x2/p2")
    with pytest.raises(igamg.IgamgError) as e:
        gpu_solver(cfg, smoother="scms", operator_apply="rows")
    assert e.value.code == igamg.EUNSUPPORTED
    with pytest.raises(igamg.IgamgError) as e:
        gpu_solver(cfg, conforming=True, smoother="gs")
    assert e.value.code == igamg.EINVAL
    with pytest.raises(igamg.IgamgError) as e:
        gpu_solver(dict(cfg, p=5), smoother="gs")
    assert e.value.code == igamg.EUNSUPPORTED


@pytest.mark.parametrize("outer,precision", [("ir", "fp32"), ("ir", "bf16"), ("mg", "fp64")])
def test_outer_iterations_3d(outer, precision):
    """The other outer iterations on the C3 layout divided by 8 (hybrid):
    float64 iterative refinement around float32 / bf16-SCMS inner solves and
    the cycle used as the iteration itself; the float64 residual decides, so
    the true residual meets the tolerance and the solution matches the
    oracle's PCG solution to 1e-6."""
    cfg, ob = _oracle("c3/8", "hybrid")
    f = ob.load_manufactured()
    uo, its, _, _ = ob.pcg(f)
    sv = gpu_solver(cfg, precision=precision, outer=outer)
    try:
        u, info = sv.solve(_to_gpu(f), tol=1e-8, maxit=200)
        ug = u.cpu().numpy()
        assert info[0]["converged"], info
        assert np.linalg.norm(f - ob.A[-1] @ ug) / np.linalg.norm(f) <= 1e-8
        assert rel_err(ug, uo) < 1e-6
    finally:
        sv.close()
