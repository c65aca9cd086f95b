"""Pins of the oracle's discretization (Sections 2 and 3): matrix invariants,
exact reproduction of polynomial solutions by the SIPG form, the Galerkin
property of the fine-grid penalty (eq. a:galerkin), manufactured-solution
convergence rates, and the conforming limit of SIPG."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import oracle
import workloads
from oracle.discretize import Topology, Level, penalty
from oracle.hierarchy import prolongation


def rect_corners(xs, ys):
    """Axis-aligned rectangles (affine maps) on the grid xs x ys, x fastest."""
    out = []
    for j in range(len(ys) - 1):
        for i in range(len(xs) - 1):
            x0, x1, y0, y1 = xs[i], xs[i + 1], ys[j], ys[j + 1]
            out.append([[x0, y0], [x1, y0], [x0, y1], [x1, y1]])
    return np.array(out, float)


def test_sizes_match_configurations():
    """Unknown counts of the configurations: C1 1,089 (33^2), C2 115,652."""
    c1 = workloads.config("c1")
    topo = Topology(c1["corners"])
    assert Level(topo, c1["elems"], 2, True).N == 1089
    c2 = workloads.config("c2")
    topo = Topology(c2["corners"])
    lv = Level(topo, c2["elems"], 4, False)
    assert lv.N == 115652
    assert len(topo.interfaces) == 24
    assert topo.patch_color == [(i + j) % 2 for j in range(4) for i in range(4)]


@pytest.mark.parametrize("conforming", [False, True])
def test_symmetric_positive_definite(conforming):
    """P3: A symmetric, Cholesky succeeds; per-patch volume matrices have
    constants in their kernel (zero row sums) before Dirichlet elimination."""
    cfg = workloads.config("c2", scale=16)
    elems = cfg["elems"] if not conforming else np.full_like(cfg["elems"], 6)
    pb = oracle.setup(cfg["corners"], elems, 3, conforming=conforming, smoother="scms")
    for A in pb.A:
        Ad = A.toarray()
        assert np.abs(Ad - Ad.T).max() <= 1e-13 * np.abs(Ad).max()
        sla.cholesky(Ad)
    lev = pb.levels[-1]
    Kp = lev.volume_matrix(5)
    assert np.abs(Kp @ np.ones(Kp.shape[0])).max() < 1e-11 * abs(Kp).max()


@pytest.mark.parametrize("elems", [[[2, 2], [3, 3], [3, 3], [2, 2]], [[4, 4], [5, 5], [3, 3], [4, 4]]])
def test_sipg_reproduces_polynomial_solution(elems):
    """Consistency of eq. model:discr2: u = x(1-x)y(1-y) lies in every patch
    space (p = 2, affine maps), so the SIPG solution equals it and its
    coefficient vector satisfies A u = (f, phi) with f = -Delta u, also on
    non-matching interfaces.  A wrong sign, normal or missing flux term
    breaks this identity."""
    corners = rect_corners([0, 0.4, 1], [0, 0.65, 1])
    p = 2
    topo = Topology(corners)
    eta = penalty(topo, elems, p, 5.0)
    lev = Level(topo, elems, p, False, eta)
    A = lev.assemble()
    uex = lambda X: X[:, 0] * (1 - X[:, 0]) * X[:, 1] * (1 - X[:, 1])
    f = lambda X: 2 * X[:, 1] * (1 - X[:, 1]) + 2 * X[:, 0] * (1 - X[:, 0])
    b = lev.load(f)
    # patchwise L2 projection of u (exact because u is in the space)
    ut = np.zeros(lev.N_torn)
    for k in range(topo.K):
        C0, _, W, xh = lev.patch_collocation(k, p + 2)
        X, J = oracle.geometry.multilinear(corners[k], xh)
        w = W * np.abs(np.linalg.det(J))
        M = (C0.T @ (C0.multiply(w[:, None]))).toarray()
        ut[lev.offsets[k]:lev.offsets[k + 1]] = np.linalg.solve(M, C0.T @ (w * uex(X)))
    assert np.abs(ut[lev.dirichlet_torn]).max() < 1e-13
    u = lev.S @ ut
    np.testing.assert_allclose(A @ u, b, atol=1e-12 * np.abs(b).max())


def test_galerkin_identity_fine_penalty():
    """P5 / eq. a:galerkin: with the penalty of the finest grid on every level
    and affine maps, A_{l-1} = P^T A_l P (non-matching interfaces)."""
    corners = rect_corners([0, 0.45, 1], [0, 0.3, 1])
    elems = np.array([[4, 4], [6, 6], [6, 6], [4, 4]])
    pb = oracle.setup(corners, elems, 3, smoother="scms")
    for l in range(1, len(pb.levels)):
        P = pb.P[l]
        Ag = (P.T @ pb.A[l] @ P).toarray()
        Ac = pb.A[l - 1].toarray()
        assert np.abs(Ag - Ac).max() < 1e-11 * np.abs(Ac).max()


@pytest.mark.parametrize("conforming,p", [(True, 2), (False, 2), (False, 3)])
def test_manufactured_convergence_rate(conforming, p):
    """P13: L2 error of u = sin(pi x) sin(pi y) decays like h^(p+1) on a
    perturbed 2x2 layout (bilinear maps)."""
    corners = workloads.grid_corners((2, 2), frac=0.10 if not conforming else 0.0, seed=7)
    errs = []
    ns = [4, 8, 16]
    for n in ns:
        elems = np.full((4, 2), n)
        if not conforming:
            elems[1] = elems[2] = 3 * n // 2 if n >= 4 else n
        pb = oracle.setup(corners, elems, p, conforming=conforming, smoother="scms", coarse_min=n)
        b = pb.load_manufactured()
        u = spla.spsolve(pb.A[-1].tocsc(), b)
        errs.append(pb.l2_error(u))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert abs(rates[-1] - (p + 1)) < 0.35, rates


def test_sipg_tends_to_conforming():
    """On matching meshes the SIPG solution tends to the conforming one as
    sigma grows (Section 5): the gap shrinks proportionally to 1/sigma."""
    corners = rect_corners([0, 0.4, 1], [0, 0.65, 1])   # no mirror symmetry
    elems = np.full((4, 2), 4)
    conf = oracle.setup(corners, elems, 2, conforming=True, smoother="scms", coarse_min=4)
    uc = conf.levels[-1].E @ spla.spsolve(conf.A[-1].tocsc(), conf.load_manufactured())
    gaps = []
    for s in (1e2, 1e4):
        sip = oracle.setup(corners, elems, 2, sigma=s, smoother="scms", coarse_min=4)
        us = sip.levels[-1].E @ spla.spsolve(sip.A[-1].tocsc(), sip.load_manufactured())
        gaps.append(np.abs(us - uc).max())
    assert gaps[1] < gaps[0] / 50


@pytest.mark.parametrize("d", [2, 3])
def test_volume_row_matches_assembled_rows(d):
    """One stiffness row integrated over the support elements of its basis
    function equals the row of the whole-patch assembly (perturbed
    multilinear patches; interior, edge and corner basis functions)."""
    counts = (2, 1) if d == 2 else (1, 1, 2)
    corners = workloads.grid_corners(counts, frac=0.08, seed=7)
    elems = np.array([[5, 4][:d] + [3] * (d - 2), [4, 6][:d] + [5] * (d - 2)])
    lev = Level(Topology(corners), elems, 3, False, None)
    rng = np.random.default_rng(3)
    for k in range(2):
        A = lev.volume_matrix(k).toarray()
        n = lev.n[k]
        picks = [np.zeros(d, dtype=int), n - 1, n // 2] + [rng.integers(0, n) for _ in range(4)]
        for i in picks:
            li = 0
            for delta in range(d - 1, -1, -1):
                li = li * int(n[delta]) + int(i[delta])
            row = lev.volume_row(k, i)
            assert np.allclose(row, A[li], rtol=0, atol=1e-13 * np.abs(A[li]).max())


def test_volume_row_identity_cube_is_kronecker_sum():
    """On the identity-mapped unit cube the stiffness is the Kronecker sum
    K (x) M (x) M + M (x) K (x) M + M (x) M (x) K of the 1D mass and stiffness
    matrices of the B-spline bases (separation of variables)."""
    from oracle.smoothers import mass_stiffness_1d
    corners = workloads.grid_corners((1, 1, 1))
    ne = (3, 4, 5)
    lev = Level(Topology(corners), np.array([ne]), 2, False, None)
    M = [mass_stiffness_1d(e, 2)[0] for e in ne]
    K = [mass_stiffness_1d(e, 2)[1] for e in ne]
    A = (np.kron(M[2], np.kron(M[1], K[0])) + np.kron(M[2], np.kron(K[1], M[0]))
         + np.kron(K[2], np.kron(M[1], M[0])))
    n = lev.n[0]
    for i in ([0, 0, 0], [2, 3, 4], [4, 5, 6], [1, 2, 3]):
        li = (i[2] * n[1] + i[1]) * n[0] + i[0]
        assert np.allclose(lev.volume_row(0, i), A[li], rtol=0, atol=1e-13 * np.abs(A[li]).max())
