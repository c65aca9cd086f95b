"""Pins of the oracle's three-dimensional parts (Sections 2, 3 and 5):

* consistency of eq. model:discr2 on faces: a polynomial solution that lies
  in every patch space is reproduced exactly, A u = (f, phi), on 2x1x1 and
  2x2x1 layouts of sheared boxes (a general affine map: oblique faces, a
  surface element different from one, normals that are not coordinate
  directions) with non-matching faces;
* symmetry and positive definiteness of the 3D SIPG and conforming matrices;
* manufactured-solution L2 error of order p+1 in 3D, SIPG on perturbed
  trilinear patches and the conforming space (glued faces, edges, vertices);
* the conforming 3D space as the large-penalty limit of SIPG on matching
  meshes;
* the piece decomposition of the full 3D layout (Section 5, Figure decomp:
  12 faces of 6,626, 6 edges of 228 and one vertex of 8 unknowns);
* independence of the 3D colour classes on every level, and a 3D sweep equal
  to the triangular solve with the permuted lower triangle.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import workloads
from oracle.discretize import Level, Topology, penalty
from oracle.smoothers import gs_color_keys, pieces

SHEAR = np.array([[1.0, 0.2, 0.1], [0.1, 0.9, 0.15], [0.05, -0.1, 1.1]])


def box_corners(xs, ys, zs, A=SHEAR):
    """Boxes of the grid xs x ys x zs of the unit cube (x fastest), mapped by
    the affine map x -> A x."""
    out = []
    for k in range(len(zs) - 1):
        for j in range(len(ys) - 1):
            for i in range(len(xs) - 1):
                cs = []
                for b in range(8):
                    r = np.array([xs[i + (b & 1)], ys[j + ((b >> 1) & 1)], zs[k + ((b >> 2) & 1)]])
                    cs.append(A @ r)
                out.append(cs)
    return np.array(out, float)


def _poly_and_rhs(A=SHEAR):
    """u = prod_i g(l_i) with g(s) = s(1-s) and l = A^-1 x the reference
    coordinates (zero on the boundary of the sheared cube), and f = -Delta u
    written out by the chain rule: Delta u = sum_ij G_ij d_i d_j u~ with
    G = A^-1 A^-T."""
    Ai = np.linalg.inv(A)
    G = Ai @ Ai.T

    def ref(X):
        return X @ Ai.T

    def u(X):
        L = ref(X)
        return np.prod(L * (1 - L), axis=1)

    def f(X):
        L = ref(X)
        g = L * (1 - L)
        g1 = 1 - 2 * L
        lap = np.zeros(len(X))
        for i in range(3):
            for j in range(3):
                if i == j:
                    t = -2.0 * np.prod(np.delete(g, i, axis=1), axis=1)
                else:
                    k = 3 - i - j
                    t = g1[:, i] * g1[:, j] * g[:, k]
                lap += G[i, j] * t
        return -lap
    return u, f


def _projection(lev, corners, uex):
    """Patchwise L2 projection of uex onto the patch spaces (exact when uex
    lies in them), torn ordering."""
    ut = np.zeros(lev.N_torn)
    p = lev.p
    for k in range(lev.topo.K):
        C0, _, W, xh = lev.patch_collocation(k, p + 2)
        X, J = oracle.geometry.multilinear(corners[k], xh)
        w = W * np.abs(np.linalg.det(J))
        M = (C0.T @ (C0.multiply(w[:, None]))).toarray()
        ut[lev.offsets[k]:lev.offsets[k + 1]] = np.linalg.solve(M, C0.T @ (w * uex(X)))
    return ut


LAYOUTS = {
    "2x1x1": (box_corners([0, 0.4, 1], [0, 1], [0, 1]), np.array([[3, 3, 3], [4, 5, 4]])),
    # patches in reverse order: the lower-numbered patch meets its neighbour
    # on its low side, so the outer normal of its face points to -x
    "2x1x1-reversed": (box_corners([0, 0.4, 1], [0, 1], [0, 1])[::-1].copy(),
                       np.array([[4, 5, 4], [3, 3, 3]])),
    "2x2x1": (box_corners([0, 0.4, 1], [0, 0.55, 1], [0, 1]),
              np.array([[3, 3, 2], [4, 5, 3], [5, 4, 4], [3, 3, 3]])),
}


@pytest.mark.parametrize("name", sorted(LAYOUTS))
def test_sipg_3d_reproduces_polynomial_solution(name):
    """eq. model:discr2 in 3D: the exact solution lies in the discrete space
    (p = 2, affine maps), so its coefficients satisfy A u = (f, phi) on
    non-matching faces.  A wrong sign or surface element of the face terms, a
    wrong normal or a dropped flux term breaks this identity."""
    corners, elems = LAYOUTS[name]
    p = 2
    topo = Topology(corners)
    assert len(topo.interfaces) == (4 if name == "2x2x1" else 1)
    lev = Level(topo, elems, p, False, penalty(topo, elems, p, 5.0))
    A = lev.assemble()
    uex, f = _poly_and_rhs()
    ut = _projection(lev, corners, uex)
    assert np.abs(ut[lev.dirichlet_torn]).max() < 1e-13
    u = lev.S @ ut
    b = lev.load(f)
    np.testing.assert_allclose(A @ u, b, atol=1e-12 * np.abs(b).max())


def test_sipg_3d_flux_term_is_pinned():
    """The reproduction identity fails when the face flux terms are dropped
    (the identity is not satisfied by the volume part alone)."""
    corners, elems = LAYOUTS["2x1x1"]
    topo = Topology(corners)
    lev = Level(topo, elems, 2, False, penalty(topo, elems, 2, 5.0))
    uex, f = _poly_and_rhs()
    u = lev.S @ _projection(lev, corners, uex)
    Avol = (lev.E.T @ sp.block_diag([lev.volume_matrix(k) for k in range(2)]) @ lev.E).tocsr()
    b = lev.load(f)
    assert np.abs(Avol @ u - b).max() > 1e-3 * np.abs(b).max()


@pytest.mark.parametrize("conforming", [False, True])
def test_3d_symmetric_positive_definite(conforming):
    corners = workloads.grid_corners((2, 2, 1), frac=0.0 if conforming else 0.08, seed=5)
    elems = np.full((4, 3), 3) if conforming else workloads.checkerboard_elems((2, 2, 1), 3, 4)
    pb = oracle.setup(corners, elems, 2, conforming=conforming, smoother="scms", coarse_min=3)
    A = pb.A[-1].toarray()
    assert np.abs(A - A.T).max() < 1e-14 * np.abs(A).max()
    np.linalg.cholesky(A)


@pytest.mark.parametrize("conforming,p", [(False, 2), (True, 2), (False, 3)])
def test_3d_manufactured_convergence_rate(conforming, p):
    """L2 error of u = sin(pi x) sin(pi y) sin(pi z) decays like h^(p+1):
    SIPG on perturbed trilinear 2x1x1 patches with non-matching faces, the
    conforming space on a matching 2x1x1 layout."""
    corners = workloads.grid_corners((2, 1, 1), frac=0.0 if conforming else 0.08, seed=9)
    errs = []
    ns = [2, 4, 8] if p == 2 else [2, 4, 6]
    for n in ns:
        elems = np.full((2, 3), n)
        if not conforming:
            elems[1] = [n + 1, n + 2, n + 1] if n < 8 else [12, 12, 12]
        pb = oracle.setup(corners, elems, p, conforming=conforming, smoother="scms",
                          coarse_min=n + 8)
        u = spla.spsolve(pb.A[-1].tocsc(), pb.load_manufactured())
        errs.append(pb.l2_error(u))
    hs = np.array([1.0 / n for n in ns])
    rates = np.log(np.array(errs[:-1]) / np.array(errs[1:])) / np.log(hs[:-1] / hs[1:])
    assert abs(rates[-1] - (p + 1)) < 0.45, (rates, errs)


def test_3d_sipg_tends_to_conforming():
    """On matching 3D meshes the SIPG solution tends to the conforming one as
    sigma grows; the gap shrinks like 1/sigma (pins the glue of faces, edges
    and vertices against the independently assembled face terms)."""
    corners = box_corners([0, 0.4, 1], [0, 0.55, 1], [0, 1])
    elems = np.full((4, 3), 2)
    conf = oracle.setup(corners, elems, 2, conforming=True, smoother="scms", coarse_min=2)
    uc = conf.levels[-1].E @ spla.spsolve(conf.A[-1].tocsc(), conf.load_manufactured())
    gaps = []
    for s in (1e2, 1e4):
        sip = oracle.setup(corners, elems, 2, sigma=s, smoother="scms", coarse_min=2)
        us = sip.levels[-1].E @ spla.spsolve(sip.A[-1].tocsc(), sip.load_manufactured())
        gaps.append(np.abs(us - uc).max())
    assert gaps[1] < gaps[0] / 50, gaps


def test_piece_structure_c3():
    """Pieces of the full 3D layout (2x2x2 patches, 48/64 elements, p = 3):
    8 interiors, 12 faces of 49^2 + 65^2 = 6,626 unknowns, 6 interior edges
    of 2 x 49 + 2 x 65 = 228 and the centre vertex with one unknown of each
    of the 8 patches (Section 5, Figure decomp right); they cover every
    unknown once (1,649,984)."""
    cfg = workloads.config("c3")
    lev = Level(Topology(cfg["corners"]), cfg["elems"], 3, False)
    assert lev.N == 1649984
    ints, iface = pieces(lev)
    sizes = sorted(len(T) for T in iface)
    assert sizes == [8] + [228] * 6 + [6626] * 12
    assert sorted(c.size for c, _ in ints) == [49 ** 3] * 4 + [65 ** 3] * 4
    assert sum(c.size for c, _ in ints) + sum(sizes) == lev.N


def test_3d_color_classes_independent_every_level():
    """Equal colour keys never share a matrix entry on any level of the 3D
    layout at 1/8 of its element counts (6/8 elements, p = 3), with the tile
    width of the library and with the plain per-unknown colouring."""
    cfg = workloads.config("c3", 8)
    pb = oracle.setup(cfg["corners"], cfg["elems"], cfg["p"], smoother="hybrid", tau=0.25,
                      delta=0.12)
    assert len(pb.levels) == 2
    for l in range(len(pb.levels)):
        A = pb.A[l].tocoo()
        off = A.row != A.col
        for tile in (pb.gs_tile, 10 ** 6):
            keys = gs_color_keys(pb.levels[l], tile)
            assert not np.any(keys[A.row[off]] == keys[A.col[off]]), (l, tile)
        # 2 patch colours x 8 tile parities x (p+1)^3 positions at most
        assert len(np.unique(gs_color_keys(pb.levels[l], pb.gs_tile))) <= 2 * 8 * 4 ** 3


def test_3d_gauss_seidel_equals_triangular_solve():
    """A forward 3D sweep equals u + L^-1 (f - A u), L the lower triangle of A
    permuted by the colour keys; backward with the upper triangle."""
    corners = workloads.grid_corners((2, 1, 1), frac=0.05, seed=3)
    elems = workloads.checkerboard_elems((2, 1, 1), 4, 6)
    pb = oracle.setup(corners, elems, 2, smoother="hybrid", tau=0.25, delta=0.12)
    l = pb.L
    A = pb.A[l].tocsr()
    keys = gs_color_keys(pb.levels[l], pb.gs_tile)
    perm = np.argsort(keys, kind="stable")
    Ap = A[perm][:, perm]
    rng = np.random.default_rng(8)
    f = rng.standard_normal(A.shape[0])
    u = rng.standard_normal(A.shape[0])
    r = (f - A @ u)[perm]
    fw = u.copy()
    fw[perm] += spla.spsolve_triangular(sp.tril(Ap, format="csr"), r, lower=True)
    np.testing.assert_allclose(pb.gs[l].forward(f, u), fw, rtol=1e-11, atol=1e-11)
    bw = u.copy()
    bw[perm] += spla.spsolve_triangular(sp.triu(Ap, format="csr"), r, lower=False)
    np.testing.assert_allclose(pb.gs[l].backward(f, u), bw, rtol=1e-11, atol=1e-11)
