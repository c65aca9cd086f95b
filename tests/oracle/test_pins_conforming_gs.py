"""Multicolour Gauss-Seidel in the conforming space (Section 4, Table GS1;
Section 6, Table HYB3): the oracle's colour ordering of glued unknowns
against what fixes it.

* independence: unknowns of equal colour key never share a matrix entry, on
  every smoothed level of the L-shape (2D, three patches around a corner),
  the 2 x 2 square and the Fichera corner (3D, seven cubes around a vertex);
* a forward / backward sweep equals the triangular solve with the matrix
  permuted by the keys (scipy), so the ordering is a Gauss-Seidel method;
* the vertex-sharing colouring: patches with a common corner differ;
* Table GS1 (b) (tests/golden): PCG counts on the L-shape equal the printed
  ones within one iteration for p = 2, 3, 4 on levels 4 and 5;
* Table HYB3 (a) as a trend on the Fichera corner.  With the additive piece
  smoother read as eq. Ldef at the paper's damping 1 the cycle is not
  positive definite (smallest eigenvalue below zero, asserted), so the
  trend check runs at damping 0.5, the value used for the conforming
  SCMS elsewhere in this build.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import workloads
from oracle.smoothers import gs_color_keys

GOLDEN = os.path.join(os.path.dirname(os.path.dirname(__file__)), "golden")


def read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([None if v == "-" else int(v) for v in line.split()])
    return rows


def lshape(level, p, smoother="gs", **kw):
    return oracle.setup(workloads.lshape_corners(), workloads.lshape_elems(level), p,
                        conforming=True, smoother=smoother, coarse_min=1, **kw)


def fichera(level, p, smoother="hybrid", tau=0.5, **kw):
    return oracle.setup(workloads.fichera_corners(), workloads.fichera_elems(level), p,
                        conforming=True, smoother=smoother, tau=tau, delta=0.12, coarse_min=1,
                        **kw)


def test_vertex_colouring():
    """Patches with a common corner get different colours: the L-shape's
    three squares and the Fichera corner's seven cubes all meet at one
    vertex; the 2 x 2 square needs four colours, its face colouring two."""
    assert oracle.setup(workloads.lshape_corners(), workloads.lshape_elems(1), 2,
                        conforming=True, smoother="scms").topo.vertex_color == [0, 1, 2]
    assert sorted(fichera(1, 2, smoother="scms").topo.vertex_color) == list(range(7))
    cfg = workloads.config("c1", 8)
    topo = oracle.setup(cfg["corners"], cfg["elems"], 2, conforming=True,
                        smoother="scms").topo
    assert sorted(topo.vertex_color) == [0, 1, 2, 3] and max(topo.patch_color) == 1


@pytest.mark.parametrize("case", ["lshape_p2", "lshape_p3", "square_p2", "fichera_p2"])
def test_conforming_color_classes_independent_every_level(case):
    if case.startswith("lshape"):
        pb = lshape(3, int(case[-1]))
    elif case == "square_p2":
        cfg = workloads.config("c1", 2)
        pb = oracle.setup(cfg["corners"], cfg["elems"], 2, conforming=True, smoother="gs")
    else:
        pb = fichera(2, 2, smoother="gs")
    for l in range(1, len(pb.levels)):
        A = pb.A[l].tocoo()
        off = A.row != A.col
        for tile in (pb.gs_tile, 10 ** 6):
            keys = gs_color_keys(pb.levels[l], tile)
            assert not np.any(keys[A.row[off]] == keys[A.col[off]]), (case, l, tile)


@pytest.mark.parametrize("case", ["lshape", "fichera"])
def test_conforming_gauss_seidel_equals_triangular_solve(case):
    pb = lshape(3, 3) if case == "lshape" else fichera(2, 2, smoother="gs")
    l = pb.L
    A = pb.A[l].tocsr()
    keys = gs_color_keys(pb.levels[l], pb.gs_tile)
    perm = np.argsort(keys, kind="stable")
    Ap = A[perm][:, perm]
    rng = np.random.default_rng(11)
    f = rng.standard_normal(A.shape[0])
    u = rng.standard_normal(A.shape[0])
    r = (f - A @ u)[perm]
    fw = u.copy()
    fw[perm] += spla.spsolve_triangular(sp.tril(Ap, format="csr"), r, lower=True)
    np.testing.assert_allclose(pb.gs[l].forward(f, u), fw, rtol=1e-11, atol=1e-11)
    bw = u.copy()
    bw[perm] += spla.spsolve_triangular(sp.triu(Ap, format="csr"), r, lower=False)
    np.testing.assert_allclose(pb.gs[l].backward(f, u), bw, rtol=1e-11, atol=1e-11)


def test_gs1_lshape_pcg_counts():
    """Table GS1 (b): PCG with the Gauss-Seidel V-cycle on the L-shape takes
    the printed number of iterations within one (levels 4, 5; p = 2, 3, 4).
    Block (a), the multigrid iteration itself, converges here too but more
    slowly than printed (the printed ordering is not stated); it is checked
    to converge and to grow with p."""
    tab = {r[0]: r for r in read_table("gs1_lshape_conforming.txt")}
    for level in (4, 5):
        direct = []
        for p in (2, 3, 4):
            pb = lshape(level, p)
            f = pb.load_manufactured()
            its = pb.pcg(f)[1]
            printed = tab[level][8 + p - 2]
            assert abs(its - printed) <= 1, (level, p, its, printed)
            if p <= 3:
                _, itd, _ = pb.mg_iteration(f, maxit=200)
                assert itd < 200
                direct.append(itd)
        assert direct[0] < direct[1], direct


def cycle_matrix(pb):
    return np.stack([pb.vcycle(e) for e in np.eye(pb.N)], axis=1)


def test_hyb3_fichera_trend_and_damping():
    """Table HYB3 (a) as a trend: conforming hybrid PCG on the Fichera corner
    at damping 0.5 takes at most twice the printed count and stays flat from
    level 2 to 3 (p = 2).  At the paper's damping 1 the cycle of this reading
    has a negative eigenvalue (recorded: the PCG preconditioner is then not
    SPD and PCG stagnates)."""
    tab = {r[0]: r for r in read_table("hyb3_fichera.txt")}
    its = {}
    for level, p in ((2, 2), (3, 2), (2, 3)):
        pb = fichera(level, p)
        its[level, p] = pb.pcg(pb.load_manufactured())[1]
        assert its[level, p] <= 2 * tab[level][1 + p - 2], (level, p, its)
    assert abs(its[3, 2] - its[2, 2]) <= 1, its
    B = cycle_matrix(fichera(2, 2, tau=1.0))
    lam = np.linalg.eigvalsh(0.5 * (B + B.T))
    assert lam[0] < 0, lam[:3]
    B = cycle_matrix(fichera(2, 2, tau=0.5))
    assert np.linalg.eigvalsh(0.5 * (B + B.T))[0] > 0
