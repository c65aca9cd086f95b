"""Pins of the oracle's smoothers and cycles (Sections 4-6): the subspace
corrected mass smoother against its definition with explicit projections,
generalized-eigenproblem residuals, Gauss-Seidel against a library
triangular solve, symmetry / positivity / contraction of the cycle, direct
solves against library solvers, and the iteration counts the paper prints."""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import workloads
from oracle.smoothers import SCMS1D, scms_interior_apply, gs_color_keys, pieces

GOLDEN = os.path.join(os.path.dirname(os.path.dirname(__file__)), "golden")


def projected_scms_matrix(n_el, p, sigma, d):
    """L = sum_alpha Pi_alpha^T (sigma M_d + sum_{delta: alpha_delta = 1} K_delta) Pi_alpha
    with the M-orthogonal projections Pi_0 onto S~ = null(C) and Pi_1 = I - Pi_0,
    assembled densely from the definition of the splitting."""
    f = SCMS1D(n_el, p)
    M, K = f.M, f.K
    n = M.shape[0]
    if f.C.shape[0]:
        Z = sla.null_space(f.C)
        Pi0 = Z @ np.linalg.solve(Z.T @ M @ Z, Z.T @ M)
    else:
        Pi0 = np.eye(n)
    Pi = [Pi0, np.eye(n) - Pi0]

    def kron_all(ms):          # ms[0] = x (fastest)
        out = ms[-1]
        for m in ms[-2::-1]:
            out = np.kron(out, m)
        return out
    L = np.zeros((n ** d, n ** d))
    for alpha in range(2 ** d):
        a = [(alpha >> g) & 1 for g in range(d)]
        P = kron_all([Pi[a[g]] for g in range(d)])
        op = sigma * kron_all([M] * d)
        for g in range(d):
            if a[g]:
                op = op + kron_all([K if h == g else M for h in range(d)])
        L += P.T @ op @ P
    return L, f


@pytest.mark.parametrize("p,n_el,d", [(2, 6, 2), (3, 5, 2), (4, 6, 2), (5, 8, 2), (6, 9, 2), (3, 4, 3), (4, 5, 3)])
def test_scms_fast_form_equals_projected_definition(p, n_el, d):
    """P7: the fast-diagonalization apply equals L^-1 r with L built from the
    splitting S = S~ + S1 by explicit projections (basis independent)."""
    sigma = 1.0 / (0.1 / n_el ** 2)
    L, f = projected_scms_matrix(n_el, p, sigma, d)
    rng = np.random.default_rng(p * 7 + n_el)
    n = f.M.shape[0]
    r = rng.standard_normal(n ** d)
    y = scms_interior_apply([f] * d, sigma, 1.0, r.reshape((n,) * d)).ravel()
    np.testing.assert_allclose(y, np.linalg.solve(L, r), rtol=1e-10, atol=1e-12 * np.abs(y).max())


def test_scms_p2_is_scaled_mass():
    """P8: for p = 2 the complement S1 is empty and L_T = sigma M (x) M."""
    f = SCMS1D(8, 2)
    assert f.dim_S1 == 0
    sigma = 123.0
    n = f.M.shape[0]
    r = np.random.default_rng(0).standard_normal(n * n)
    y = scms_interior_apply([f, f], sigma, 1.0, r.reshape(n, n)).ravel()
    np.testing.assert_allclose(y, np.linalg.solve(sigma * np.kron(f.M, f.M), r), rtol=1e-11)


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6, 7, 8])
def test_scms_generalized_eigen_residuals(p):
    """P6: Q^T M Q = I, Q1^T K Q1 = diag(lam1), C Q~ = 0, dim S1 = 2 floor((p-1)/2)."""
    f = SCMS1D(16, p)
    n = f.M.shape[0]
    assert f.dim_S1 == 2 * ((p - 1) // 2)
    assert f.Q.shape == (n, n)
    np.testing.assert_allclose(f.Q.T @ f.M @ f.Q, np.eye(n), atol=1e-10)
    if f.dim_S1:
        # Galerkin residual of the eigenproblem restricted to S1 = range(Q1)
        R = f.Q1.T @ (f.K @ f.Q1 - f.M @ f.Q1 @ np.diag(f.lam1))
        assert np.abs(R).max() < 1e-9 * np.abs(f.lam1).max()
        # S1 is M-orthogonal to S~
        assert np.abs(f.Qt.T @ f.M @ f.Q1).max() < 1e-10
        assert np.abs(f.C @ f.Qt).max() < 1e-10
        assert np.all(f.lam1 > 0)


def test_scms_robust_in_degree():
    """P9: lambda_max(L^-1 K) of the parameter-domain interior problem stays in a
    narrow band for p = 2..8 (the smoother is robust in p)."""
    vals = []
    for p in range(2, 9):
        n_el = 12
        f = SCMS1D(n_el, p)
        sigma = n_el ** 2 / 0.1
        K2 = np.kron(f.M, f.K) + np.kron(f.K, f.M)
        n = f.M.shape[0]
        Linv = np.stack([scms_interior_apply([f, f], sigma, 1.0, e.reshape(n, n)).ravel()
                         for e in np.eye(n * n)], axis=1)
        vals.append(np.max(np.real(np.linalg.eigvals(Linv @ K2))))
    assert max(vals) < 3.0 and min(vals) > 0.5, vals


def small_c2(scale=16, **kw):
    cfg = workloads.config("c2", scale=scale)
    opts = dict(smoother="hybrid", tau=0.25, delta=0.1)
    opts.update(kw)
    return oracle.setup(cfg["corners"], cfg["elems"], cfg["p"], **opts)


def test_piece_structure_c2():
    """Pieces of the full C2 layout: 16 interiors, 24 edges of 164 unknowns,
    9 interior vertices of 4 unknowns (Section 5, Figure decomp right)."""
    from oracle.discretize import Topology, Level
    cfg = workloads.config("c2")
    lev = Level(Topology(cfg["corners"]), cfg["elems"], 4, False)
    ints, iface = pieces(lev)
    sizes = sorted(len(T) for T in iface)
    assert sizes == [4] * 9 + [164] * 24
    assert sum(len(c) for c, _ in ints) + sum(sizes) == lev.N


def test_gauss_seidel_equals_triangular_solve():
    """P10: a forward multicolour sweep equals u + L^-1 (f - A u) with L the
    lower triangle of A permuted by the colour keys (scipy triangular solve);
    the backward sweep uses the upper triangle."""
    pb = small_c2(scale=16)
    l = pb.L
    A = pb.A[l].tocsr()
    keys = gs_color_keys(pb.levels[l], pb.gs_tile)
    perm = np.argsort(keys, kind="stable")
    Ap = A[perm][:, perm]
    rng = np.random.default_rng(5)
    f = rng.standard_normal(A.shape[0])
    u = rng.standard_normal(A.shape[0])
    r = (f - A @ u)[perm]
    Lo = sp.tril(Ap, format="csr")
    Up = sp.triu(Ap, format="csr")
    fw = u.copy()
    fw[perm] += spla.spsolve_triangular(Lo, r, lower=True)
    np.testing.assert_allclose(pb.gs[l].forward(f, u), fw, rtol=1e-11, atol=1e-11)
    bw = u.copy()
    bw[perm] += spla.spsolve_triangular(Up, r, lower=False)
    np.testing.assert_allclose(pb.gs[l].backward(f, u), bw, rtol=1e-11, atol=1e-11)


def test_color_classes_are_independent():
    """Equal colour keys never share a matrix entry (race-freedom of a
    parallel sweep), also with the plain per-unknown colouring (tile = inf)."""
    pb = small_c2(scale=8)
    for l in range(1, len(pb.levels)):
        A = pb.A[l].tocoo()
        for tile in (pb.gs_tile, 10 ** 6):
            keys = gs_color_keys(pb.levels[l], tile)
            off = A.row != A.col
            assert not np.any(keys[A.row[off]] == keys[A.col[off]])


def cycle_matrix(pb):
    N = pb.N
    return np.stack([pb.vcycle(e) for e in np.eye(N)], axis=1)


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_cycle_symmetric_positive(which):
    """P11: one cycle B (zero initial guess) is symmetric and positive
    definite, as the conjugate gradient method requires (Section 4)."""
    if which == "c1":
        cfg = workloads.config("c1", scale=2)
        pb = oracle.setup(cfg["corners"], cfg["elems"], 2, conforming=True, smoother="scms",
                          tau=0.5, delta=0.12)
    else:
        pb = small_c2(scale=16)
    B = cycle_matrix(pb)
    assert np.abs(B - B.T).max() < 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_cycle_contracts_and_hybrid_not_worse():
    """P12: spectral radius of I - BA below 1 (the iteration matrix contracts
    in the energy norm) and the hybrid cycle is not worse than the pure
    SCMS cycle (Section 6, corollary on the hybrid iteration matrix)."""
    rho = {}
    for sm in ("hybrid", "scms"):
        pb = small_c2(scale=16, smoother=sm)
        B = cycle_matrix(pb)
        A = pb.A[-1].toarray()
        ev = np.linalg.eigvals(np.eye(pb.N) - B @ A)
        rho[sm] = np.max(np.abs(ev))
    assert rho["hybrid"] < 1.0
    assert rho["hybrid"] <= rho["scms"] + 1e-12


def test_coarse_and_final_solution_vs_library():
    """P14 / P15: the Cholesky coarse solve equals numpy.linalg.solve; PCG to
    1e-12 equals scipy's sparse direct solver to 1e-10."""
    pb = small_c2(scale=8)
    rng = np.random.default_rng(1)
    r0 = rng.standard_normal(pb.levels[0].N)
    np.testing.assert_allclose(pb.coarse_solve(r0), np.linalg.solve(pb.A[0].toarray(), r0), rtol=1e-10)
    f = workloads.normal_rhs(pb.N, 2002)
    u, it, hist, _ = pb.pcg(f, tol=1e-12)
    ud = spla.spsolve(pb.A[-1].tocsc(), f)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-10
    assert hist[-1] <= 1e-12


def read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([int(v) for v in line.split()])
    return np.array(rows)


def test_iteration_counts_in_paper_range():
    """P16 (trend only): PCG iteration counts of the hybrid SIPG cycle on the
    perturbed 4x4 layout with p = 4 stay within the range the paper prints
    for its hybrid SIPG experiments at p = 4 (Table HYB2 (b), tests/golden),
    widened by 3, and do not grow under refinement."""
    tab = read_table("hyb2_yeti_sipg_pcg.txt")      # columns: L, p=2..8
    lo, hi = tab[:, 3].min(), tab[:, 3].max()        # p = 4
    its = []
    for scale in (8, 4):
        pb = small_c2(scale=scale)
        f = workloads.normal_rhs(pb.N, 2002)
        its.append(pb.pcg(f)[1])
    assert all(lo - 3 <= i <= hi + 3 for i in its), (its, lo, hi)
    assert its[1] <= its[0] + 2
