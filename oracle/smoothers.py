"""Multigrid smoothers (Sections 4-6).

* Gauss-Seidel (Section 4): u <- u + L^-1 (f - A u), L = lower triangle of A
  in a fixed ordering of the unknowns; the backward sweep uses L^T.  The
  ordering is a multicolour one (colour key below), so every colour class is
  a set of mutually uncoupled unknowns and a sweep equals the triangular
  solve with the permuted matrix.
* Subspace corrected mass smoother (Section 5, eq. Ldef):
  L^-1 = tau sum_T P_T L_T^-1 P_T^T over pieces T (patch interiors, edges,
  vertices, faces).  Interface pieces: L_T = P_T^T A P_T, solved directly.
  Patch interiors: the subspace corrected mass smoother of Hofreither and
  Takacs (2017) with scaling sigma = 1/(delta h^2) on the parameter domain.

Oracle code: test infrastructure only.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import bspline


# ---------------------------------------------------------------------------
# 1D ingredients of the subspace corrected mass smoother
# ---------------------------------------------------------------------------
def mass_stiffness_1d(n_el, p, q=None):
    """Parameter-domain mass and stiffness matrices of all n_el+p B-splines,
    Gauss quadrature with q = p+1 points per element (exact)."""
    q = p + 1 if q is None else q
    knots = bspline.open_uniform_knots(n_el, p)
    x, w = bspline.element_quadrature(n_el, q)
    B = bspline.basis_table(knots, p, x)[-1]
    D = bspline.basis_derivative(knots, p, x, 1)
    M = B.T @ (w[:, None] * B)
    Kst = D.T @ (w[:, None] * D)
    return M, Kst


def scms_constraints(n_el, p):
    """Rows h^{2l} B_i^{(2l)}(0) and h^{2l} B_i^{(2l)}(1), 1 <= l, 2l < p, for the
    interior B-splines i = 1..n-2.  Their null space is the subspace
    S~ = {v : v^{(2l)}(0) = v^{(2l)}(1) = 0}."""
    knots = bspline.open_uniform_knots(n_el, p)
    n = n_el + p
    h = 1.0 / n_el
    rows = []
    l = 1
    while 2 * l < p:
        for x in (0.0, 1.0):
            r = bspline.basis_derivative(knots, p, np.array([x]), 2 * l)[0, 1:n - 1]
            rows.append(h ** (2 * l) * r)
        l += 1
    return np.array(rows).reshape(len(rows), n - 2)


class SCMS1D:
    """Fast-diagonalization factors of one direction:
    Q = [Q~, Q1] with Q^T M Q = I, Q1^T K Q1 = diag(lam1), lam = [0.., lam1]."""

    def __init__(self, n_el, p):
        M, Kst = mass_stiffness_1d(n_el, p)
        self.M = M[1:-1, 1:-1]
        self.K = Kst[1:-1, 1:-1]
        C = scms_constraints(n_el, p)
        self.C = C
        npr = self.M.shape[0]
        m = C.shape[0]
        if m:
            Zt = sla.null_space(C)
            assert Zt.shape[1] == npr - m, "constraints not of full rank"
            Z1 = np.linalg.solve(self.M, C.T)        # M-orthogonal complement
        else:
            Zt = np.eye(npr)
            Z1 = np.zeros((npr, 0))
        w, V = sla.eigh(Zt.T @ self.K @ Zt, Zt.T @ self.M @ Zt)
        Qt = Zt @ V
        if m:
            lam1, V1 = sla.eigh(Z1.T @ self.K @ Z1, Z1.T @ self.M @ Z1)
            Q1 = Z1 @ V1
        else:
            lam1 = np.zeros(0)
            Q1 = np.zeros((npr, 0))
        self.Qt, self.Q1, self.lam1 = Qt, Q1, lam1
        self.Q = np.hstack([Qt, Q1])
        self.lam = np.concatenate([np.zeros(Qt.shape[1]), lam1])
        self.dim_S1 = m


def scms_interior_apply(factors, sigma, gamma, r):
    """L_T^-1 r = gamma^-1 (x)Q diag(1/(sigma + sum_d lam_d)) (x)Q^T r for a
    patch interior; r has shape (n'_{d-1}, ..., n'_0) (x fastest)."""
    d = len(factors)
    y = r
    for delta in range(d):          # apply Q^T along every direction
        ax = d - 1 - delta
        y = np.moveaxis(np.tensordot(factors[delta].Q.T, y, axes=([1], [ax])), 0, ax)
    denom = np.full(y.shape, sigma)
    for delta in range(d):
        ax = d - 1 - delta
        shape = [1] * d
        shape[ax] = -1
        denom = denom + factors[delta].lam.reshape(shape)
    y = y / denom
    for delta in range(d):
        ax = d - 1 - delta
        y = np.moveaxis(np.tensordot(factors[delta].Q, y, axes=([1], [ax])), 0, ax)
    return y / gamma


# ---------------------------------------------------------------------------
# pieces (Section 5, Figure decomp)
# ---------------------------------------------------------------------------
def pieces(level):
    """Split the compact unknowns into pieces: one per patch interior, one per
    physical edge / face / vertex (the DOFs of all adjacent patches, Section 5
    for the conforming and the SIPG case).  Returns (interiors, interface)
    where interiors[k] = (compact indices in lexicographic order, shape) and
    interface = list of compact index arrays."""
    topo = level.topo
    d = level.d
    interiors = []
    groups = {}
    order = []
    for k in range(topo.K):
        I = level.idx[k]
        n = level.n[k]
        off = level.offsets[k]
        inner = np.all((I >= 1) & (I <= n - 2), axis=1)
        comp = level.comp_of_torn[off + np.nonzero(inner)[0]]
        assert np.all(comp >= 0)
        interiors.append((comp, tuple(int(m) for m in (n - 2)[::-1])))
        for loc in np.nonzero(~inner)[0]:
            c = level.comp_of_torn[off + loc]
            if c < 0:
                continue
            fixed = {}
            for delta in range(d):
                if I[loc, delta] == 0:
                    fixed[delta] = 0
                elif I[loc, delta] == n[delta] - 1:
                    fixed[delta] = 1
            vs = frozenset(int(topo.vid[k, b]) for b in range(2 ** d)
                           if all(((b >> dl) & 1) == s for dl, s in fixed.items()))
            if vs not in groups:
                groups[vs] = []
                order.append(vs)
            groups[vs].append(int(c))
    iface = [np.unique(np.array(groups[v], dtype=np.int64)) for v in order]
    return interiors, iface


class SCMSSmoother:
    """Additive piece smoother of eq. Ldef on one level."""

    def __init__(self, level, A, tau, delta_scal):
        self.level = level
        self.tau = tau
        topo = level.topo
        d = level.d
        self.interiors, self.iface = pieces(level)
        self.factors = []
        self.sigma = []
        self.gamma = []
        for k in range(topo.K):
            self.factors.append([SCMS1D(int(level.elems[k, g]), int(level.pk[k]))
                                 for g in range(d)])
            h = 1.0 / float(np.max(level.elems[k]))
            self.sigma.append(1.0 / (delta_scal * h * h))
            self.gamma.append(topo.measure[k] ** ((d - 2.0) / d))
        self.chol = []
        A = sp.csr_matrix(A)
        for T in self.iface:
            LT = A[T][:, T].toarray()
            self.chol.append(sla.cho_factor(LT, lower=True))
        # every compact unknown lies in exactly one piece
        cover = np.zeros(level.N, dtype=np.int64)
        for comp, _ in self.interiors:
            cover[comp] += 1
        for T in self.iface:
            cover[T] += 1
        assert np.all(cover == 1)

    def apply(self, r):
        """y = L^-1 r = tau sum_T P_T L_T^-1 P_T^T r."""
        y = np.zeros_like(r)
        for k, (comp, shape) in enumerate(self.interiors):
            y[comp] += scms_interior_apply(self.factors[k], self.sigma[k], self.gamma[k],
                                           r[comp].reshape(shape)).ravel()
        for T, c in zip(self.iface, self.chol):
            y[T] += sla.cho_solve(c, r[T])
        return self.tau * y


# ---------------------------------------------------------------------------
# multicolour Gauss-Seidel
# ---------------------------------------------------------------------------
def gs_color_keys(level, tile):
    """Colour key of every compact unknown, taken at its first copy (patch k,
    index i in k): key = ((c_k * 2^d + pi) * (p+1)^d + s) with c_k the patch
    colour, pi = sum_d (floor(i_d / tile) mod 2) 2^d the tile parity and
    s = sum_d (i_d mod (p+1)) (p+1)^d the position inside the (p+1)^d block.

    SIPG space (one copy per unknown): c_k colours the face-adjacency graph.
    Two unknowns of equal key are never coupled: inside a patch they differ
    by a multiple of p+1 >= p+1 in some index, across patches equal colour
    means no common interface.

    Conforming space: c_k colours the vertex-sharing graph (a glued unknown
    couples the patches around its vertex or edge).  Equal keys again mean no
    coupling: two unknowns first seen in the same patch differ by >= p+1 in
    some index of that patch, and a patch holding copies of both sees the
    same distance along the side it shares with it; unknowns first seen in
    different patches of one colour lie in patches without a common corner,
    and a third patch holding copies of both would hold them on two of its
    sides without a common corner, at least n_el + p - 1 >= p + 1 apart
    (n_el >= 2 on every smoothed level).

    tile >= p keeps tiles of equal parity uncoupled as well.  With a degree
    per patch the tile (None: 2(p+1)) and the positions (i mod (p+1)) are
    those of the largest degree p on every patch: two unknowns of equal key
    still differ by at least p+1 >= p_k+1 in some index, beyond the coupling
    range p_k of their patch."""
    topo = level.topo
    d = level.d
    pm = level.p
    color = topo.vertex_color if level.conforming else topo.patch_color
    keys = np.zeros(level.N, dtype=np.int64)
    for t in range(level.N_torn):
        c = level.comp_of_torn[t]
        if c < 0 or level.rep_torn[c] != t:
            continue
        k = int(np.searchsorted(level.offsets, t, side="right") - 1)
        tk = 2 * (pm + 1) if tile is None else tile
        assert tk >= pm
        i = level.idx[k][t - level.offsets[k]]
        par = sum(((int(i[g]) // tk) % 2) << g for g in range(d))
        sub = sum((int(i[g]) % (pm + 1)) * (pm + 1) ** g for g in range(d))
        keys[c] = (color[k] * 2 ** d + par) * (pm + 1) ** d + sub
    return keys


class GaussSeidel:
    """Forward / backward Gauss-Seidel sweeps in the multicolour ordering."""

    def __init__(self, A, keys):
        self.A = sp.csr_matrix(A)
        self.keys = keys
        self.diag = self.A.diagonal()
        ukeys = np.unique(keys)
        self.groups = [np.nonzero(keys == k)[0] for k in ukeys]
        self.rows = [self.A[g] for g in self.groups]

    def forward(self, f, u):
        u = u.copy()
        for g, R in zip(self.groups, self.rows):
            u[g] += (f[g] - R @ u) / self.diag[g]
        return u

    def backward(self, f, u):
        u = u.copy()
        for g, R in zip(self.groups[::-1], self.rows[::-1]):
            u[g] += (f[g] - R @ u) / self.diag[g]
        return u
