"""Discretization of the Poisson model problem on a multi-patch domain.

* conforming Galerkin space V^c (Section 2, eq. igaspace0 and the linear
  system eq. linear:system:0), interface DOFs glued by their Greville points
  as in Figure dof;
* SIPG space V^n (Section 3, eq. igaspace) with the bilinear form
  eq. model:discr2: (u,v)_A = (u,v)_K + sigma p^2/h (u,v)_J - (u,v)_B - (v,u)_B,
  penalty taken from the finest grid on every level (eq. a:galerkin);
* Dirichlet conditions imposed strongly: every basis function with a
  non-vanishing trace on the boundary is removed (Section 3, below eq.
  igaspace).

Matrices are written exactly as their definitions: with collocation
matrices C (basis functions or their parameter derivatives at all quadrature
points) the stiffness matrix is sum_ab C_a^T diag(w |det J| (J^-1 J^-T)_ab) C_b,
and interface terms are built from trace / normal-derivative collocation.
Oracle code: test infrastructure only.
"""
import itertools

import numpy as np
import scipy.sparse as sp

from . import bspline
from .geometry import corner_bits, multilinear, tensor_points, tensor_weights, patch_measure


# ---------------------------------------------------------------------------
# topology: shared vertices, interfaces, boundary sides (Assumption 1)
# ---------------------------------------------------------------------------
class Topology:
    """Vertex identification, interfaces and boundary sides of the patch
    decomposition (Section 2, eq. omega:1 and Assumption 1)."""

    def __init__(self, corners, tol=1e-9):
        corners = np.asarray(corners, dtype=np.float64)
        self.K, nc, self.d = corners.shape
        assert nc == 2 ** self.d
        self.corners = corners
        d = self.d
        keys = {}
        self.vid = np.zeros((self.K, nc), dtype=np.int64)
        for k in range(self.K):
            for b in range(nc):
                key = tuple(np.round(corners[k, b] / tol).astype(np.int64))
                if key not in keys:
                    keys[key] = len(keys)
                self.vid[k, b] = keys[key]
        self.n_vertices = len(keys)
        bits = corner_bits(d)
        # corners of side (delta, s), ordered by the remaining (tangential) bits
        self.side_corners = {}
        for delta in range(d):
            tang = [g for g in range(d) if g != delta]
            for s in (0, 1):
                lst = []
                for tb in range(2 ** (d - 1)):
                    b = s << delta
                    for j, g in enumerate(tang):
                        b |= ((tb >> j) & 1) << g
                    lst.append(b)
                self.side_corners[(delta, s)] = lst
        self.interfaces = []  # (k, dk, sk, l, dl, sl), k < l
        used = set()
        for k in range(self.K):
            for l in range(k + 1, self.K):
                for (dk, sk), ck in self.side_corners.items():
                    vk = [self.vid[k, b] for b in ck]
                    for (dl, sl), cl in self.side_corners.items():
                        vl = [self.vid[l, b] for b in cl]
                        if set(vk) == set(vl):
                            if vk != vl:
                                raise NotImplementedError(
                                    "interface with flipped orientation")
                            self.interfaces.append((k, dk, sk, l, dl, sl))
                            used.add((k, dk, sk))
                            used.add((l, dl, sl))
        self.boundary_sides = set()
        for k in range(self.K):
            for delta in range(d):
                for s in (0, 1):
                    if (k, delta, s) not in used:
                        self.boundary_sides.add((k, delta, s))
        # greedy first-fit colouring of the face-adjacency graph in patch order
        nbr = [set() for _ in range(self.K)]
        for (k, _, _, l, _, _) in self.interfaces:
            nbr[k].add(l)
            nbr[l].add(k)
        self.neighbours = nbr
        self.patch_color = []
        for k in range(self.K):
            taken = {self.patch_color[j] for j in nbr[k] if j < k}
            c = 0
            while c in taken:
                c += 1
            self.patch_color.append(c)
        # greedy first-fit colouring of the vertex-sharing graph in patch order:
        # patches with a common corner get different colours (the conforming
        # Gauss-Seidel ordering, where a glued unknown couples every patch
        # around its vertex or edge)
        vset = [set(int(v) for v in self.vid[k]) for k in range(self.K)]
        self.vertex_color = []
        for k in range(self.K):
            taken = {self.vertex_color[j] for j in range(k) if vset[j] & vset[k]}
            c = 0
            while c in taken:
                c += 1
            self.vertex_color.append(c)
        self.measure = np.array([patch_measure(corners[k]) for k in range(self.K)])


# ---------------------------------------------------------------------------
# per-direction collocation tables
# ---------------------------------------------------------------------------
def collocation_1d(n_el, p, pts, deriv):
    knots = bspline.open_uniform_knots(n_el, p)
    if deriv == 0:
        M = bspline.basis_table(knots, p, pts)[-1]
    else:
        M = bspline.basis_derivative(knots, p, pts, deriv)
    M[np.abs(M) < 1e-300] = 0.0
    return sp.csr_matrix(M)


def kron_dirs(mats):
    """Kronecker product over directions, mats[0] = x (fastest index)."""
    out = mats[-1]
    for m in mats[-2::-1]:
        out = sp.kron(out, m, format="csr")
    return sp.csr_matrix(out)


def merged_breakpoints(na, nb):
    """Union of the breakpoints i/na and j/nb, written as m/lcm(na, nb)."""
    L = int(np.lcm(na, nb))
    m = np.union1d(np.arange(na + 1) * (L // na), np.arange(nb + 1) * (L // nb))
    return m.astype(np.float64) / L


# ---------------------------------------------------------------------------
# one grid level
# ---------------------------------------------------------------------------
class Level:
    """DOF bookkeeping and the assembled system of one grid level.

    Torn ordering: all patch-local B-spline coefficients, patch after patch,
    lexicographic with x fastest (Dirichlet ones included).  Compact ordering
    (the unknowns of eq. linear:system / linear:system:0): the torn ordering
    with Dirichlet DOFs skipped; in the conforming case a glued DOF keeps the
    index of its first visit.
    """

    def __init__(self, topo, elems, p, conforming, eta=None):
        self.topo = topo
        self.d = topo.d
        # degree per patch (an int: the same on every patch); p = the largest
        self.pk = np.broadcast_to(np.asarray(p, dtype=np.int64), (topo.K,)).copy()
        self.p = int(self.pk.max())
        self.conforming = conforming
        self.elems = np.asarray(elems, dtype=np.int64).reshape(topo.K, topo.d)
        self.n = self.elems + self.pk[:, None]
        self.sizes = np.prod(self.n, axis=1)
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)])
        self.N_torn = int(self.offsets[-1])
        self.eta = eta
        self._dofs()
        self._numbering()

    # -- DOF sets ----------------------------------------------------------
    def multi_index(self, k):
        n = self.n[k]
        grids = np.meshgrid(*[np.arange(m) for m in n[::-1]], indexing="ij")
        return np.stack([g.ravel() for g in grids[::-1]], axis=1)  # x fastest

    def _dofs(self):
        topo = self.topo
        dirich = np.zeros(self.N_torn, dtype=bool)
        self.idx = []
        for k in range(topo.K):
            I = self.multi_index(k)
            self.idx.append(I)
            sl = slice(self.offsets[k], self.offsets[k + 1])
            mask = np.zeros(len(I), dtype=bool)
            for (kk, delta, s) in topo.boundary_sides:
                if kk != k:
                    continue
                ext = 0 if s == 0 else self.n[k, delta] - 1
                mask |= I[:, delta] == ext
            dirich[sl] = mask
        self.dirichlet_torn = dirich

    def _greville_points(self, k):
        d = self.d
        axes = []
        pk = int(self.pk[k])
        for delta in range(d):
            kn = bspline.open_uniform_knots(int(self.elems[k, delta]), pk)
            axes.append(bspline.greville(kn, pk))
        pts = tensor_points(axes)
        X, _ = multilinear(self.topo.corners[k], pts)
        return X

    def _numbering(self):
        topo = self.topo
        K = topo.K
        group = -np.ones(self.N_torn, dtype=np.int64)
        if self.conforming:
            # glue patch-boundary DOFs with coinciding Greville points (Fig. dof)
            table = {}
            gid = 0
            for k in range(K):
                I = self.idx[k]
                on_bd = np.zeros(len(I), dtype=bool)
                for delta in range(self.d):
                    on_bd |= (I[:, delta] == 0) | (I[:, delta] == self.n[k, delta] - 1)
                X = self._greville_points(k)
                for loc in np.nonzero(on_bd)[0]:
                    key = tuple(np.round(X[loc] * 1e9).astype(np.int64))
                    if key not in table:
                        table[key] = gid
                        gid += 1
                    group[self.offsets[k] + loc] = table[key]
            # a glued DOF is Dirichlet if one of its copies is
            ng = gid
            gd = np.zeros(ng, dtype=bool)
            sel = group >= 0
            np.logical_or.at(gd, group[sel], self.dirichlet_torn[sel])
            self.dirichlet_torn[sel] = gd[group[sel]]
            # Assumption 2: the two sides of every interface carry equally many DOFs
            for (k, dk, sk, l, dl, sl_) in topo.interfaces:
                ik = self.idx[k]
                il = self.idx[l]
                ek = 0 if sk == 0 else self.n[k, dk] - 1
                el = 0 if sl_ == 0 else self.n[l, dl] - 1
                gk = set(group[self.offsets[k] + np.nonzero(ik[:, dk] == ek)[0]])
                gl = set(group[self.offsets[l] + np.nonzero(il[:, dl] == el)[0]])
                if gk != gl:
                    raise ValueError("conforming discretization needs fully matching "
                                     "interfaces (Assumption 2)")
        comp = -np.ones(self.N_torn, dtype=np.int64)
        rep = []
        gmap = {}
        for t in range(self.N_torn):
            if self.dirichlet_torn[t]:
                continue
            g = group[t]
            if g >= 0 and g in gmap:
                comp[t] = gmap[g]
                continue
            comp[t] = len(rep)
            rep.append(t)
            if g >= 0:
                gmap[g] = comp[t]
        self.group = group
        self.comp_of_torn = comp
        self.rep_torn = np.array(rep, dtype=np.int64)
        self.N = len(rep)
        rows = np.nonzero(comp >= 0)[0]
        self.E = sp.csr_matrix((np.ones(len(rows)), (rows, comp[rows])),
                               shape=(self.N_torn, self.N))
        self.S = sp.csr_matrix((np.ones(self.N), (np.arange(self.N), self.rep_torn)),
                               shape=(self.N, self.N_torn))

    # -- quadrature on the whole patch -------------------------------------
    def patch_collocation(self, k, q):
        """Collocation matrices C[g] of d/dxh_g (g=0..d-1) and C0 of values at
        all q-point Gauss points of patch k, plus weights and parameter points."""
        d = self.d
        pts1, wts1, B1, D1 = [], [], [], []
        for delta in range(d):
            ne = int(self.elems[k, delta])
            x, w = bspline.element_quadrature(ne, q)
            pts1.append(x)
            wts1.append(w)
            B1.append(collocation_1d(ne, int(self.pk[k]), x, 0))
            D1.append(collocation_1d(ne, int(self.pk[k]), x, 1))
        C0 = kron_dirs(B1)
        Cg = []
        for g in range(d):
            Cg.append(kron_dirs([D1[delta] if delta == g else B1[delta] for delta in range(d)]))
        return C0, Cg, tensor_weights(wts1), tensor_points(pts1)

    def volume_matrix(self, k):
        """Patch stiffness (grad u, grad v)_{L2(Omega_k)} with q = p+1 Gauss
        points per element and direction (Section 2, eq. model), p = the
        patch's degree."""
        C0, Cg, W, xh = self.patch_collocation(k, int(self.pk[k]) + 1)
        _, J = multilinear(self.topo.corners[k], xh)
        detJ = np.linalg.det(J)
        if np.any(detJ <= 0):
            raise ValueError("geometry map is not orientation preserving")
        Jinv = np.linalg.inv(J)
        G = np.einsum("qai,qbi->qab", Jinv, Jinv) * (W * detJ)[:, None, None]
        A = sp.csr_matrix((self.sizes[k], self.sizes[k]))
        for a in range(self.d):
            for b in range(self.d):
                A = A + Cg[a].T @ sp.diags(G[:, a, b]) @ Cg[b]
        return sp.csr_matrix(A)

    def volume_row(self, k, i):
        """Row of patch k's stiffness matrix (volume_matrix) for the basis
        function with multi-index i (x first), integrated with the same Gauss
        rule over the elements of its support only (elsewhere the row's
        integrand vanishes).  Returns the row as a dense vector over the
        patch's local unknowns.  Used to check single outputs of the operator
        at sizes whose full assembly is out of reach."""
        d, p = self.d, int(self.pk[k])
        q = p + 1
        pts1, wts1, B1, D1 = [], [], [], []
        for delta in range(d):
            ne = int(self.elems[k, delta])
            x, w = bspline.element_quadrature(ne, q)
            els = np.arange(max(0, int(i[delta]) - p), min(ne - 1, int(i[delta])) + 1)
            sel = (els[:, None] * q + np.arange(q)[None, :]).ravel()
            pts1.append(x[sel])
            wts1.append(w[sel])
            B1.append(collocation_1d(ne, p, x[sel], 0))
            D1.append(collocation_1d(ne, p, x[sel], 1))
        Cg = [kron_dirs([D1[delta] if delta == g else B1[delta] for delta in range(d)])
              for g in range(d)]
        W = tensor_weights(wts1)
        _, J = multilinear(self.topo.corners[k], tensor_points(pts1))
        detJ = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        G = np.einsum("qai,qbi->qab", Jinv, Jinv) * (W * detJ)[:, None, None]
        li = 0
        for delta in range(d - 1, -1, -1):
            li = li * int(self.n[k, delta]) + int(i[delta])
        row = np.zeros(int(self.sizes[k]))
        for a in range(d):
            ca = Cg[a][:, li].toarray().ravel()
            for b in range(d):
                row += Cg[b].T @ (ca * G[:, a, b])
        return row

    def load_vector(self, k, f):
        """(f, phi_i)_{L2(Omega_k)} with q = p+1 Gauss points."""
        C0, _, W, xh = self.patch_collocation(k, int(self.pk[k]) + 1)
        X, J = multilinear(self.topo.corners[k], xh)
        detJ = np.abs(np.linalg.det(J))
        return C0.T @ (W * detJ * f(X))

    # -- SIPG interface terms ----------------------------------------------
    def side_collocation(self, k, delta, s, tang, tpts):
        """Values and parameter gradients of patch k's basis at points of side
        (delta, s); tang = tangential directions, tpts = their 1D point arrays."""
        d = self.d
        val1, der1 = [], []
        for g in range(d):
            ne = int(self.elems[k, g])
            if g == delta:
                x = np.array([float(s)])
            else:
                x = tpts[tang.index(g)]
            val1.append(collocation_1d(ne, int(self.pk[k]), x, 0))
            der1.append(collocation_1d(ne, int(self.pk[k]), x, 1))
        V = kron_dirs(val1)
        Gr = [kron_dirs([der1[h] if h == g else val1[h] for h in range(d)]) for g in range(d)]
        xh_axes = []
        for g in range(d):
            xh_axes.append(np.array([float(s)]) if g == delta else tpts[tang.index(g)])
        return V, Gr, tensor_points(xh_axes)

    def interface_matrix(self):
        """sum over interfaces of eta([u],[v]) - ([u],{grad v}.n) - ([v],{grad u}.n)
        (eq. model:discr2) in torn numbering.  Quadrature: q = p+1 Gauss points
        (p = the larger of the two sides' degrees) on every segment of the
        union of both sides' breakpoints."""
        topo = self.topo
        d = self.d
        rows, cols, vals = [], [], []
        for (k, dk, sk, l, dl, sl_) in topo.interfaces:
            q = int(max(self.pk[k], self.pk[l])) + 1
            tk = [g for g in range(d) if g != dk]
            tl = [g for g in range(d) if g != dl]
            tpts_k, tw = [], []
            for j in range(d - 1):
                br = merged_breakpoints(int(self.elems[k, tk[j]]), int(self.elems[l, tl[j]]))
                xi, w = bspline.gauss_legendre(q)
                a = br[:-1, None]
                h = (br[1:] - br[:-1])[:, None]
                tpts_k.append((a + h * xi[None, :]).ravel())
                tw.append((h * w[None, :]).ravel())
            Vk, Gk, xk = self.side_collocation(k, dk, sk, tk, tpts_k)
            Vl, Gl, xl = self.side_collocation(l, dl, sl_, tl, tpts_k)
            Xk, Jk = multilinear(topo.corners[k], xk)
            Xl, Jl = multilinear(topo.corners[l], xl)
            assert np.allclose(Xk, Xl, atol=1e-12), "interface parametrizations differ"
            Wt = tensor_weights(tw)
            # surface element of side k
            tv = [Jk[:, :, g] for g in tk]
            if d == 2:
                ds = np.linalg.norm(tv[0], axis=1)
            else:
                ds = np.linalg.norm(np.cross(tv[0], tv[1]), axis=1)
            # outer unit normal of Omega_k
            e = np.zeros(d)
            e[dk] = 1.0 if sk == 1 else -1.0
            JkinvT = np.transpose(np.linalg.inv(Jk), (0, 2, 1))
            nrm = JkinvT @ e
            nrm /= np.linalg.norm(nrm, axis=1)[:, None]
            # normal derivatives: grad phi . n = grad_hat phi . (J^-1 n)
            ck = np.einsum("qab,qb->qa", np.linalg.inv(Jk), nrm)
            cl = np.einsum("qab,qb->qa", np.linalg.inv(Jl), nrm)
            Nk = sum(sp.diags(ck[:, g]) @ Gk[g] for g in range(d))
            Nl = sum(sp.diags(cl[:, g]) @ Gl[g] for g in range(d))
            nk, nl = self.sizes[k], self.sizes[l]
            Jmp = sp.hstack([Vk, -Vl]).tocsr()
            Avg = 0.5 * sp.hstack([Nk, Nl]).tocsr()
            Wd = sp.diags(Wt * ds)
            M = (self.eta[(k, l)] * (Jmp.T @ Wd @ Jmp) - Avg.T @ Wd @ Jmp - Jmp.T @ Wd @ Avg).tocoo()
            idx = np.concatenate([np.arange(nk) + self.offsets[k], np.arange(nl) + self.offsets[l]])
            rows.append(idx[M.row])
            cols.append(idx[M.col])
            vals.append(M.data)
        if not rows:
            return sp.csr_matrix((self.N_torn, self.N_torn))
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.N_torn, self.N_torn))

    # -- assembled system ----------------------------------------------------
    def assemble(self):
        blocks = [self.volume_matrix(k) for k in range(self.topo.K)]
        At = sp.block_diag(blocks, format="csr")
        if not self.conforming:
            At = At + self.interface_matrix()
        self.A_torn = sp.csr_matrix(At)
        A = (self.E.T @ At @ self.E).tocsr()
        A.sum_duplicates()
        A.eliminate_zeros()
        self.A = A
        return A

    def load(self, f):
        bt = np.concatenate([self.load_vector(k, f) for k in range(self.topo.K)])
        return self.E.T @ bt

    def to_torn(self, x):
        """Compact vector -> torn vector (copies filled, Dirichlet zero)."""
        return self.E @ x


def penalty(topo, elems_fine, p, sigma):
    """eta_kl = sigma p^2 / h_kl per interface, h from the finest grid on every
    level (Section 3, eq. a:galerkin).  h_kl = min(h_k, h_l) with the physical
    element size h_s = |Omega_s|^(1/d) / max_delta n_el(s, delta); with a
    degree per patch, p = max(p_k, p_l)."""
    d = topo.d
    pk = np.broadcast_to(np.asarray(p, dtype=np.int64), (topo.K,))
    h = topo.measure ** (1.0 / d) / np.max(np.asarray(elems_fine).reshape(topo.K, d), axis=1)
    etas = {}
    for (k, dk, sk, l, dl, sl) in topo.interfaces:
        pkl = float(max(pk[k], pk[l]))
        etas[(k, l)] = sigma * pkl * pkl / min(h[k], h[l])
    return etas
