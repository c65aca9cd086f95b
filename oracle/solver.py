"""Multigrid cycle and outer iterations of the oracle.

* Algorithm 1 (V-cycle mu = 1 / W-cycle mu = 2, nu pre- and post-smoothing
  steps, direct solver on level 0, prolongation = canonical embedding,
  restriction = its transpose), used with the Gauss-Seidel and the subspace
  corrected mass smoother (Sections 4, 5);
* Algorithm 2 (hybrid smoother: forward Gauss-Seidel then nu SCMS steps
  before the coarse-grid correction, nu SCMS steps then backward Gauss-Seidel
  after it, Section 6);
* the multigrid method used directly as a solver or as preconditioner in
  conjugate gradients, stopped at ||A u - f|| / ||f|| <= eps (Section 4).

Oracle code: test infrastructure only.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .discretize import Topology, Level, penalty
from .hierarchy import level_elements, prolongation
from .smoothers import SCMSSmoother, GaussSeidel, gs_color_keys
from . import bspline
from .geometry import multilinear


class OracleProblem:
    """Hierarchy, matrices and smoothers of one problem instance."""

    def __init__(self, corners, elems, p, sigma=5.0, conforming=False,
                 smoother="hybrid", tau=0.25, delta=0.1, gs_tile=None,
                 mu=1, nu=1, coarse_min=2):
        corners = np.asarray(corners, dtype=np.float64)
        self.topo = Topology(corners)
        K, d = self.topo.K, self.topo.d
        elems = np.asarray(elems, dtype=np.int64).reshape(K, d)
        # p: one degree, or a degree per patch (non-matching spaces of Section 5)
        self.pk = np.broadcast_to(np.asarray(p, dtype=np.int64), (K,)).copy()
        self.p, self.d = int(self.pk.max()), d
        self.conforming = conforming
        self.smoother = smoother
        self.mu, self.nu = mu, nu
        self.tau, self.delta = tau, delta
        if gs_tile is None:
            gs_tile = 2 * (self.p + 1)  # the largest degree's on every patch
        self.gs_tile = gs_tile
        self.eta = None if conforming else penalty(self.topo, elems, self.pk, sigma)
        self.level_elems = level_elements(elems, coarse_min)
        self.levels = [Level(self.topo, e, self.pk, conforming, self.eta)
                       for e in self.level_elems]
        self.A = [lev.assemble() for lev in self.levels]
        self.P = [None] + [prolongation(self.levels[l - 1], self.levels[l])
                           for l in range(1, len(self.levels))]
        self.coarse = sla.cho_factor(self.A[0].toarray(), lower=True)
        self.scms = [None] + [SCMSSmoother(self.levels[l], self.A[l], tau, delta)
                              if smoother in ("scms", "hybrid") else None
                              for l in range(1, len(self.levels))]
        self.gs = [None] + [GaussSeidel(self.A[l], gs_color_keys(self.levels[l], self.gs_tile))
                            if smoother in ("gs", "hybrid") else None
                            for l in range(1, len(self.levels))]

    # -- basic operations ----------------------------------------------------
    @property
    def N(self):
        return self.levels[-1].N

    @property
    def L(self):
        return len(self.levels) - 1

    def apply(self, x):
        return self.A[-1] @ x

    def coarse_solve(self, r):
        return sla.cho_solve(self.coarse, r)

    def _pre(self, l, f, u):
        A = self.A[l]
        if self.smoother == "gs":
            for _ in range(self.nu):
                u = self.gs[l].forward(f, u)
            return u
        if self.smoother == "hybrid":
            u = self.gs[l].forward(f, u)
        for _ in range(self.nu):
            u = u + self.scms[l].apply(f - A @ u)
        return u

    def _post(self, l, f, u):
        A = self.A[l]
        if self.smoother == "gs":
            for _ in range(self.nu):
                u = self.gs[l].backward(f, u)
            return u
        for _ in range(self.nu):
            u = u + self.scms[l].apply(f - A @ u)
        if self.smoother == "hybrid":
            u = self.gs[l].backward(f, u)
        return u

    def mg(self, l, f, u):
        """Algorithm 1 / Algorithm 2 on level l >= 1 (level 0: direct solve)."""
        if l == 0:
            return self.coarse_solve(f)
        A = self.A[l]
        u = self._pre(l, f, u)
        reps = 1 if l == 1 else self.mu
        for _ in range(reps):
            rc = self.P[l].T @ (f - A @ u)
            if l == 1:
                e = self.coarse_solve(rc)
            else:
                e = self.mg(l - 1, rc, np.zeros(self.levels[l - 1].N))
            u = u + self.P[l] @ e
        return self._post(l, f, u)

    def vcycle(self, f, u=None):
        u = np.zeros(self.N) if u is None else u
        return self.mg(self.L, f, u)

    # -- outer iterations ------------------------------------------------------
    def pcg(self, f, tol=1e-8, maxit=500):
        """Conjugate gradients preconditioned with one cycle, zero initial
        guess, stopped when ||r_k|| / ||f|| <= tol with the recursively updated
        residual r_k (= f - A u_k in exact arithmetic).
        Returns (u, iterations, residual history, iterates)."""
        A = self.A[-1]
        nf = np.linalg.norm(f)
        x = np.zeros_like(f)
        r = f.copy()
        hist = [1.0 if nf > 0 else 0.0]
        iterates = []
        if nf == 0:
            return x, 0, hist, iterates
        z = self.vcycle(r)
        pdir = z.copy()
        rz = r @ z
        it = 0
        for it in range(1, maxit + 1):
            q = A @ pdir
            alpha = rz / (pdir @ q)
            x = x + alpha * pdir
            r = r - alpha * q
            res = np.linalg.norm(r) / nf
            hist.append(res)
            iterates.append(x.copy())
            if res <= tol:
                break
            z = self.vcycle(r)
            rz_new = r @ z
            beta = rz_new / rz
            rz = rz_new
            pdir = z + beta * pdir
        return x, it, hist, iterates

    def mg_iteration(self, f, tol=1e-8, maxit=500):
        """Multigrid used directly as solver: u <- MG(L, f, u)."""
        A = self.A[-1]
        nf = np.linalg.norm(f)
        u = np.zeros_like(f)
        hist = [1.0]
        it = 0
        for it in range(1, maxit + 1):
            u = self.mg(self.L, f, u)
            res = np.linalg.norm(f - A @ u) / nf
            hist.append(res)
            if res <= tol:
                break
        return u, it, hist

    # -- manufactured solution (Section 2: g = prod sin(pi x)) ----------------
    def load_manufactured(self):
        d = self.d

        def f(X):
            return d * np.pi ** 2 * np.prod(np.sin(np.pi * X), axis=1)
        return self.levels[-1].load(f)

    def l2_error(self, u):
        """||u_h - prod sin(pi x)||_{L2} with q = p+3 Gauss points per element
        and direction on every patch (p = the largest degree)."""
        lev = self.levels[-1]
        ut = lev.to_torn(u)
        err2 = 0.0
        q = self.p + 3
        for k in range(self.topo.K):
            C0, _, W, xh = lev.patch_collocation(k, q)
            X, J = multilinear(self.topo.corners[k], xh)
            uh = C0 @ ut[lev.offsets[k]:lev.offsets[k + 1]]
            ex = np.prod(np.sin(np.pi * X), axis=1)
            err2 += np.sum(W * np.abs(np.linalg.det(J)) * (uh - ex) ** 2)
        return float(np.sqrt(err2))


def setup(corners, elems, p, sigma=5.0, **opts):
    return OracleProblem(corners, elems, p, sigma=sigma, **opts)
