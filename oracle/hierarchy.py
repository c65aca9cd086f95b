"""Grid hierarchy and intergrid transfer (Section 4: nested spaces,
I_{l-1}^l is the canonical embedding, the restriction is its transpose).

The 1D embedding is obtained by Boehm's knot insertion: inserting a knot
t* into span [t_m, t_{m+1}) replaces the coefficients c_i by
alpha_i c_i + (1 - alpha_i) c_{i-1}, alpha_i = (t* - t_i)/(t_{i+p} - t_i)
for m-p < i <= m (1 below, 0 above).  Oracle code: test infrastructure only.
"""
import numpy as np
import scipy.sparse as sp

from . import bspline
from .discretize import kron_dirs


def level_elements(elems_fine, coarse_min=2):
    """Element counts per level, coarsest first.  Halve all counts while every
    count is even and its half is at least coarse_min (uniform refinement,
    Section 2 below eq. local)."""
    e = np.asarray(elems_fine, dtype=np.int64)
    levels = [e.copy()]
    while np.all(e % 2 == 0) and np.all(e // 2 >= coarse_min):
        e = e // 2
        levels.append(e.copy())
    return levels[::-1]


def insert_knot(knots, p, t):
    """Matrix R with c_new = R c_old for the insertion of knot t (Boehm)."""
    n = len(knots) - 1 - p
    m = np.searchsorted(knots, t, side="right") - 1  # t in [t_m, t_{m+1})
    R = np.zeros((n + 1, n))
    for i in range(n + 1):
        if i <= m - p:
            if i < n:
                R[i, i] = 1.0
        elif i > m:
            R[i, i - 1] = 1.0
        else:
            a = (t - knots[i]) / (knots[i + p] - knots[i])
            if i < n:
                R[i, i] = a
            R[i, i - 1] = 1.0 - a
    new = np.sort(np.concatenate([knots, [t]]))
    return R, new


def prolongation_1d(n_el_coarse, p):
    """Embedding of S_{p,1/n} into S_{p,1/(2n)} as a dense (n_f x n_c) matrix."""
    knots = bspline.open_uniform_knots(n_el_coarse, p)
    P = np.eye(n_el_coarse + p)
    for e in range(n_el_coarse):
        t = (2 * e + 1) / (2.0 * n_el_coarse)
        R, knots = insert_knot(knots, p, t)
        P = R @ P
    ref = bspline.open_uniform_knots(2 * n_el_coarse, p)
    assert np.allclose(knots, ref)
    return P


def prolongation(level_c, level_f):
    """I_{l-1}^l in compact numbering: per patch the Kronecker product of the
    1D embeddings, the fine row of a glued DOF taken from its first copy."""
    blocks = []
    for k in range(level_c.topo.K):
        mats = []
        for delta in range(level_c.d):
            nc = int(level_c.elems[k, delta])
            assert int(level_f.elems[k, delta]) == 2 * nc
            mats.append(sp.csr_matrix(prolongation_1d(nc, int(level_c.pk[k]))))
        blocks.append(kron_dirs(mats))
    Pt = sp.block_diag(blocks, format="csr")
    P = (level_f.S @ Pt @ level_c.E).tocsr()
    P.eliminate_zeros()
    return P
