"""The subspace corrected mass smoother of Section 5 against what the paper
fixes about it, on the paper's L-shaped domain (three unit squares, one
element per patch on level 0, conforming space, damping tau, scaling delta):

* a closed form: for p = 2 the spline space has no outlier subspace, the
  patch-interior smoother is sigma M (x) M with sigma = 1/(delta h^2), and
  the highest-frequency symbol of the quadratic B-spline mass and stiffness
  matrices, (2/15) h and (4/3)/h, gives the generalized eigenvalue 10 h^-2
  per direction; the largest eigenvalue of L^-1 A (tau = 1) therefore tends
  to 2 x 10 delta = 20 delta;
* the appendix Lemma smp1: A <= L with a constant independent of h and p --
  the largest eigenvalue of tau L^-1 A stays bounded uniformly in the level
  and the degree, and A <= L holds once tau <= 1 / lambda_max;
* Table SCMS1 (golden fixture) as a trend: PCG counts flat in the level and
  falling with the degree, as printed.

Recorded here (and not parity with the paper): with this reading the largest
eigenvalue of L^-1 A at the paper's tau = 1, delta = 0.12 is 2.40, so the
lemma's inequality holds only for tau <= 0.41, the smoothing step amplifies
the highest modes at tau = 1 and the multigrid iteration itself diverges
for p = 2, 3, where the table prints 27 and 23 iterations; PCG converges in
fewer iterations than printed.  The paper defers the smoother's definition
to earlier work, so the printed counts are not reproduced.
"""
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.dirname(__file__)), "golden")


def lshape_problem(level, p, tau=1.0, delta=0.12):
    return oracle.setup(workloads.lshape_corners(), workloads.lshape_elems(level), p,
                        conforming=True, smoother="scms", tau=tau, delta=delta, coarse_min=1)


def smoother_spectrum(pb, level=None):
    """Eigenvalues of L^-1 A on a level (dense; the smoother applied to the
    columns of A)."""
    l = pb.L if level is None else level
    A = pb.A[l].toarray()
    S = np.stack([pb.scms[l].apply(A[:, j]) for j in range(A.shape[0])], axis=1)
    return np.sort(np.linalg.eigvals(S).real)


def test_lshape_sizes_and_levels():
    """Three unit squares glued along two edges, the re-entrant corner at
    (1, 1), one element per patch on level 0.  With n = 2^L + p functions per
    patch direction the glued coefficients form an L-shaped grid of 2n - 1
    points per direction; removing its boundary leaves (2n - 3)^2 - (n - 1)^2
    unknowns."""
    for level, p in ((4, 2), (3, 4)):
        pb = lshape_problem(level, p)
        assert len(pb.topo.interfaces) == 2
        assert [int(e[0, 0]) for e in pb.level_elems] == [2 ** l for l in range(level + 1)]
        n = 2 ** level + p
        assert pb.N == (2 * n - 3) ** 2 - (n - 1) ** 2


def test_scms_p2_highest_mode_closed_form():
    """lambda_max(L^-1 A) = 20 delta for p = 2 (closed form, see the header),
    on two levels and two scalings (pins sigma = 1/(delta h^2), h of the
    level, and the additive combination of the pieces)."""
    for level, delta in ((4, 0.12), (5, 0.12), (4, 0.2)):
        lam = smoother_spectrum(lshape_problem(level, 2, tau=1.0, delta=delta))
        assert abs(lam[-1] / (20 * delta) - 1) < 0.005, (level, delta, lam[-1])
        assert lam[0] > 0


def test_lemma_smp1_uniform_bound():
    """Lemma smp1: lambda_max(tau L^-1 A) bounded independently of h and p
    (p = 2, 3, 4 on levels 3 and 4); A <= L holds at tau = 0.4 < 1 / 2.41;
    recorded: it does not hold at the paper's tau = 1 (value above 2)."""
    lam = {}
    for p in (2, 3, 4):
        for level in (3, 4):
            lam[p, level] = smoother_spectrum(lshape_problem(level, p, tau=1.0))[-1]
    vals = np.array(list(lam.values()))
    assert vals.max() < 2.45 and vals.min() > 1.9, lam
    for p in (2, 3, 4):
        assert abs(lam[p, 4] - lam[p, 3]) < 0.3, lam
        assert 0.4 * lam[p, 4] <= 1.0
        assert lam[p, 4] > 2.0


def read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    return np.array(rows)


def test_scms1_lshape_pcg_trend():
    """Table SCMS1 (b) as a trend (tests/golden): PCG counts with the paper's
    tau = 1, delta = 0.12 on levels 4 and 5 for p = 2, 3, 4 are flat in the
    level (growth at most 3) and do not increase with the degree, as in the
    table; they stay at or below the printed counts."""
    tab = read_table("scms1_lshape_conforming.txt")   # L, (a) p=2..8, (b) p=2..8
    printed = {(int(r[0]), p): int(r[8 + p - 2]) for r in tab for p in range(2, 9)}
    its = {}
    for p in (2, 3, 4):
        for level in (4, 5):
            pb = lshape_problem(level, p)
            f = pb.load_manufactured()
            its[p, level] = pb.pcg(f)[1]
    for p in (2, 3, 4):
        assert its[p, 5] <= its[p, 4] + 3, its
        for level in (4, 5):
            assert its[p, level] <= printed[level, p], (p, level, its[p, level], printed[level, p])
    for level in (4, 5):
        assert its[2, level] >= its[3, level] >= its[4, level], its
