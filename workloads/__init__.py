"""Seeded synthetic inputs shared by the oracle tests, the HIP-path tests and
the benchmark.  This module only produces patch layouts, element counts,
option sets and random right-hand sides; it holds none of the method's
arithmetic.

Grid layouts: vertices on a regular grid of the unit square / cube, patch
(i, j[, k]) spans the 2^d surrounding vertices, corner bit order x fastest.
Perturbation: vertices are visited lexicographically (x fastest); for each
coordinate in the order x, y, z a vertex that does not lie on a boundary
plane normal to that coordinate is moved by U(-eps, eps), eps = frac * patch
width.  The domain therefore stays the unit square / cube.
"""
import numpy as np


def grid_corners(counts, frac=0.0, seed=None):
    """Patch corners of a perturbed grid layout.

    counts: patches per direction, e.g. (4, 4) or (2, 2, 2).
    Returns (K, 2^d, d) float64, patches ordered x fastest.
    """
    counts = tuple(int(c) for c in counts)
    d = len(counts)
    axes = [np.linspace(0.0, 1.0, c + 1) for c in counts]
    grids = np.meshgrid(*axes[::-1], indexing="ij")
    V = np.stack([g for g in grids[::-1]], axis=-1)  # shape (n_z+1.., n_y+1, n_x+1, d)
    if frac > 0.0:
        rng = np.random.default_rng(seed)
        shape = V.shape[:-1]
        for flat in range(int(np.prod(shape))):
            idx = np.unravel_index(flat, shape)  # last index = x fastest
            for delta in range(d):
                i_delta = idx[d - 1 - delta]
                if 0 < i_delta < counts[delta]:
                    eps = frac / counts[delta]
                    V[idx + (delta,)] += rng.uniform(-eps, eps)
    K = int(np.prod(counts))
    corners = np.zeros((K, 2 ** d, d))
    for kk in range(K):
        pidx = np.unravel_index(kk, counts[::-1])[::-1]  # (i_x, i_y, ...)
        for b in range(2 ** d):
            vidx = tuple(pidx[g] + ((b >> g) & 1) for g in range(d))
            corners[kk, b] = V[vidx[::-1]]
    return corners


def patch_indices(counts):
    counts = tuple(int(c) for c in counts)
    K = int(np.prod(counts))
    return [np.unravel_index(kk, counts[::-1])[::-1] for kk in range(K)]


def checkerboard_elems(counts, n_even, n_odd):
    """n_even elements per direction where the patch index sum is even,
    n_odd where it is odd (every interface is then non-matching)."""
    d = len(counts)
    out = []
    for pidx in patch_indices(counts):
        n = n_even if sum(int(i) for i in pidx) % 2 == 0 else n_odd
        out.append([n] * d)
    return np.array(out, dtype=np.int64)


def lshape_corners():
    """The paper's L-shaped domain of three unit squares (Section 2: identity
    and translations as geometry maps): (0,1)^2, (1,2) x (0,1), (0,1) x (1,2),
    corner bit order x fastest."""
    def square(x0, y0):
        return [[x0, y0], [x0 + 1, y0], [x0, y0 + 1], [x0 + 1, y0 + 1]]
    return np.array([square(0, 0), square(1, 0), square(0, 1)], dtype=np.float64)


def lshape_elems(level, degrees=None):
    """Element counts of the L-shape after `level` uniform refinements of one
    element per patch: 2^level per direction."""
    return np.full((3, 2), 2 ** int(level), dtype=np.int64)


def nonmatching_spaces(elems_fine, p):
    """The non-matching spaces of the paper's SIPG experiments (Section 5):
    of every three patches (in patch order) the first keeps S_{p,h}, the
    second takes S_{p+1,2h}, the third S_{p,2h}.  Returns (element counts,
    degree per patch) from the element counts of S_{p,h} (even counts)."""
    e = np.asarray(elems_fine, dtype=np.int64).copy()
    deg = np.full(e.shape[0], int(p), dtype=np.int64)
    for k in range(e.shape[0]):
        if k % 3 == 1:
            e[k] //= 2
            deg[k] = p + 1
        elif k % 3 == 2:
            e[k] //= 2
    return e, deg


def fichera_corners():
    """The Fichera corner: the cube (0,2)^3 without the octant (1,2)^3, as
    seven axis-aligned unit cubes (identity and translations as geometry
    maps), listed with x fastest, then y, then z; corner bit order x
    fastest."""
    cubes = []
    for kz in range(2):
        for ky in range(2):
            for kx in range(2):
                if kx == 1 and ky == 1 and kz == 1:
                    continue
                cubes.append([[kx + (b & 1), ky + ((b >> 1) & 1), kz + ((b >> 2) & 1)]
                              for b in range(8)])
    return np.array(cubes, dtype=np.float64)


def fichera_elems(level):
    """Element counts of the Fichera corner after `level` uniform refinements
    of one element per patch: 2^level per direction."""
    return np.full((7, 3), 2 ** int(level), dtype=np.int64)


def normal_rhs(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


# ---------------------------------------------------------------------------
# the benchmark configurations
# ---------------------------------------------------------------------------
def config(name, scale=1):
    """Problem description of a named configuration.

    scale divides every element count (must keep them integral), giving
    reduced problems with the same structure for fast oracle runs.
    Keys: corners, elems, p, sigma, conforming, smoother, tau, delta,
    rhs ('manufactured' or ('normal', seed)), outer, precision.
    """
    if name == "c1":
        # 2x2 identity-mapped patches, conforming, p=2, 16 elements, SCMS V(1,1)
        corners = grid_corners((2, 2))
        elems = np.full((4, 2), 16 // scale, dtype=np.int64)
        return dict(corners=corners, elems=elems, p=2, sigma=5.0, conforming=True,
                    smoother="scms", tau=0.5, delta=0.12, rhs="manufactured",
                    outer="pcg", precision="fp64")
    if name == "c2":
        # 4x4 bilinear patches, 10% perturbation, 64/96 checkerboard, p=4, SIPG, hybrid
        corners = grid_corners((4, 4), frac=0.10, seed=1902)
        elems = checkerboard_elems((4, 4), 64 // scale, 96 // scale)
        return dict(corners=corners, elems=elems, p=4, sigma=5.0, conforming=False,
                    smoother="hybrid", tau=0.25, delta=0.1, rhs=("normal", 2002),
                    outer="pcg", precision="fp64")
    if name == "c3":
        corners = grid_corners((2, 2, 2), frac=0.05, seed=1903)
        elems = checkerboard_elems((2, 2, 2), 48 // scale, 64 // scale)
        return dict(corners=corners, elems=elems, p=3, sigma=5.0, conforming=False,
                    smoother="hybrid", tau=0.25, delta=0.12, rhs="manufactured",
                    outer="fcg", precision="fp32")
    if name == "c4":
        corners = grid_corners((4, 4), frac=0.10, seed=1902)
        elems = np.full((16, 2), 256 // scale, dtype=np.int64)
        return dict(corners=corners, elems=elems, p=6, sigma=5.0, conforming=False,
                    smoother="hybrid", tau=0.25, delta=0.1, rhs=("normal", 4000),
                    nrhs=64, outer="ir", precision="fp32")
    raise KeyError(name)


def serving_requests(n_requests=2000, master_seed=5000):
    """Heterogeneous 2D SIPG requests: grid a x b patches (a, b ~ U{2..8}),
    10% perturbation, p ~ U{2..6}, n0 ~ U{16,32,64,128,256} with checkerboard
    partner 3 n0 / 2 (3 n0 / 4 above 256), N(0,1) right-hand side."""
    ss = np.random.SeedSequence(master_seed)
    out = []
    for child in ss.spawn(n_requests):
        rng = np.random.default_rng(child)
        a = int(rng.integers(2, 9))
        b = int(rng.integers(2, 9))
        p = int(rng.integers(2, 7))
        n0 = int(rng.choice([16, 32, 64, 128, 256]))
        n1 = 3 * n0 // 2 if 3 * n0 // 2 <= 256 else 3 * n0 // 4
        gseed = int(rng.integers(0, 2 ** 31 - 1))
        rseed = int(rng.integers(0, 2 ** 31 - 1))
        out.append(dict(counts=(a, b), p=p, n0=n0, n1=n1, geom_seed=gseed, rhs_seed=rseed))
    return out


def request_problem(req):
    corners = grid_corners(req["counts"], frac=0.10, seed=req["geom_seed"])
    elems = checkerboard_elems(req["counts"], req["n0"], req["n1"])
    return dict(corners=corners, elems=elems, p=req["p"], sigma=5.0, conforming=False,
                smoother="hybrid", tau=0.25, delta=0.1, rhs=("normal", req["rhs_seed"]),
                outer="pcg", precision="fp32")
