"""Patch geometry maps G_k : (0,1)^d -> Omega_k (Section 2, eq. omega:2).

The workloads use multilinear maps: G_k interpolates the 2^d patch corners,
corner b has parameter coordinates (bit_0(b), ..., bit_{d-1}(b)), x fastest.
Oracle code: test infrastructure only.
"""
import numpy as np


def corner_bits(d):
    return np.array([[(b >> k) & 1 for k in range(d)] for b in range(2 ** d)])


def multilinear(corners, xh):
    """Evaluate G and its Jacobian at parameter points.

    corners: (2^d, d) physical corner coordinates.
    xh: (npts, d) parameter points.
    Returns X (npts, d) and J (npts, d, d) with J[:, a, b] = dX_a / dxh_b.
    """
    corners = np.asarray(corners, dtype=np.float64)
    xh = np.atleast_2d(np.asarray(xh, dtype=np.float64))
    d = corners.shape[1]
    bits = corner_bits(d)
    npts = xh.shape[0]
    X = np.zeros((npts, d))
    J = np.zeros((npts, d, d))
    for b in range(2 ** d):
        fac = np.where(bits[b][None, :] == 1, xh, 1.0 - xh)  # (npts, d)
        w = np.prod(fac, axis=1)
        X += w[:, None] * corners[b][None, :]
        for g in range(d):
            dfac = fac.copy()
            dfac[:, g] = 1.0 if bits[b][g] == 1 else -1.0
            dw = np.prod(dfac, axis=1)
            J[:, :, g] += dw[:, None] * corners[b][None, :]
    return X, J


def tensor_points(axes):
    """Tensor grid of 1D point arrays (axes[0] = x fastest).  Returns (npts, d)."""
    grids = np.meshgrid(*axes[::-1], indexing="ij")
    return np.stack([g.ravel() for g in grids[::-1]], axis=1)


def tensor_weights(axes_w):
    W = np.ones(1)
    for w in axes_w[::-1]:
        W = np.kron(W, w)
    return W


def patch_measure(corners, q=4):
    """|Omega_k| by Gauss quadrature of det J (exact for multilinear maps)."""
    corners = np.asarray(corners, dtype=np.float64)
    d = corners.shape[1]
    xi, w = np.polynomial.legendre.leggauss(q)
    xi = 0.5 * (xi + 1.0)
    w = 0.5 * w
    pts = tensor_points([xi] * d)
    W = tensor_weights([w] * d)
    _, J = multilinear(corners, pts)
    return float(np.sum(W * np.abs(np.linalg.det(J))))
