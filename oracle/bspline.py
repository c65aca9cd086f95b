"""Univariate B-splines of maximum smoothness (Section 2, the patch spaces
S_{p,h}: degree p, C^{p-1}, grid size h on the parameter domain (0,1)).

Cox--de Boor recursion written out on full arrays; Gauss--Legendre tables.
Oracle code: test infrastructure only.
"""
import numpy as np


def open_uniform_knots(n_el, p):
    """Open knot vector on [0,1]: p+1 fold end knots, n_el-1 simple interior
    knots at i/n_el.  The space has n_el + p basis functions (Section 2,
    uniform grid of size h = 1/n_el)."""
    inner = np.arange(1, n_el, dtype=np.float64) / n_el
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def _degree0(knots, x):
    """Indicator functions of the knot spans, closed on the right at x = 1."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(knots) - 1
    out = np.zeros((x.size, m))
    for i in range(m):
        a, b = knots[i], knots[i + 1]
        if b > a:
            out[:, i] = (x >= a) & (x < b)
    # right end point belongs to the last non-empty span
    last = max(i for i in range(m) if knots[i + 1] > knots[i])
    out[x == knots[-1], :] = 0.0
    out[x == knots[-1], last] = 1.0
    return out


def _safe_div(num, den):
    return np.where(den != 0.0, num / np.where(den != 0.0, den, 1.0), 0.0)


def basis_table(knots, p, x):
    """All degrees 0..p of the Cox--de Boor recursion.
    Returns list T with T[k] of shape (len(x), len(knots)-1-k)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    T = [_degree0(knots, x)]
    for k in range(1, p + 1):
        prev = T[-1]
        m = len(knots) - 1 - k
        cur = np.zeros((x.size, m))
        for i in range(m):
            left = _safe_div(x - knots[i], knots[i + k] - knots[i])
            right = _safe_div(knots[i + k + 1] - x, knots[i + k + 1] - knots[i + 1])
            cur[:, i] = left * prev[:, i] + right * prev[:, i + 1]
        T.append(cur)
    return T


def basis_derivative(knots, p, x, order):
    """order-th derivative of all degree-p B-splines at x, shape (len(x), n).
    Uses d/dx B_{i,k} = k (B_{i,k-1}/(t_{i+k}-t_i) - B_{i+1,k-1}/(t_{i+k+1}-t_{i+1}))
    applied `order` times."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    if order > p:
        return np.zeros((x.size, len(knots) - 1 - p))
    T = basis_table(knots, p - order, x)
    D = T[-1]
    for k in range(p - order + 1, p + 1):
        m = len(knots) - 1 - k
        nxt = np.zeros((x.size, m))
        for i in range(m):
            a = _safe_div(np.float64(k), knots[i + k] - knots[i])
            b = _safe_div(np.float64(k), knots[i + k + 1] - knots[i + 1])
            nxt[:, i] = a * D[:, i] - b * D[:, i + 1]
        D = nxt
    return D


def gauss_legendre(q):
    """q-point Gauss--Legendre rule on [0,1]."""
    xi, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (xi + 1.0), 0.5 * w


def element_quadrature(n_el, q):
    """Points and weights of q-point Gauss on every element of the uniform
    grid with n_el elements on [0,1], ordered element by element."""
    xi, w = gauss_legendre(q)
    h = 1.0 / n_el
    e = np.arange(n_el)[:, None]
    pts = (e + xi[None, :]) * h
    wts = np.broadcast_to(w[None, :] * h, pts.shape)
    return pts.ravel(), wts.ravel().copy()


def greville(knots, p):
    """Greville abscissae (averages of p consecutive interior knots)."""
    n = len(knots) - 1 - p
    return np.array([knots[i + 1:i + p + 1].mean() for i in range(n)])
