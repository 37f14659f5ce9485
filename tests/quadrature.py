"""Brute-force references for the oracle pins (independent of any recursion).

* ``uquad_eri``: primitive Cartesian ERI from the Gaussian transform
  1/r = (2/sqrt(pi)) int_0^inf exp(-u^2 r^2) du (lower limit omega for the
  erfc kernel).  For fixed u the six-dimensional integral factorises into
  three two-dimensional Gaussian integrals of polynomials, done exactly by
  tensor Gauss-Hermite quadrature after a Cholesky change of variables; the
  u integral uses Gauss-Legendre on u = u0 + tan(pi t / 2).
* ``overlap_1d`` / ``cart_overlap``: same-centre overlaps by Gauss-Hermite.
"""
import numpy as np

_GH_X, _GH_W = np.polynomial.hermite.hermgauss(12)
_GL_X, _GL_W = np.polynomial.legendre.leggauss(240)


def _pair_2d(u, A, B, C, D, a, b, c, d, i, j, k, l):
    p = a + b
    q = c + d
    M = np.array([[p + u * u, -u * u], [-u * u, q + u * u]])
    v = np.array([a * A + b * B, c * C + d * D])
    const = a * A * A + b * B * B + c * C * C + d * D * D
    m = np.linalg.solve(M, v)
    L = np.linalg.cholesky(M)
    LinvT = np.linalg.inv(L.T)
    W1, W2 = np.meshgrid(_GH_X, _GH_X, indexing="ij")
    WW = np.outer(_GH_W, _GH_W)
    z = m[:, None, None] + np.einsum("ij,jab->iab", LinvT, np.stack([W1, W2]))
    x, xp = z
    poly = (x - A) ** i * (x - B) ** j * (xp - C) ** k * (xp - D) ** l
    return np.sum(WW * poly) / np.linalg.det(L) * np.exp(m @ M @ m - const)


def uquad_eri(A, B, C, D, a, b, c, d, pa, pb, pc, pd, u0=0.0, scale=1.0):
    """(ab|cd) for unnormalised primitives x_A^pa[0] y_A^pa[1] z_A^pa[2] exp(-a r_A^2) ..."""
    th = (_GL_X + 1) / 2
    wt = _GL_W / 2
    u = u0 + scale * np.tan(np.pi * th / 2)
    du = scale * np.pi / 2 / np.cos(np.pi * th / 2) ** 2
    tot = 0.0
    for uu, dd, w in zip(u, du, wt):
        f = 1.0
        for k in range(3):
            f *= _pair_2d(uu, A[k], B[k], C[k], D[k], a, b, c, d, pa[k], pb[k], pc[k], pd[k])
        tot += w * dd * f
    return 2.0 / np.sqrt(np.pi) * tot


def overlap_1d(n, p):
    """int x^n exp(-p x^2) dx by Gauss-Hermite."""
    return np.sum(_GH_W * (_GH_X / np.sqrt(p)) ** n) / np.sqrt(p)


def cart_powers(l):
    out = []
    for x in range(l, -1, -1):
        for y in range(l - x, -1, -1):
            out.append((x, y, l - x - y))
    return out


def uquad_eri_fast(A, B, C, D, a, b, c, d, pa, pb, pc, pd, u0=0.0, scale=1.0):
    """``uquad_eri`` with every u node at once (same rules, same result to
    rounding): the 2x2 Cholesky factor and solve are written out so that all
    nodes are evaluated as arrays."""
    th = (_GL_X + 1) / 2
    wt = _GL_W / 2
    u = u0 + scale * np.tan(np.pi * th / 2)
    du = scale * np.pi / 2 / np.cos(np.pi * th / 2) ** 2
    u2 = u * u
    p = a + b
    q = c + d
    m11, m12, m22 = p + u2, -u2, q + u2
    l11 = np.sqrt(m11)
    l21 = m12 / l11
    l22 = np.sqrt(m22 - l21 * l21)
    det_m = m11 * m22 - m12 * m12
    w1 = _GH_X[:, None]
    w2 = _GH_X[None, :]
    WW = np.outer(_GH_W, _GH_W)
    f = np.ones_like(u)
    for k in range(3):
        v1 = a * A[k] + b * B[k]
        v2 = c * C[k] + d * D[k]
        const = a * A[k] ** 2 + b * B[k] ** 2 + c * C[k] ** 2 + d * D[k] ** 2
        mu1 = (m22 * v1 - m12 * v2) / det_m
        mu2 = (m11 * v2 - m12 * v1) / det_m
        # z = mu + L^-T w, L^-T = [[1/l11, -l21/(l11 l22)], [0, 1/l22]]
        x = mu1[:, None, None] + w1[None] / l11[:, None, None] - (l21 / (l11 * l22))[:, None, None] * w2[None]
        xp = mu2[:, None, None] + w2[None] / l22[:, None, None]
        poly = (x - A[k]) ** pa[k] * (x - B[k]) ** pb[k] * (xp - C[k]) ** pc[k] * (xp - D[k]) ** pd[k]
        quad = np.sum(WW[None] * poly, axis=(1, 2))
        expo = mu1 * (m11 * mu1 + m12 * mu2) + mu2 * (m12 * mu1 + m22 * mu2) - const
        f = f * quad / (l11 * l22) * np.exp(expo)
    return 2.0 / np.sqrt(np.pi) * np.sum(wt * du * f)
