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
