"""The SCF density series of the seeded input generator: one pass over the
iterations gives each iteration's density_blocks bit for bit, and the values
follow their definition (D_0 times the product of 1 + noise * xi_t, xi_t the
Box-Muller normal of two counter-based uniforms; |D| below d_drop set to 0)."""
import numpy as np

import systems
from systems.generate import hash_uniform


def _blocks(s, n=40, seed=3):
    rng = np.random.default_rng(seed)
    nsh = s.n_shells
    I = rng.integers(0, nsh, n)
    J = rng.integers(0, nsh, n)
    img = rng.integers(-1, 2, (n, 3))
    return np.column_stack([I, J, img]).astype(np.int64)


def test_series_equals_each_iteration():
    s = systems.diamond_cell(n=(1, 1, 1), name="cell8")
    b = _blocks(s)
    ser = systems.density_series(s, b, 5)
    assert len(ser) == 5
    for k in range(5):
        one = systems.density_blocks(s, b, iteration=k)
        for x, y in zip(ser[k], one):
            assert x.shape == y.shape and np.array_equal(x, y)
    tail = systems.density_series(s, b, 5, first=3)
    assert len(tail) == 2
    for x, y in zip(tail[1], ser[4]):
        assert np.array_equal(x, y)


def test_series_follows_its_definition():
    s = systems.diamond_cell(n=(1, 1, 1), name="cell8")
    b = _blocks(s, n=12, seed=5)
    noise = 1e-3
    d0 = systems.density_series(s, b, 1)[0]
    d3 = systems.density_series(s, b, 4, first=3)[0]
    # undo the d_drop threshold where it did not apply, then recompute the
    # factor of one element from the counter-based draws
    from systems.generate import _canonical_keys
    off = s.shell_func_offset()
    for q, (I, J, n1, n2, n3) in enumerate(b):
        if d0[q].size == 0:
            continue
        a, c = 0, 0
        gi = np.array([off[I] + a]); gj = np.array([off[J] + c]); img = np.array([[n1, n2, n3]])
        ci, cj, cn = _canonical_keys(gi, gj, img)
        fac = 1.0
        for t in range(1, 4):
            u1 = hash_uniform(s.seed ^ 0x5A5A5A5A, t, ci, cj, cn[:, 0], cn[:, 1], cn[:, 2])
            u2 = hash_uniform(s.seed ^ 0x3C3C3C3C, t, ci, cj, cn[:, 0], cn[:, 1], cn[:, 2])
            xi = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
            fac = fac * (1.0 + noise * xi)
        v0, v3 = d0[q][a, c], d3[q][a, c]
        if v0 != 0.0 and v3 != 0.0:
            assert abs(v3 - v0 * float(fac[0])) <= 1e-15 * abs(v0)
