"""Pins of the oracle's periodic mode: every pair at its nearest image in a
cube of side L (the treatment the paper gives the jerk of its periodic
problem, Sec. 3.4).  Fixed by: the open-boundary sum when the box is large, the
closed form of a pair whose nearest image lies across the boundary,
invariance under a shift of every particle modulo L, Newton's third law,
cubic-lattice symmetry, the Poisson identity, and finite differences."""
import numpy as np
import pytest

from test_oracle_field import W_m4, sym6


def _box_set(n, L, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, L, (n, 3))
    v = rng.normal(size=(n, 3))
    m = rng.uniform(0.5, 1.5, n) / n
    return x, v, m


def test_large_box_is_open_boundary(orc):
    """With L far beyond the set's extent no pair is wrapped: bit-identical."""
    x, v, m = _box_set(300, 1.0, 1)
    ref = orc.direct(x, v, m, 0.01, 1.0)
    got = orc.direct(x, v, m, 0.01, 1.0, box=1e4)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_pair_across_the_boundary(orc):
    """Two bodies 0.8 L apart along x: each feels the other's image 0.2 L
    away on the other side, with the point-mass a, j and T of that image."""
    L, G = 2.0, 1.3
    x = np.array([[0.1, 0.5, 0.5], [0.1 + 0.8 * L, 0.5, 0.5]])
    v = np.array([[0.0, 0.3, 0.0], [0.2, -0.1, 0.4]])
    m = np.array([0.7, 1.1])
    a, j, T = orc.direct(x, v, m, 1e-4, G, box=L)
    d = np.array([-0.2 * L, 0.0, 0.0])     # image of body 1 as seen from body 0
    nu = v[1] - v[0]
    r = np.linalg.norm(d)
    np.testing.assert_allclose(a[0], G * m[1] * d / r**3, rtol=1e-13)
    np.testing.assert_allclose(j[0], G * m[1] * (nu / r**3 - 3 * np.dot(nu, d) * d / r**5), rtol=1e-12,
                               atol=1e-14)
    T_ref = -G * m[1] * (np.eye(3) / r**3 - 3 * np.outer(d, d) / r**5)
    np.testing.assert_allclose(sym6(T)[0], T_ref, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(a[1], -G * m[0] * d / r**3, rtol=1e-13)


def test_shift_modulo_box(orc):
    """Shifting every particle by one vector and wrapping the positions back
    into [0, L) changes nothing but rounding."""
    L = 3.0
    x, v, m = _box_set(400, L, 2)
    a0, j0, T0 = orc.direct(x, v, m, 0.02, 1.0, box=L)
    s = np.array([1.234, -2.5, 7.75])
    xs = np.mod(x + s, L)
    a1, j1, T1 = orc.direct(xs, v, m, 0.02, 1.0, box=L)
    scale = orc.abs_scale(x, m, 0.02, 1.0, box=L)[:, None]
    assert np.max(np.abs(a1 - a0) / scale) < 1e-10
    assert np.max(np.abs(T1 - T0)) < 1e-9 * np.abs(T0).max()
    assert np.max(np.abs(j1 - j0)) < 1e-9 * np.abs(j0).max()
    # and positions given outside the box (any image) give the same result
    xo = x + L * np.random.default_rng(3).integers(-3, 4, x.shape)
    a2, _, _ = orc.direct(xo, v, m, 0.02, 1.0, box=L)
    assert np.max(np.abs(a2 - a0) / scale) < 1e-10


def test_newton_third_law_periodic(orc):
    L = 1.0
    x, v, m = _box_set(500, L, 4)
    a, j, _ = orc.direct(x, v, m, 0.01, 1.0, box=L)
    scale = np.sum(m[:, None] * orc.abs_scale(x, m, 0.01, 1.0, box=L)[:, None])
    assert np.max(np.abs(np.sum(m[:, None] * a, axis=0))) < 1e-13 * scale
    assert np.max(np.abs(np.sum(m[:, None] * j, axis=0))) < 1e-12 * np.sum(m[:, None] * np.abs(j))


@pytest.mark.parametrize("k", [3, 5])
def test_cubic_lattice(orc, k):
    """A k^3 lattice (k odd) filling the box: each particle sees a neighbourhood
    symmetric under the cube's reflections, so g = 0, and T is isotropic
    and traceless (Newtonian pairs only), hence 0."""
    L = 1.0
    g = (np.arange(k) + 0.5) * L / k
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    n = len(x)
    m = np.full(n, 1.0 / n)
    a, _, T = orc.direct(x, np.zeros_like(x), m, 1e-3, 1.0, box=L)
    scale = orc.abs_scale(x, m, 1e-3, 1.0, box=L).max()
    assert np.max(np.abs(a)) < 1e-13 * scale
    assert np.max(np.abs(T)) < 1e-12 * scale * k / L


def test_poisson_identity_periodic(orc):
    """tr T_i = -4 pi G sum_j m_j W(|d_ij|) with d the nearest image."""
    L, h = 1.0, 0.15
    x, v, m = _box_set(200, L, 5)
    _, _, T = orc.direct(x, v, m, h, 1.0, box=L)
    d = x[None, :, :] - x[:, None, :]
    d -= L * np.round(d / L)
    r = np.linalg.norm(d, axis=2)
    W = W_m4(r, h)
    np.fill_diagonal(W, 0.0)
    ref = -4 * np.pi * (W * m[None, :]).sum(axis=1)
    np.testing.assert_allclose(T[:, 0] + T[:, 1] + T[:, 2], ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_derivatives_periodic(orc):
    """T = finite difference of g in the probe position; j = finite
    difference of g along the velocities (no pair near the half-box cut)."""
    L, eps = 1.0, 0.02
    x, v, m = _box_set(150, L, 6)
    p = np.array([[0.93, 0.05, 0.51]])     # near a face: many pairs wrap
    h = 1e-6
    _, _, T = orc.field(x, v, m, eps, 1.0, p, box=L)
    Tm = sym6(T)[0]
    for b in range(3):
        e = np.zeros((1, 3))
        e[0, b] = h
        ap, _, _ = orc.field(x, v, m, eps, 1.0, p + e, box=L)
        am, _, _ = orc.field(x, v, m, eps, 1.0, p - e, box=L)
        np.testing.assert_allclose((ap - am)[0] / (2 * h), Tm[:, b], rtol=1e-6, atol=1e-6 * np.abs(Tm).max())
    _, j, _ = orc.direct(x, v, m, eps, 1.0, box=L)
    ap, _, _ = orc.direct(x + h * v, v, m, eps, 1.0, box=L)
    am, _, _ = orc.direct(x - h * v, v, m, eps, 1.0, box=L)
    np.testing.assert_allclose((ap - am) / (2 * h), j, rtol=1e-5, atol=1e-5 * np.abs(j).max())
