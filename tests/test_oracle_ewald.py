"""Pins of the oracle's Ewald sums (the periodic g and T of Sec. 3.4's
cosmological problem; the jerk stays nearest-image there).

Fixed by: independence of the splitting parameter alpha (a wrong sign or
factor in either half of the split breaks it), the zeros at the half-box
symmetry points, the background's pull -(4 pi / 3) G m d / L^3 and tide
(4 pi / 3) G m / L^3 I near d = 0, Poisson's tr T = 4 pi G m / L^3 away from
the mass, T as a finite difference of g, periodicity, and a perfect lattice
(no force, isotropic tide of the mean density)."""
import itertools

import numpy as np
import pytest

from test_oracle_field import sym6

L = 1.7


def _cell_points(k, seed):
    return np.random.default_rng(seed).uniform(-L / 2, L / 2, (k, 3))


def test_alpha_independence(orc):
    d = _cell_points(40, 1)
    ref = orc.ewald_unit(d, L, alpha=2.0 / L, nr=3, nk=4)
    for a, nr, nk in ((1.5 / L, 4, 4), (3.0 / L, 3, 7), (2.5 / L, 3, 6)):
        got = orc.ewald_unit(d, L, alpha=a, nr=nr, nk=nk)
        for x, y in zip(got, ref):
            np.testing.assert_allclose(x, y, rtol=0, atol=1e-12 * np.abs(y).max())


def test_half_box_points_feel_nothing(orc):
    pts = [np.array(p) * L / 2 for p in itertools.product([0, 1], repeat=3) if any(p)]
    g, T, dg, dT = orc.ewald_unit(np.array(pts), L)
    assert np.max(np.abs(g)) < 1e-13 / L**2
    # and dg there is minus the single image's Newtonian pull
    r = np.linalg.norm(pts, axis=1)
    np.testing.assert_allclose(dg, -np.array(pts) / r[:, None] ** 3, rtol=1e-12, atol=1e-13)


def test_background_near_zero(orc):
    c = 4 * np.pi / 3 / L**3
    g, T, dg, dT = orc.ewald_unit(np.zeros((1, 3)), L)
    np.testing.assert_allclose(dg[0], 0.0, atol=1e-14)
    np.testing.assert_allclose(sym6(dT)[0], c * np.eye(3), rtol=1e-12, atol=1e-12 * c)
    rng = np.random.default_rng(2)
    for s in (1e-3, 1e-2):
        d = rng.normal(size=(5, 3))
        d *= s * L / np.linalg.norm(d, axis=1)[:, None]
        _, _, dg, _ = orc.ewald_unit(d, L)
        # cubic symmetry: the images' own field is O(d^3) near the origin
        np.testing.assert_allclose(dg, -c * d, rtol=5 * s**2, atol=1e-15)


def test_poisson_trace(orc):
    d = _cell_points(50, 3)
    _, T, _, _ = orc.ewald_unit(d, L)
    np.testing.assert_allclose(T[:, 0] + T[:, 1] + T[:, 2], 4 * np.pi / L**3, rtol=1e-11)


def test_tide_is_gradient(orc):
    d = _cell_points(10, 4) * 0.9
    _, T, _, _ = orc.ewald_unit(d, L)
    h = 1e-6 * L
    for b in range(3):
        e = np.zeros(3)
        e[b] = h
        gp, _, _, _ = orc.ewald_unit(d + e, L)
        gm, _, _, _ = orc.ewald_unit(d - e, L)
        # T = dg/dx_target = -dg/dd
        np.testing.assert_allclose(-(gp - gm) / (2 * h), sym6(T)[:, :, b], rtol=1e-6,
                                   atol=1e-7 * np.abs(T).max())


def test_periodicity(orc):
    d = _cell_points(20, 5) * 0.8
    g0, T0, _, _ = orc.ewald_unit(d, L, nr=5)
    for shift in ([L, 0, 0], [0, -L, L], [L, L, -L]):
        g1, T1, _, _ = orc.ewald_unit(d + np.array(shift), L, nr=5)
        np.testing.assert_allclose(g1, g0, rtol=0, atol=1e-11 * np.abs(g0).max())
        np.testing.assert_allclose(T1, T0, rtol=0, atol=1e-11 * np.abs(T0).max())


def test_pair_is_ewald_field(orc):
    """Two bodies: each feels the other's periodic field; the self term adds
    only the background tide of its own images; j stays nearest-image."""
    x = np.array([[0.1, 0.2, 0.3], [1.4, 0.9, 0.35]])
    v = np.array([[0.0, 1.0, 0.0], [0.5, 0.0, -0.2]])
    m = np.array([0.3, 0.8])
    G, eps = 1.3, 1e-3
    a, j, T = orc.direct(x, v, m, eps, G, box=L, ewald=True)
    d = x[1] - x[0]
    d -= L * np.round(d / L)
    g, Tu, _, dT0 = orc.ewald_unit(np.stack([d, np.zeros(3)]), L)
    np.testing.assert_allclose(a[0], G * m[1] * g[0], rtol=1e-12)
    np.testing.assert_allclose(T[0], G * (m[1] * Tu[0] + m[0] * dT0[1]), rtol=1e-11, atol=1e-12)
    _, jn, _ = orc.direct(x, v, m, eps, G, box=L)
    assert np.array_equal(j, jn)


@pytest.mark.parametrize("k", [3, 4])
def test_perfect_lattice(orc, k):
    """A k^3 lattice filling the box is the box's uniform density: no force,
    and the tide of the neutralising mean density, (4 pi / 3) G M / L^3 I."""
    g = (np.arange(k) + 0.5) * L / k
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    n = len(x)
    m = np.full(n, 2.0 / n)
    a, _, T = orc.direct(x, np.zeros_like(x), m, 1e-3, 1.0, box=L, ewald=True)
    c = 4 * np.pi / 3 * 2.0 / L**3
    assert np.max(np.abs(a)) < 1e-12 * c * L
    np.testing.assert_allclose(sym6(T), np.broadcast_to(c * np.eye(3), (n, 3, 3)), rtol=1e-11, atol=1e-11 * c)


def test_newton_third_law_ewald(orc):
    rng = np.random.default_rng(6)
    n = 60
    x = rng.uniform(0, L, (n, 3))
    m = rng.uniform(0.5, 1.5, n) / n
    a, _, _ = orc.direct(x, np.zeros_like(x), m, 1e-2, 1.0, box=L, ewald=True)
    scale = np.sum(m[:, None] * np.abs(a))
    assert np.max(np.abs((m[:, None] * a).sum(0))) < 1e-13 * scale
