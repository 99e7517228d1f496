"""Pins of the oracle's direct sum with a softening length per particle
(each pair takes the mean of its two particles' kernels): it reduces bit for
bit to the single-length sum, keeps the pair forces equal and opposite,
satisfies the Poisson identity with the mean kernel, and its T and j are
finite differences of its g."""
import numpy as np
import pytest

import workloads
from test_oracle_field import W_m4, sym6


def _set(n, seed):
    x, v, m = workloads.plummer(n, seed=seed)
    h = np.exp(np.random.default_rng(seed).uniform(np.log(0.02), np.log(0.3), n))
    return x, v, m, h


def test_equal_lengths_reduce_to_single_softening(orc):
    x, v, m, _ = _set(300, 1)
    h = np.full(len(m), 0.07)
    for a, b in zip(orc.direct_soft(x, v, m, h, 1.3), orc.direct(x, v, m, 0.07, 1.3)):
        assert np.array_equal(a, b)


def test_pair_forces_equal_and_opposite(orc):
    x, v, m, h = _set(400, 2)
    a, j, _ = orc.direct_soft(x, v, m, h, 1.0)
    sa = np.sum(m[:, None] * np.abs(a))
    assert np.max(np.abs((m[:, None] * a).sum(0))) < 1e-13 * sa
    assert np.max(np.abs((m[:, None] * j).sum(0))) < 1e-12 * np.sum(m[:, None] * np.abs(j))
    # and the one-sided choice (the target's own length only) is not
    a1 = np.stack([orc.direct(x, v, m, h[i], 1.0, [i])[0][0] for i in range(40)])
    assert np.max(np.abs(a1 - a[:40])) > 1e-6


def test_poisson_identity_mean_kernel(orc):
    """tr T_i = -4 pi G sum_j m_j (W(r, h_i) + W(r, h_j)) / 2."""
    x, v, m, h = _set(250, 3)
    _, _, T = orc.direct_soft(x, v, m, h, 1.0)
    r = np.linalg.norm(x[None, :, :] - x[:, None, :], axis=2)
    W = 0.5 * (W_m4(r, h[:, None]) + W_m4(r, h[None, :]))
    np.fill_diagonal(W, 0.0)
    ref = -4 * np.pi * (W * m[None, :]).sum(1)
    np.testing.assert_allclose(T[:, 0] + T[:, 1] + T[:, 2], ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_tide_and_jerk_are_derivatives(orc):
    x, v, m, h = _set(120, 4)
    a, j, T = orc.direct_soft(x, v, m, h, 1.0)
    d = 1e-6
    for i in (0, 7, 50):
        for b in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, b] += d
            xm[i, b] -= d
            ap = orc.direct_soft(xp, v, m, h, 1.0, [i])[0][0]
            am = orc.direct_soft(xm, v, m, h, 1.0, [i])[0][0]
            np.testing.assert_allclose((ap - am) / (2 * d), sym6(T)[i][:, b], rtol=1e-5,
                                       atol=1e-6 * np.abs(T[i]).max())
    ap = orc.direct_soft(x + d * v, v, m, h, 1.0)[0]
    am = orc.direct_soft(x - d * v, v, m, h, 1.0)[0]
    np.testing.assert_allclose((ap - am) / (2 * d), j, rtol=1e-5, atol=1e-6 * np.abs(j).max())


def test_neighbour_length_brute_force(orc):
    """A plain loop over a small set, and scipy's k-d tree on a larger one."""
    rng = np.random.default_rng(9)
    x = rng.normal(size=(40, 3))
    for k in (1, 5, 39):
        got = orc.neighbour_length(x, k)
        for i in range(40):
            d = sorted(float(np.sqrt(np.sum((x[j] - x[i]) ** 2))) for j in range(40) if j != i)
            assert abs(got[i] - d[k - 1]) <= 1e-15 * d[k - 1]
    from scipy.spatial import cKDTree
    x, _, _ = workloads.plummer(5000, seed=10)
    ref = cKDTree(x).query(x, k=33)[0][:, 32]
    np.testing.assert_allclose(orc.neighbour_length(x, 32), ref, rtol=1e-14)


def test_neighbour_length_periodic(orc):
    """Nearest images: scipy's periodic k-d tree on clumps wrapped into the
    unit cube (some clumps cut by the faces), a plain loop over explicit
    images on a small set, and a lattice filling the box, where every point,
    the corner ones included, has its 6 neighbours at the spacing."""
    from scipy.spatial import cKDTree
    x, _, _, _ = workloads.clumps(4000, seed=12)
    x = np.mod(x, 1.0)
    ref = cKDTree(x, boxsize=1.0).query(x, k=17)[0][:, 16]
    np.testing.assert_allclose(orc.neighbour_length(x, 16, box=1.0), ref, rtol=1e-13)
    rng = np.random.default_rng(13)
    y = rng.uniform(0, 2.0, (30, 3))
    shifts = np.array([[a, b, c] for a in (-2, 0, 2) for b in (-2, 0, 2) for c in (-2, 0, 2)], float)
    for k in (1, 4):
        got = orc.neighbour_length(y, k, box=2.0)
        for i in range(30):
            d = sorted(min(float(np.linalg.norm(y[j] + s - y[i])) for s in shifts) for j in range(30) if j != i)
            assert abs(got[i] - d[k - 1]) <= 1e-14 * d[k - 1]
    a = 0.25
    g = np.arange(4) * a
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    assert np.all(orc.neighbour_length(lat, 6, box=1.0) == a)
    assert np.all(orc.neighbour_length(lat, 7, box=1.0) == pytest.approx(a * np.sqrt(2), rel=1e-15))
    # without the box the corner points see only 3 neighbours at the spacing
    assert orc.neighbour_length(lat, 6)[0] > a


def test_neighbour_length_lattice(orc):
    """On a cubic lattice of spacing a the 1st..6th neighbours sit at a,
    the 7th..18th at a sqrt(2) (interior points)."""
    a = 0.3
    g = np.arange(7) * a
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    centre = [np.argmin(np.linalg.norm(x - 3 * a, axis=1))]
    for k, d in ((1, a), (6, a), (7, a * np.sqrt(2)), (18, a * np.sqrt(2)), (19, a * np.sqrt(3))):
        assert orc.neighbour_length(x, k, centre)[0] == pytest.approx(d, rel=1e-14)


# ---- Price & Monaghan terms (oracle only) -------------------------------------
def test_soft_potential_kernel(orc):
    """psi against the force kernel it must integrate: psi(1) = -1, and
    psi(u) = -1 - int_u^1 s F(s) ds with F = h^3 f from `kernel` (scipy's
    quadrature); the known centre value -14/5; continuity at 1/2 and 1."""
    from scipy.integrate import quad
    F = lambda s: orc.kernel(np.array([s]), 1.0)[0][0]
    for u in (0.05, 0.3, 0.49, 0.5, 0.7, 0.95, 1.0):
        ref = -1.0 - quad(lambda s: s * F(s), u, 1.0, epsabs=1e-14, epsrel=1e-13, points=[0.5])[0]
        assert orc.soft_potential(u) == pytest.approx(ref, rel=1e-11, abs=1e-12)
    assert orc.soft_potential(0.0) == pytest.approx(-2.8, rel=1e-15)
    for u in (0.5, 1.0):
        assert orc.soft_potential(u - 1e-12) == pytest.approx(orc.soft_potential(u), abs=1e-10)
    assert orc.soft_potential(3.0) == pytest.approx(-1.0 / 3.0, rel=1e-15)


def test_pm_lengths(orc):
    """Every h_i satisfies its density condition, and scaling the positions
    scales the lengths."""
    rng = np.random.default_rng(31)
    x = rng.uniform(0, 1, (60, 3))
    h = orc.pm_lengths(x, 20)
    for i in range(60):
        s = orc.m4_shape(np.linalg.norm(x - x[i], axis=1) / h[i])[0].sum()
        assert s == pytest.approx(3 * 20 / 32, rel=1e-13)
    np.testing.assert_allclose(orc.pm_lengths(2.5 * x, 20), 2.5 * h, rtol=1e-13)


def test_pm_force_is_energy_gradient(orc):
    """The mean-kernel force plus the correction is -(1/m_i) dE/dx_i, the
    energy's gradient with every h re-solved (central differences, step
    1e-6); the mean-kernel force alone is not (the set is sparse, so the
    lengths and the correction are large), and the correction conserves
    momentum."""
    rng = np.random.default_rng(32)
    n, N, G = 30, 16, 1.3
    x = rng.uniform(0, 1, (n, 3))
    m = rng.uniform(0.5, 1.5, n)
    h = orc.pm_lengths(x, N)
    a = orc.direct_soft(x, np.zeros_like(x), m, h, G)[0]
    ac = orc.pm_correction(x, m, h, N, G)
    step = 1e-6
    fd = np.zeros((n, 3))
    for i in range(n):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += step
            xm[i, c] -= step
            fd[i, c] = -(orc.pm_energy(xp, m, N, G) - orc.pm_energy(xm, m, N, G)) / (2 * step) / m[i]
    scale = np.linalg.norm(fd, axis=1)
    assert np.max(np.abs(a + ac - fd).max(axis=1) / scale) <= 1e-6
    assert np.max(np.abs(a - fd).max(axis=1) / scale) >= 1e-2
    assert np.abs((m[:, None] * ac).sum(axis=0)).max() <= 1e-13 * np.abs(m[:, None] * ac).sum()
