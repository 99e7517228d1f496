"""Pins of the oracle's adjoint (gradient of L = sum_i w_i . a_i) and of its
node multipoles."""
import numpy as np
import pytest

import workloads


def _L(orc, x, v, m, w, eps):
    a, _, _ = orc.direct(x, v, m, eps, 1.0)
    return float(np.sum(w * a))


@pytest.mark.parametrize("eps,active_frac", [(0.05, 1.0), (0.3, 0.4)])
def test_adjoint_matches_central_differences(orc, eps, active_frac):
    """Central differences with h = 1e-6 in FP64 on sampled coordinates and
    masses; w is zero on inactive rows (only active targets enter L)."""
    n = 300
    x, v, m = workloads.plummer(n, seed=14)
    rng = np.random.default_rng(15)
    m = m * rng.uniform(0.5, 1.5, n)
    w = rng.normal(size=(n, 3))
    if active_frac < 1:
        w[rng.uniform(size=n) > active_frac] = 0.0
    ks = rng.choice(n, 12, replace=False)
    dx, dm = orc.adjoint(x, m, w, eps, 1.0, ks)
    h = 1e-6
    for t, k in enumerate(ks):
        for c in range(3):
            xp = x.copy(); xp[k, c] += h
            xm = x.copy(); xm[k, c] -= h
            fd = (_L(orc, xp, v, m, w, eps) - _L(orc, xm, v, m, w, eps)) / (2 * h)
            assert fd == pytest.approx(dx[t, c], rel=1e-6, abs=1e-6 * np.abs(dx).max())
        mp = m.copy(); mp[k] += h
        mm = m.copy(); mm[k] -= h
        fd = (_L(orc, x, v, mp, w, eps) - _L(orc, x, v, mm, w, eps)) / (2 * h)
        assert fd == pytest.approx(dm[t], rel=1e-6, abs=1e-6 * np.abs(dm).max())


def test_adjoint_translation_invariance(orc):
    """L is unchanged by a rigid shift, so sum_k dL/dx_k = 0."""
    n = 256
    x, v, m = workloads.plummer(n, seed=16)
    w = np.random.default_rng(17).normal(size=(n, 3))
    dx, _ = orc.adjoint(x, m, w, 0.02, 1.0)
    assert np.abs(dx.sum(0)).max() < 1e-12 * np.abs(dx).sum()


def test_adjoint_mass_scaling(orc):
    """a_i is linear in the masses, so sum_k m_k dL/dm_k = L."""
    n = 256
    x, v, m = workloads.plummer(n, seed=18)
    w = np.random.default_rng(19).normal(size=(n, 3))
    _, dm = orc.adjoint(x, m, w, 0.02, 1.0)
    assert np.dot(m, dm) == pytest.approx(_L(orc, x, v, m, w, 0.02), rel=1e-12)


def test_moments_two_body(orc):
    """Two masses m at +-s along x moving apart at +-u:
    Q_xx = 4 m s^2, Q_yy = Q_zz = -2 m s^2; Qdot = dQ/dt = 8 m s u diag(1, -1/2, -1/2)."""
    mm, s, u = 0.7, 0.3, 1.9
    x = np.array([[s, 0, 0], [-s, 0, 0]]) + np.array([1.0, 2.0, 3.0])
    v = np.array([[u, 0, 0], [-u, 0, 0]]) + np.array([0.1, 0.2, 0.3])
    r = orc.moments(x, v, np.array([mm, mm]), [0, 1])
    assert r["M"] == pytest.approx(2 * mm)
    np.testing.assert_allclose(r["com"], [1, 2, 3], rtol=1e-15)
    np.testing.assert_allclose(r["u"], [0.1, 0.2, 0.3], rtol=1e-14)
    np.testing.assert_allclose(r["Q"], [4 * mm * s * s, -2 * mm * s * s, -2 * mm * s * s, 0, 0, 0],
                               rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(r["Qdot"], 8 * mm * s * u * np.array([1, -0.5, -0.5, 0, 0, 0]),
                               rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(r["lo"], [1 - s, 2, 3])
    np.testing.assert_allclose(r["hi"], [1 + s, 2, 3])


def test_moments_rate_is_time_derivative(orc):
    x, v, m = workloads.plummer(100, seed=20)
    idx = np.arange(100)
    h = 1e-6
    qp = orc.moments(x + h * v, v, m, idx)["Q"]
    qm = orc.moments(x - h * v, v, m, idx)["Q"]
    np.testing.assert_allclose(orc.moments(x, v, m, idx)["Qdot"], (qp - qm) / (2 * h), rtol=1e-7,
                               atol=1e-9)


def _sym(q):
    return np.array([[q[0], q[3], q[4]], [q[3], q[1], q[5]], [q[4], q[5], q[2]]])


def test_quadrupole_far_field_order(orc):
    """The multipole expansion of the potential,
    Phi = -G (M/R + R^T Q R / (2 R^5)), differentiated for g, approaches the
    direct sum as (s/R)^3 with the quadrupole and as (s/R)^2 without it."""
    rng = np.random.default_rng(22)
    x = rng.uniform(-0.5, 0.5, (40, 3)) * np.array([1.0, 0.6, 0.3])
    m = rng.uniform(0.5, 1.5, 40)
    v = np.zeros_like(x)
    mo = orc.moments(x, v, m, np.arange(40))
    Q = _sym(mo["Q"])
    dirn = np.array([0.48, 0.6, 0.64])
    e_q, e_m = [], []
    for R in [8.0, 16.0, 32.0]:
        p = mo["com"] + R * dirn
        a, _, _ = orc.field(x, v, m, 1e-9, 1.0, p[None])
        Rv = p - mo["com"]
        Rn = np.linalg.norm(Rv)
        g_mono = -mo["M"] * Rv / Rn**3
        g_quad = g_mono + Q @ Rv / Rn**5 - 2.5 * (Rv @ Q @ Rv) * Rv / Rn**7
        e_m.append(np.linalg.norm(g_mono - a[0]) / np.linalg.norm(a[0]))
        e_q.append(np.linalg.norm(g_quad - a[0]) / np.linalg.norm(a[0]))
    assert 3.6 < e_m[0] / e_m[1] < 4.4 and 3.6 < e_m[1] / e_m[2] < 4.4
    assert 7.0 < e_q[0] / e_q[1] < 9.0 and 7.0 < e_q[1] / e_q[2] < 9.0
