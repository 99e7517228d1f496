"""Pins of the oracle's timestep (Eq. 7), block bins, force-age bookkeeping
(Eq. 3, Eq. 4) and jerk predictor (Eq. 6)."""
from fractions import Fraction

import numpy as np
import pytest

import workloads


ETA = 0.01  # the paper's tolerance for the tidal criterion (Sec. 3)


def test_kepler_timestep_is_orbital_time(orc):
    """Point mass: |T|_F^2 = 6 (GM/r^3)^2, so Eq. 7 gives exactly
    sqrt(eta) sqrt(r^3 / G M) (the paper's t_tidal ~ Omega^-1 becomes an
    equality)."""
    rng = np.random.default_rng(0)
    for _ in range(10):
        M = rng.uniform(0.1, 10.0)
        p = rng.normal(size=(1, 3)) * rng.uniform(0.1, 10)
        _, _, T = orc.field(np.zeros((1, 3)), np.zeros((1, 3)), np.array([M]), 1e-6, 1.0, p)
        dt, _ = orc.timestep(T, ETA, 1e3, 40)
        r = np.linalg.norm(p)
        assert dt[0] == pytest.approx(np.sqrt(ETA) * np.sqrt(r**3 / M), rel=1e-13)


def test_uniform_sphere_timestep(orc):
    """Interior of a uniform sphere: T = -(GM/R^3) I gives
    dt = 2^(1/4) sqrt(eta) sqrt(R^3 / G M)."""
    for M, R in [(1.0, 1.0), (3.0, 0.5)]:
        T = np.array([[-M / R**3, -M / R**3, -M / R**3, 0, 0, 0]])
        dt, _ = orc.timestep(T, ETA, 1e3, 40)
        assert dt[0] == pytest.approx(2**0.25 * np.sqrt(ETA) * np.sqrt(R**3 / M), rel=1e-14)


def _exact_bin(t6, eta, dt_max, k_max):
    """Smallest k >= 0 with dt_max 2^-k <= dt_grav, in exact rationals:
    dt_max 2^-k <= sqrt(eta) (n2/6)^(-1/4)  <=>  n2 dt_max^4 / (6 eta^2) <= 16^k."""
    t = [Fraction(float(c)) for c in t6]
    n2 = t[0] ** 2 + t[1] ** 2 + t[2] ** 2 + 2 * (t[3] ** 2 + t[4] ** 2 + t[5] ** 2)
    Q = n2 * Fraction(dt_max) ** 4 / (6 * Fraction(eta) ** 2)
    if Q == 0:
        return 0, Q
    k = 0
    while Q > Fraction(16) ** k and k < k_max:
        k += 1
    return k, Q


def test_bins_match_exact_rational_search(orc):
    rng = np.random.default_rng(1)
    T = rng.normal(size=(3000, 6)) * np.exp(rng.uniform(-12, 12, (3000, 1)))
    dt_max, k_max = 0.37, 30
    dt, b = orc.timestep(T, ETA, dt_max, k_max)
    for i in range(T.shape[0]):
        k, Q = _exact_bin(T[i], ETA, dt_max, k_max)
        # the oracle rounds Q once per operation; only a Q within a few ulps
        # of a power of 16 could legitimately land in the neighbouring bin
        near = any(abs(Q / Fraction(16) ** kk - 1) < Fraction(1, 10**14) for kk in range(k_max + 1))
        if not near:
            assert b[i] == k, (i, b[i], k)


def test_bin_edges_exact(orc):
    """Constructed tensors whose Q = n2 dt_max^4 / (6 eta^2) is exactly 16^k sit
    in bin k (an exact power of two stays); one ulp more moves one bin deeper.
    With eta = 1/2, dt_max = 1 and only off-diagonal entries t:
    n2 = 6 t^2, Q = 4 t^2, so t = 4^k / 2 gives Q = 16^k exactly."""
    eta, dt_max = 0.5, 1.0
    for k in range(0, 10):
        t = 0.5 * 4.0**k
        T = np.array([[0, 0, 0, t, t, t]])
        assert _exact_bin(T[0], eta, dt_max, 40)[1] == Fraction(16) ** k
        _, b = orc.timestep(T, eta, dt_max, 40)
        assert b[0] == k
        tn = np.nextafter(t, np.inf)
        _, b2 = orc.timestep(np.array([[0, 0, 0, tn, tn, tn]]), eta, dt_max, 40)
        assert b2[0] == k + 1
        assert _exact_bin(np.array([0, 0, 0, tn, tn, tn]), eta, dt_max, 40)[0] == k + 1


def test_bins_bracket_timestep(orc):
    rng = np.random.default_rng(2)
    T = rng.normal(size=(500, 6)) * np.exp(rng.uniform(-5, 5, (500, 1)))
    dt_max = 4.0
    dt, b = orc.timestep(T, ETA, dt_max, 60)
    dtb = dt_max * 2.0 ** (-b.astype(float))
    assert np.all(dtb <= dt * (1 + 1e-14))
    assert np.all((b == 0) | (2 * dtb > dt * (1 - 1e-14)))


def test_bins_clamp_and_zero(orc):
    T = np.array([[0, 0, 0, 0, 0, 0], [1e30, 0, 0, 0, 0, 0], [np.nan, 0, 0, 0, 0, 0]])
    dt, b = orc.timestep(T, ETA, 1.0, 12)
    assert b.tolist() == [0, 12, 12]
    assert np.isinf(dt[0])


def test_every_update_when_steps_are_gravity_bins(orc):
    """Sec. 2.1: for q_f <= 1 the scheme reverts exactly to updating every
    step when each element steps with its own gravity timestep.  Block
    stepping: a particle in bin k advances 2^(K-k) ticks per step."""
    K = 6
    rng = np.random.default_rng(3)
    bins = rng.integers(0, K + 1, 200).astype(np.int8)
    for q in [1 / 8, 1 / 4, 1 / 2, 1.0]:
        tf = np.zeros(200, dtype=np.int64)
        for tick in range(1, 2 ** (K + 1) + 1):
            for k in range(K + 1):
                span = 2 ** (K - k)
                if tick % span:
                    continue
                sel = np.nonzero(bins == k)[0]
                if sel.size == 0:
                    continue
                tf_new, act, _ = orc.select(tf[sel], bins[sel], span, K, q)
                assert np.all(act == 1)
                tf[sel] = tf_new
    # q_f > 1 does skip updates
    tf = np.zeros(10, dtype=np.int64)
    bins = np.zeros(10, dtype=np.int8)
    _, act, _ = orc.select(tf, bins, 2 ** K, K, 2.0)
    assert np.all(act == 0)


def test_global_step_update_period(orc):
    """Global step of one tick (the gravity-only stand-in for a hydro step):
    a particle in bin k with span s = 2^(K-k) ticks is refreshed every
    ceil(q_f s) steps (at least every step), counted from its last refresh."""
    K = 5
    bins = np.arange(K + 1, dtype=np.int8).repeat(3)
    for q in [0.0, 1 / 8, 1 / 4, 1 / 2, 1.0, 1.5]:
        tf = np.zeros(bins.size, dtype=np.int64)
        nsteps = 97
        hits = np.zeros(bins.size, dtype=np.int64)
        for _ in range(nsteps):
            tf, act, idx = orc.select(tf, bins, 1, K, q)
            hits += act
            assert np.array_equal(idx, np.nonzero(act)[0])
        span = 2.0 ** (K - bins.astype(float))
        period = np.maximum(1, np.ceil(q * span)).astype(np.int64)
        np.testing.assert_array_equal(hits, nsteps // period)


def test_bins_deeper_than_tick_update_every_step(orc):
    tf = np.zeros(4, dtype=np.int64)
    bins = np.array([7, 9, 20, 5], dtype=np.int8)
    tf, act, _ = orc.select(tf, bins, 1, 5, 1.0)
    assert act.tolist() == [1, 1, 1, 1]


def test_predictor_closed_form(orc):
    rng = np.random.default_rng(4)
    a0 = rng.normal(size=(50, 3))
    j = rng.normal(size=(50, 3))
    t0 = rng.uniform(0, 1, 50)
    out = orc.predict(a0, j, t0, 2.0)
    np.testing.assert_allclose(out, a0 + j * (2.0 - t0)[:, None], rtol=1e-15, atol=1e-15)
    # at t = t0 the predictor returns the fresh force bit for bit
    same = orc.predict(a0, j, np.full(50, 0.75), 0.75)
    assert np.array_equal(same, a0)


def test_predictor_removes_leading_lag(orc):
    """Sec. 2.2: holding g constant between updates leaves an error linear in
    the lag; the jerk predictor (Eq. 6) leaves a quadratic one.  Particles
    drift ballistically, so a(t) is the direct sum at x + v t."""
    x, v, m = workloads.plummer(256, seed=13)
    eps = 0.05
    a0, j, _ = orc.direct(x, v, m, eps, 1.0)
    t0 = np.zeros(len(m))
    errs_p, errs_n = [], []
    for tau in [4e-3, 2e-3, 1e-3]:
        at, _, _ = orc.direct(x + tau * v, v, m, eps, 1.0)
        pred = orc.predict(a0, j, t0, tau)
        errs_p.append(np.median(np.linalg.norm(pred - at, axis=1) / np.linalg.norm(at, axis=1)))
        errs_n.append(np.median(np.linalg.norm(a0 - at, axis=1) / np.linalg.norm(at, axis=1)))
    rp = [errs_p[i] / errs_p[i + 1] for i in range(2)]
    rn = [errs_n[i] / errs_n[i + 1] for i in range(2)]
    assert all(3.6 < r < 4.4 for r in rp), rp
    assert all(1.8 < r < 2.2 for r in rn), rn
    assert errs_p[-1] < 0.05 * errs_n[-1]
