"""Pins of the oracle's polynomial predictor (Sec. 2.2: extrapolate g from a
few logged past values, the alternative to the jerk predictor of Eq. 6)."""
import numpy as np
import pytest

import workloads


def _log_sequence(orc, n, depth, events, rng):
    """Apply ``events`` (time, rows) to an empty log; also return, per row,
    the full list of (t, g) it logged, newest last."""
    ha = np.zeros((depth, n, 3))
    ht = np.zeros((depth, n))
    hn = np.zeros(n, dtype=np.int32)
    full = [[] for _ in range(n)]
    for t, rows in events:
        acc0 = rng.normal(size=(n, 3))
        orc.force_log(ha, ht, hn, rows, acc0, t)
        for i in rows:
            full[i].append((t, acc0[i].copy()))
    return ha, ht, hn, full


def test_force_log_keeps_the_newest(orc):
    """Brute force: after any sequence of logs, slot k of a row holds its
    k-th newest logged force and time, and the count saturates at depth."""
    rng = np.random.default_rng(1)
    n, depth = 40, 3
    events = [(float(s), np.sort(rng.choice(n, rng.integers(0, n + 1), replace=False))) for s in range(9)]
    ha, ht, hn, full = _log_sequence(orc, n, depth, events, rng)
    for i in range(n):
        assert hn[i] == min(len(full[i]), depth)
        for k, (t, a) in enumerate(reversed(full[i][-depth:])):
            assert ht[k, i] == t
            assert np.array_equal(ha[k, i], a)


@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_reproduces_polynomials(orc, order):
    """A force that is a polynomial of degree <= order in time is
    extrapolated exactly (to rounding) from order + 1 logged values."""
    rng = np.random.default_rng(10 + order)
    n, depth = 64, 4
    coef = rng.normal(size=(order + 1, n, 3))

    def g(t):
        return sum(coef[p] * t**p for p in range(order + 1))

    ha = np.zeros((depth, n, 3))
    ht = np.zeros((depth, n))
    hn = np.zeros(n, dtype=np.int32)
    for t in np.cumsum(rng.uniform(0.2, 1.0, depth + 2)):
        orc.force_log(ha, ht, hn, np.arange(n), g(t), t)
    t = ht[0, 0] + 0.7
    out = orc.predict_poly(ha, ht, hn, order, t)
    np.testing.assert_allclose(out, g(t), rtol=1e-10, atol=1e-10 * np.abs(g(t)).max())
    if order >= 1:
        # one degree short misses the top term
        low = orc.predict_poly(ha, ht, hn, order - 1, t)
        assert np.max(np.abs(low - g(t))) > 1e-3


def test_matches_polyfit(orc):
    """Interpolation through d + 1 points equals numpy's degree-d fit."""
    rng = np.random.default_rng(2)
    n, depth = 30, 4
    events = [(t, np.arange(n)) for t in np.cumsum(rng.uniform(0.5, 1.5, 5))]
    ha, ht, hn, _ = _log_sequence(orc, n, depth, events, rng)
    t = float(ht[0, 0]) + 0.9
    for order in range(4):
        out = orc.predict_poly(ha, ht, hn, order, t)
        for i in range(n):
            ts = ht[: order + 1, i]
            for c in range(3):
                if order == 0:
                    ref = ha[0, i, c]
                else:
                    ref = np.polyval(np.polyfit(ts, ha[: order + 1, i, c], order), t)
                assert out[i, c] == pytest.approx(ref, rel=1e-8, abs=1e-8)


def test_node_rules(orc):
    """Fewer logs than order + 1 lower the degree; a repeated time stops the
    nodes; nothing logged gives NaN; at t = newest time the newest force
    comes back bit for bit."""
    rng = np.random.default_rng(3)
    n, depth = 4, 4
    ha = np.zeros((depth, n, 3))
    ht = np.zeros((depth, n))
    hn = np.zeros(n, dtype=np.int32)
    a1, a2, a3 = (rng.normal(size=(n, 3)) for _ in range(3))
    orc.force_log(ha, ht, hn, [0, 1, 2], a1, 1.0)
    orc.force_log(ha, ht, hn, [0, 1, 2], a2, 2.0)
    orc.force_log(ha, ht, hn, [1], a3, 2.0)   # row 1 logged twice at t = 2
    out = orc.predict_poly(ha, ht, hn, 3, 3.0)
    # rows 0 and 2: two logs -> linear through (1, a1), (2, a2)
    np.testing.assert_allclose(out[0], a2[0] + (a2[0] - a1[0]), rtol=1e-14)
    np.testing.assert_allclose(out[2], a2[2] + (a2[2] - a1[2]), rtol=1e-14)
    # row 1: the newest two share t = 2, so only the newest force is used
    assert np.array_equal(out[1], a3[1])
    assert np.all(np.isnan(out[3]))
    same = orc.predict_poly(ha, ht, hn, 3, 2.0)
    assert np.array_equal(same[0], a2[0]) and np.array_equal(same[2], a2[2])


def test_weight_sum(orc):
    """The Lagrange weights sum to one (constants are reproduced); their
    absolute sum grows with the extrapolation distance."""
    ht = np.array([[3.0], [2.0], [1.0]])
    hn = np.array([3], dtype=np.int32)
    assert orc.predict_poly_weight_sum(ht, hn, 2, 3.0)[0] == 1.0
    # nodes 3, 2, 1 at t = 4: weights 3, -3, 1
    assert orc.predict_poly_weight_sum(ht, hn, 2, 4.0)[0] == pytest.approx(7.0, rel=1e-15)


def test_predictors_remove_the_lag(orc):
    """Sec. 2.2: holding g leaves an error linear in the lag; a linear
    polynomial through the last two evaluations (spaced like the updates)
    leaves a quadratic one, a quadratic through three a cubic one.
    Ballistic particles, so g(t) is the direct sum at x + v t."""
    x, v, m = workloads.plummer(256, seed=13)
    eps = 0.05
    n = len(m)

    def g(t):
        return orc.direct(x + t * v, v, m, eps, 1.0)[0]

    errs = {0: [], 1: [], 2: []}
    for tau in [8e-3, 4e-3, 2e-3]:
        ha = np.zeros((3, n, 3))
        ht = np.zeros((3, n))
        hn = np.zeros(n, dtype=np.int32)
        for s in (-2, -1, 0):
            orc.force_log(ha, ht, hn, np.arange(n), g(s * tau), s * tau)
        at = g(tau)
        for order in errs:
            pred = orc.predict_poly(ha, ht, hn, order, tau)
            errs[order].append(np.median(np.linalg.norm(pred - at, axis=1) / np.linalg.norm(at, axis=1)))
    for order, lo, hi in [(0, 1.8, 2.2), (1, 3.5, 4.5), (2, 7.0, 9.0)]:
        r = [errs[order][i] / errs[order][i + 1] for i in range(2)]
        assert all(lo < x_ < hi for x_ in r), (order, r)
    assert errs[1][-1] < 0.05 * errs[0][-1]
