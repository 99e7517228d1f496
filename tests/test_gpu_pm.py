"""GPU parity of the Price & Monaghan terms of fully adaptive softening
(the lengths and Omega, the factors Z, the correction's acceleration) with
the oracle's O(n^2) FP64 sums.  The lengths are roots of a monotone sum
found by bisection on both sides, so they agree to a few ulps; the sums over
neighbours differ only in their order."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
G = 0.7


def _t(a):
    return torch.tensor(a, device=DEV)


def _sets():
    rng = np.random.default_rng(31)
    x, _, m, _ = workloads.clumps(700, seed=32)
    yield "clumps", x, m
    yield "uniform", rng.uniform(-1.0, 1.0, (601, 3)), rng.uniform(0.5, 1.5, 601) / 601
    x, _, m = workloads.plummer(650, seed=33)
    yield "plummer", x, m


@pytest.fixture(scope="module")
def cases(orc):
    out = []
    for name, x, m in _sets():
        for n_ngb in (16.0, 32.0):
            print(f"oracle {name} n={len(x)} n_ngb={n_ngb}", flush=True)
            h = orc.pm_lengths(x, n_ngb)
            om, z = orc.pm_terms(x, m, h, n_ngb, G)
            a = orc.pm_correction(x, m, h, n_ngb, G)
            out.append((name, x, m, n_ngb, h, om, z, a))
    return out


def _build(ag, c, x, m, n_leaf=16, h=None):
    n = len(x)
    c.set_softening(None if h is None else _t(h))
    c.tree_build(_t(x), _t(np.zeros((n, 3))), _t(m), n_leaf)


def test_lengths_and_omega(ag, cases):
    for name, x, m, n_ngb, hr, omr, _, _ in cases:
        print(f"lengths {name} n={len(x)} n_ngb={n_ngb}", flush=True)
        for n_leaf in (1, 16):
            with ag.Context(0) as c:
                _build(ag, c, x, m, n_leaf)
                h, om = c.pm_lengths(n_ngb)
                c.sync()
            h, om = h.cpu().numpy(), om.cpu().numpy()
            np.testing.assert_allclose(h, hr, rtol=1e-12, atol=0)
            np.testing.assert_allclose(om, omr, rtol=0, atol=1e-11)


def test_long_supports(ag, orc):
    """Supports holding far more than the 64-entry neighbour list: every
    length comes from the sum walk's bisection."""
    rng = np.random.default_rng(36)
    x = rng.uniform(-1.0, 1.0, (601, 3))
    m = np.full(601, 1.0 / 601)
    for n_ngb in (200.0, 1000.0):
        print(f"long supports n_ngb={n_ngb}", flush=True)
        hr = orc.pm_lengths(x, n_ngb)
        omr, _ = orc.pm_terms(x, m, hr, n_ngb, G)
        with ag.Context(0) as c:
            _build(ag, c, x, m)
            h, om = c.pm_lengths(n_ngb)
            c.sync()
        np.testing.assert_allclose(h.cpu().numpy(), hr, rtol=1e-12, atol=0)
        np.testing.assert_allclose(om.cpu().numpy(), omr, rtol=0, atol=1e-11)


def test_factors_and_correction(ag, cases):
    for name, x, m, n_ngb, hr, omr, zr, ar in cases:
        print(f"factors {name} n={len(x)} n_ngb={n_ngb}", flush=True)
        for n_leaf in (1, 16):
            with ag.Context(0) as c:
                _build(ag, c, x, m, n_leaf, h=hr)
                z = c.pm_factors(n_ngb, G, _t(omr))
                a = c.pm_correct(_t(zr))
                c.sync()
            z, a = z.cpu().numpy(), a.cpu().numpy()
            np.testing.assert_allclose(z, zr, rtol=0, atol=1e-12 * np.abs(zr).max())
            np.testing.assert_allclose(a, ar, rtol=0, atol=1e-12 * np.abs(ar).max())
        # the correction added at a list of rows (count on the device) equals
        # the written one there (to rounding: a walk over other target groups
        # meets the pairs in another order) and leaves every other row as it was
        n = len(x)
        rows = np.random.default_rng(7).permutation(n)[: n // 3].astype(np.int32)
        base = np.random.default_rng(8).normal(size=(n, 3))
        with ag.Context(0) as c:
            _build(ag, c, x, m, 16, h=hr)
            full = c.pm_correct(_t(zr))
            acc = _t(base)
            c.pm_correct_add(_t(zr), acc, _t(rows), torch.tensor([len(rows)], dtype=torch.int64, device=DEV))
            acc_all = _t(base)
            c.pm_correct_add(_t(zr), acc_all)
            c.sync()
        full, acc, acc_all = full.cpu().numpy(), acc.cpu().numpy(), acc_all.cpu().numpy()
        other = np.setdiff1d(np.arange(n), rows)
        np.testing.assert_array_equal(acc[other], base[other])
        tol = 1e-12 * (np.abs(full).max() + np.abs(base).max())
        np.testing.assert_allclose(acc[rows], base[rows] + full[rows], rtol=0, atol=tol)
        np.testing.assert_array_equal(acc_all, base + full)


def test_chain_on_device(ag, orc, cases):
    """Lengths, factors and correction each from the previous step's device
    output, against the oracle's own chain."""
    name, x, m, n_ngb, hr, omr, zr, ar = cases[1]
    with ag.Context(0) as c:
        _build(ag, c, x, m)
        h, om = c.pm_lengths(n_ngb)
        c.set_softening(h)
        c.tree_build(_t(x), _t(np.zeros((len(x), 3))), _t(m), 16)
        z = c.pm_factors(n_ngb, G, om)
        a = c.pm_correct(z)
        c.sync()
    np.testing.assert_allclose(a.cpu().numpy(), ar, rtol=0, atol=1e-10 * np.abs(ar).max())


def test_large_property(ag, orc):
    """At 2^20 particles: on sampled rows the lengths solve the density
    condition over every particle, and Omega matches its definition."""
    x = workloads.turbulent_sphere(1 << 20, seed=2)[0]
    n = len(x)
    n_ngb = 24.0
    with ag.Context(0) as c:
        _build(ag, c, x, np.full(n, 1.0 / n))
        h, om = c.pm_lengths(n_ngb)
        c.sync()
    h, om = h.cpu().numpy(), om.cpu().numpy()
    assert np.all(np.isfinite(h)) and np.all(h > 0)
    rows = np.random.default_rng(34).choice(n, 128, replace=False)
    for i in rows:
        u = np.sqrt(np.sum((x - x[i])**2, axis=1)) / h[i]
        w, wp = orc.m4_shape(u)
        assert abs(w.sum() - 3.0 * n_ngb / 32.0) < 1e-12 * n_ngb
        assert abs(om[i] + 32.0 / (9.0 * n_ngb) * np.sum(u * wp)) < 1e-11


def test_arguments(ag):
    x, v, m, _ = workloads.clumps(2000, seed=35)
    n = len(x)
    zeros = torch.zeros(n, dtype=torch.float64, device=DEV)
    with ag.Context(0) as c:
        with pytest.raises(ag.AgError) as e:
            c.pm_lengths(32.0, h=zeros, omega=zeros.clone())
        assert e.value.code == ag.AG_ESTATE               # no tree
        _build(ag, c, x, m)
        for bad in (10.0, 32.0 * n / 3.0, float("nan")):
            with pytest.raises(ag.AgError) as e:
                c.pm_lengths(bad)
            assert e.value.code == ag.AG_EINVAL
        with pytest.raises(ag.AgError) as e:
            c.pm_factors(32.0, G, zeros)                 # tree without softening lengths
        assert e.value.code == ag.AG_ESTATE
        with pytest.raises(ag.AgError) as e:
            c.pm_correct(zeros)
        assert e.value.code == ag.AG_ESTATE
        h, _ = c.pm_lengths(32.0)
        _build(ag, c, x, m, h=h.cpu().numpy())
        for bad in (5.0, float("nan")):
            with pytest.raises(ag.AgError) as e:
                c.pm_factors(bad, G, zeros)
            assert e.value.code == ag.AG_EINVAL
        c.set_periodic(4.0)
        _build(ag, c, np.mod(x, 4.0), m, h=h.cpu().numpy())
        with pytest.raises(ag.AgError) as e:
            c.pm_factors(32.0, G, zeros)
        assert e.value.code == ag.AG_ESTATE
        c.set_periodic(0.0)
        off = torch.tensor([0, 1000, n], dtype=torch.int64, device=DEV)
        c.set_softening(None)
        c.tree_build_batched(_t(x), _t(v), _t(m), off, 16)
        with pytest.raises(ag.AgError) as e:
            c.pm_lengths(32.0)
        assert e.value.code == ag.AG_ESTATE
        # a failed call leaves the context usable
        _build(ag, c, x, m)
        h, _ = c.pm_lengths(32.0)
        c.sync()
        assert torch.all(torch.isfinite(h))
