"""GPU parity with a softening length per particle (each pair takes the mean
of its two kernels): the direct sum against the oracle's (FP64 to 1e-12 of a
cancellation-free bound), and the tree walk at theta = 0 and at the tree
tolerances, with lengths that follow the local particle spacing."""
import numpy as np
import pytest
import torch

import workloads
from conftest import rel_err, tensor_rel_err

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _t(a, dtype=None):
    return torch.tensor(a, device=DEV) if dtype is None else torch.tensor(a, dtype=dtype, device=DEV)


def _outputs(n):
    return [torch.full((n, k), float("nan"), dtype=torch.float64, device=DEV) for k in (3, 3, 6)]


def _clumps_soft(n, seed=3, k=32):
    x, v, m, _ = workloads.clumps(n, seed=seed)
    return x, v, m, workloads.neighbour_lengths(x, k)


def _bound(x, m, h, rows):
    """sum_j m_j 11 / max(r, min(h_i, h_j))^2 >= sum_j m_j |f_ij| r: a
    cancellation-free size of g (the spline's f r never exceeds 32 / (3 h^2))."""
    out = np.empty(len(rows))
    for t, i in enumerate(rows):
        r = np.linalg.norm(x - x[i], axis=1)
        hm = np.minimum(h[i], h)
        w = m / np.maximum(r, hm) ** 2
        w[i] = 0.0
        out[t] = 11.0 * w.sum()
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_direct_soft(ag, orc, prec):
    x, v, m, h = _clumps_soft(3001, seed=5)
    with ag.Context(0) as c:
        c.set_softening(_t(h))
        out = _outputs(len(m))
        c.grav_direct(_t(x), _t(v), _t(m), None, 1e-3, 1.0, *out,
                      precision=ag.AG_FP64 if prec == "fp64" else ag.AG_FP32_PAIRS)
        c.sync()
    a, j, T = (o.cpu().numpy() for o in out)
    ar, jr, Tr = orc.direct_soft(x, v, m, h, 1.0)
    if prec == "fp64":
        rows = np.arange(0, len(m), 7)
        sa = _bound(x, m, h, rows)
        assert np.max(np.abs(a[rows] - ar[rows]).max(axis=1) / sa) <= 1e-12
        assert np.median(rel_err(a, ar)) <= 1e-12
        assert np.median(tensor_rel_err(T, Tr)) <= 1e-11
        assert np.median(rel_err(j, jr)) <= 1e-11
    else:
        assert np.median(rel_err(a, ar)) <= 1e-5
        assert np.median(tensor_rel_err(T, Tr)) <= 1e-4


@pytest.mark.parametrize("n,frac", [(9000, 1.0), (3001, 0.05)])
def test_direct_soft_launch_shapes(ag, orc, n, frac):
    """Per-particle softening in the direct sum at 16 targets per workgroup
    (every row of 9000) and with a small listed set split over workgroups;
    sampled rows against the oracle."""
    x, v, m, h = _clumps_soft(n, seed=n)
    act = None if frac == 1.0 else np.sort(workloads.random_subset(n, frac, seed=n))
    rows = np.random.default_rng(n).choice(n if act is None else act, 48, replace=False)
    ar, jr, Tr = orc.direct_soft(x, v, m, h, 1.0, rows)
    sa = _bound(x, m, h, rows)
    for prec in ("fp64", "fp32"):
        with ag.Context(0) as c:
            c.set_softening(_t(h))
            out = _outputs(n)
            ia = None if act is None else _t(act.astype(np.int32), torch.int32)
            c.grav_direct(_t(x), _t(v), _t(m), ia, 1e-3, 1.0, *out,
                          precision=ag.AG_FP64 if prec == "fp64" else ag.AG_FP32_PAIRS)
            c.sync()
        a, j, T = (o.cpu().numpy() for o in out)
        if act is not None:
            other = np.setdiff1d(np.arange(n), act)
            assert np.all(np.isnan(a[other]))
        if prec == "fp64":
            assert np.max(np.abs(a[rows] - ar).max(axis=1) / sa) <= 1e-12
            assert np.median(rel_err(a[rows], ar)) <= 1e-12
            assert np.median(tensor_rel_err(T[rows], Tr)) <= 1e-11
            assert np.median(rel_err(j[rows], jr)) <= 1e-11
        else:
            assert np.median(rel_err(a[rows], ar)) <= 1e-5
            assert np.median(tensor_rel_err(T[rows], Tr)) <= 1e-4


def _tree_soft(ag, x, v, m, h, theta, active=None, box=0.0, ewald=False):
    with ag.Context(0) as c:
        if box:
            c.set_periodic(box, ewald=ewald)
        c.set_softening(_t(h))
        c.tree_build(_t(x), _t(v), _t(m), 16)
        out = _outputs(len(m))
        ia = None if active is None else _t(active, torch.int32)
        c.grav_eval(ia, theta, 1e-3, 1.0, *out)
        c.sync()
    return [o.cpu().numpy() for o in out]


def test_tree_soft_theta0(ag, orc):
    x, v, m, h = _clumps_soft(4099, seed=6)
    a, j, T = _tree_soft(ag, x, v, m, h, 0.0)
    ar, jr, Tr = orc.direct_soft(x, v, m, h, 1.0)
    assert np.median(rel_err(a, ar)) <= 1e-5
    assert np.median(tensor_rel_err(T, Tr)) <= 1e-4
    assert np.median(rel_err(j, jr)) <= 1e-4


@pytest.mark.parametrize("theta", [0.5, 0.7])
def test_tree_soft(ag, orc, theta):
    x, v, m, h = _clumps_soft(1 << 15, seed=7)
    a, j, T = _tree_soft(ag, x, v, m, h, theta)
    rows = np.random.default_rng(1).choice(len(m), 2048, replace=False)
    ar, jr, Tr = orc.direct_soft(x, v, m, h, 1.0, rows)
    ea, ej, et = rel_err(a[rows], ar), rel_err(j[rows], jr), tensor_rel_err(T[rows], Tr)
    print(f"\nsoftened tree theta={theta}: median g {np.median(ea):.2e} j {np.median(ej):.2e} T {np.median(et):.2e}; "
          f"p99 {np.percentile(ea, 99):.2e} {np.percentile(ej, 99):.2e} {np.percentile(et, 99):.2e}")
    assert np.median(ea) <= 1e-3 and np.percentile(ea, 99) <= 1e-2
    assert np.median(et) <= 5e-3 and np.percentile(et, 99) <= 5e-2
    assert np.median(ej) <= 1.5e-2 and np.percentile(ej, 99) <= 1e-1


def test_tree_soft_subset_and_equal_lengths(ag, orc):
    """A listed subset gets the same values as a full evaluation; equal
    lengths give the single-length walk."""
    x, v, m, h = _clumps_soft(1 << 14, seed=8)
    n = len(m)
    a_full, _, _ = _tree_soft(ag, x, v, m, h, 0.6)
    act = np.sort(np.random.default_rng(2).choice(n, 3000, replace=False))
    a_sub, _, _ = _tree_soft(ag, x, v, m, h, 0.6, active=act)
    assert np.all(np.isnan(a_sub[np.setdiff1d(np.arange(n), act)]))
    rows = act[:1024]
    ar, _, _ = orc.direct_soft(x, v, m, h, 1.0, rows)
    assert np.median(rel_err(a_sub[rows], ar)) <= 1e-3
    eps = 1e-3
    a_eq, _, T_eq = _tree_soft(ag, x, v, m, np.full(n, eps), 0.6)
    with ag.Context(0) as c:
        c.tree_build(_t(x), _t(v), _t(m), 16)
        out = _outputs(n)
        c.grav_eval(None, 0.6, eps, 1.0, *out)
        c.sync()
    a1, _, T1 = (o.cpu().numpy() for o in out)
    assert np.median(rel_err(a_eq, a1)) <= 1e-6
    assert np.median(tensor_rel_err(T_eq, T1)) <= 1e-6


def test_soft_ewald(ag, orc):
    """Per-particle softening in a periodic box with Ewald sums."""
    x, v, m, _ = workloads.clumps(8192, seed=10)
    x = np.mod(x, 1.0)
    h = workloads.neighbour_lengths(x, 32, box=1.0)
    a, j, T = _tree_soft(ag, x, v, m, h, 0.0, box=1.0, ewald=True)
    rows = np.random.default_rng(4).choice(len(m), 128, replace=False)
    # the oracle: the softened nearest-image sum plus the images' correction
    an, _, Tn = orc.direct(x, v, m, 1e-9, 1.0, rows, box=1.0)
    ae, _, Te = orc.direct(x, v, m, 1e-9, 1.0, rows, box=1.0, ewald=True)
    # softened nearest-image part: every source at its nearest image of the target
    a_soft = np.empty((len(rows), 3))
    for t, i in enumerate(rows):
        dd = x - x[i]
        dd -= np.round(dd)
        a_soft[t] = orc.direct_soft(x[i] + dd, np.zeros_like(x), m, h, 1.0, [i])[0][0]
    ref = a_soft + (ae - an)
    err = np.linalg.norm(a[rows] - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert np.median(err) <= 1e-5


def test_soft_arguments(ag):
    x, v, m, h = _clumps_soft(2048, seed=11)
    with ag.Context(0) as c:
        c.set_softening(_t(h[:1000]))
        with pytest.raises(ag.AgError) as e:
            c.tree_build(_t(x), _t(v), _t(m), 16)
        assert e.value.code == ag.AG_ESTATE
        c.set_softening(_t(h))
        c.tree_build(_t(x), _t(v), _t(m), 16)
        w = torch.zeros((2048, 3), dtype=torch.float64, device=DEV)
        with pytest.raises(ag.AgError) as e:
            c.grav_backward(None, w, 0.7, 1e-3, 1.0, torch.zeros_like(w),
                            torch.zeros(2048, dtype=torch.float64, device=DEV))
        assert e.value.code == ag.AG_ESTATE
        bad = h.copy()
        bad[5] = -1.0
        c.set_softening(_t(bad))
        with pytest.raises(ag.AgError) as e:
            c.sync()
        assert e.value.code == ag.AG_ENONFINITE
        c.set_softening(None)
        c.tree_build(_t(x), _t(v), _t(m), 16)
        c.sync()
