"""GPU parity in a periodic cube, every pair at its nearest image (the jerk
treatment of Sec. 3.4): the direct sum against the oracle's (FP64 to 1e-12 of
the cancellation-free scale), and the tree walk against it to the tree
tolerances, on clumps straddling the faces (inputs in several images), a
pancake-mode lattice and a uniform box."""
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


def _direct(ag, box, x, v, m, eps, prec, active=None):
    with ag.Context(0) as c:
        c.set_periodic(box)
        out = _outputs(len(m))
        ia = None if active is None else _t(active, torch.int32)
        c.grav_direct(_t(x), _t(v), _t(m), ia, eps, 1.0, *out, precision=prec)
        c.sync()
    return [o.cpu().numpy() for o in out]


def _tree(ag, box, x, v, m, theta, eps, active=None, n_leaf=16):
    with ag.Context(0) as c:
        c.set_periodic(box)
        c.tree_build(_t(x), _t(v), _t(m), n_leaf)
        out = _outputs(len(m))
        ia = None if active is None else _t(active, torch.int32)
        c.grav_eval(ia, theta, eps, 1.0, *out)
        c.sync()
    return [o.cpu().numpy() for o in out]


def _scales(orc, x, v, m, eps, rows, L):
    """Cancellation-free sizes sum_j m_j |term_j| of g, j and T at `rows`,
    pairs at their nearest images."""
    sa, sj, st = (np.empty(len(rows)) for _ in range(3))
    for t, i in enumerate(rows):
        d = x - x[i]
        d -= L * np.round(d / L)
        nu = v - v[i]
        r = np.linalg.norm(d, axis=1)
        f, D, _ = orc.kernel(r, eps)
        mm = m.copy()
        mm[i] = 0.0
        sa[t] = np.sum(mm * np.abs(f) * r)
        sj[t] = np.sum(mm * (np.abs(f) * np.linalg.norm(nu, axis=1) + np.abs(D) * r * r * np.linalg.norm(nu, axis=1)))
        st[t] = np.sum(mm * (np.abs(f) + np.abs(D) * r * r))
    return sa, sj, st


def _clumps_in_box(n, seed=3):
    x, v, m, _ = workloads.clumps(n, seed=seed)
    # clumps near the faces reach past them; hand a third of the particles
    # over in other images too
    k = np.random.default_rng(seed).integers(-2, 3, x.shape)
    k[::3] = 0
    return x + k, v, m


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_direct_periodic(ag, orc, prec):
    n, L, eps = 3001, 1.0, 1e-2
    x, v, m = _clumps_in_box(n)
    p = ag.AG_FP64 if prec == "fp64" else ag.AG_FP32_PAIRS
    a, j, T = _direct(ag, L, x, v, m, eps, p)
    ar, jr, Tr = orc.direct(x, v, m, eps, 1.0, box=L)
    if prec == "fp64":
        sa, sj, st = _scales(orc, x, v, m, eps, np.arange(n), L)
        assert np.max(np.abs(a - ar).max(axis=1) / sa) <= 1e-12
        assert np.max(np.abs(j - jr).max(axis=1) / sj) <= 1e-12
        assert np.max(np.abs(T - Tr).max(axis=1) / st) <= 1e-12
        assert np.median(rel_err(a, ar)) <= 1e-12
    else:
        assert np.median(rel_err(a, ar)) <= 1e-5
        assert np.median(tensor_rel_err(T, Tr)) <= 1e-4


@pytest.mark.parametrize("n,frac", [(9000, 1.0), (3001, 0.05)])
def test_direct_periodic_launch_shapes(ag, orc, n, frac):
    """The nearest-image direct sum at the launch shapes the 3001-particle
    test does not reach: 16 targets per workgroup (every row of 9000), and a
    small listed set whose sources are split over workgroups; sampled rows
    against the oracle at the FP64 bound of the cancellation-free sizes."""
    L, eps = 1.0, 1e-2
    x, v, m = _clumps_in_box(n, seed=n)
    act = None if frac == 1.0 else np.sort(workloads.random_subset(n, frac, seed=n))
    rows = np.random.default_rng(n).choice(n if act is None else act, 48, replace=False)
    for prec in ("fp64", "fp32"):
        p = ag.AG_FP64 if prec == "fp64" else ag.AG_FP32_PAIRS
        a, j, T = _direct(ag, L, x, v, m, eps, p, act)
        ar, jr, Tr = orc.direct(x, v, m, eps, 1.0, rows, box=L)
        if act is not None:
            other = np.setdiff1d(np.arange(n), act)
            assert np.all(np.isnan(a[other]))
        if prec == "fp64":
            sa, sj, st = _scales(orc, x, v, m, eps, rows, L)
            assert np.max(np.abs(a[rows] - ar).max(axis=1) / sa) <= 1e-12
            assert np.max(np.abs(j[rows] - jr).max(axis=1) / sj) <= 1e-12
            assert np.max(np.abs(T[rows] - Tr).max(axis=1) / st) <= 1e-12
        else:
            assert np.median(rel_err(a[rows], ar)) <= 1e-5
            assert np.median(tensor_rel_err(T[rows], Tr)) <= 1e-4


def _tree_case(name):
    if name == "clumps":
        x, v, m = _clumps_in_box(1 << 15)
        return x, v, m, 1.0, 1e-3
    if name == "pancake":
        x, v, m = workloads.zeldovich_box(32, box=2.0)
        return x, v, m, 2.0, 2.0 / 32 / 8
    rng = np.random.default_rng(7)
    n = 1 << 15
    return rng.uniform(0, 1, (n, 3)), rng.normal(size=(n, 3)), np.full(n, 1.0 / n), 1.0, 1e-3


@pytest.mark.parametrize("name", ["clumps", "pancake", "uniform"])
@pytest.mark.parametrize("theta", [0.5, 0.7])
def test_tree_periodic(ag, orc, name, theta):
    x, v, m, L, eps = _tree_case(name)
    n = len(m)
    a, j, T = _tree(ag, L, x, v, m, theta, eps)
    assert np.isfinite(a).all() and np.isfinite(j).all() and np.isfinite(T).all()
    rows = np.random.default_rng(11).choice(n, 2048, replace=False)
    ar, jr, Tr = orc.direct(x, v, m, eps, 1.0, rows, box=L)
    ea, ej, et = rel_err(a[rows], ar), rel_err(j[rows], jr), tensor_rel_err(T[rows], Tr)
    print(f"\n{name} theta={theta} relative: median", [float(np.median(e)) for e in (ea, ej, et)],
          "p99", [float(np.percentile(e, 99)) for e in (ea, ej, et)])
    if name == "clumps":
        assert np.median(ea) <= 1e-3 and np.percentile(ea, 99) <= 1e-2
        assert np.median(et) <= 5e-3 and np.percentile(et, 99) <= 5e-2
        assert np.median(ej) <= 1.5e-2 and np.percentile(ej, 99) <= 1e-1
        return
    # A uniform box has no mean field and a uniform sheet no tide off the
    # sheet: g, j and T are near-cancelling sums there, and a relative error
    # is ill-conditioned.  Measure them against their cancellation-free sizes
    # (sum of |pair terms|), at the tree's bounds for each quantity.  (The
    # lattice's T outliers at theta = 0.7 are the same with open boundaries.)
    sa, sj, st = _scales(orc, x, v, m, eps, rows, L)
    w = np.array([1, 1, 1, 2, 2, 2], dtype=float)
    ea = np.linalg.norm(a[rows] - ar, axis=1) / sa
    et = np.sqrt(((T[rows] - Tr) ** 2 * w).sum(1)) / st
    ej = np.linalg.norm(j[rows] - jr, axis=1) / sj
    print(f"{name} theta={theta} against cancellation-free sizes: median",
          [float(np.median(e)) for e in (ea, ej, et)], "p99", [float(np.percentile(e, 99)) for e in (ea, ej, et)])
    assert np.median(ea) <= 1e-3 and np.percentile(ea, 99) <= 1e-2
    assert np.median(et) <= 5e-3 and np.percentile(et, 99) <= 5e-2
    assert np.median(ej) <= 1.5e-2 and np.percentile(ej, 99) <= 1e-1


def test_tree_periodic_theta0_is_direct(ag, orc):
    """theta = 0 opens every node: every pair at its nearest image, FP32 pair terms."""
    x, v, m = _clumps_in_box(4099, seed=8)
    a, j, T = _tree(ag, 1.0, x, v, m, 0.0, 1e-3)
    ar, jr, Tr = orc.direct(x, v, m, 1e-3, 1.0, box=1.0)
    assert np.median(rel_err(a, ar)) <= 1e-5
    assert np.median(tensor_rel_err(T, Tr)) <= 1e-4


def test_tree_periodic_subset(ag, orc):
    """Only the listed rows are written; they match a full evaluation's
    quality."""
    x, v, m, L, eps = _tree_case("clumps")
    n = len(m)
    act = np.sort(np.random.default_rng(2).choice(n, 5000, replace=False))
    a, j, T = _tree(ag, L, x, v, m, 0.7, eps, active=act)
    rest = np.setdiff1d(np.arange(n), act)
    assert np.all(np.isnan(a[rest])) and np.all(np.isnan(T[rest]))
    rows = act[:1024]
    ar, _, _ = orc.direct(x, v, m, eps, 1.0, rows, box=L)
    assert np.median(rel_err(a[rows], ar)) <= 1e-3


def test_large_box_matches_open(ag, orc):
    """In a box far larger than the set (which lies inside it) no pair is
    wrapped: the periodic tree approximates the open-boundary sum."""
    x, v, m, _ = workloads.clumps(1 << 14, seed=4)
    x = x - x.min(axis=0) + 1.0
    a1, _, T1 = _tree(ag, 8.0, x, v, m, 0.7, 1e-3)
    rows = np.random.default_rng(1).choice(len(m), 1024, replace=False)
    ar, _, Tr = orc.direct(x, v, m, 1e-3, 1.0, rows)
    assert np.median(rel_err(a1[rows], ar)) <= 1e-3
    assert np.median(tensor_rel_err(T1[rows], Tr)) <= 5e-3


def test_periodic_arguments(ag):
    x, v, m, _ = workloads.clumps(4096, seed=4)
    with ag.Context(0) as c:
        for bad in (-1.0, float("inf"), float("nan")):
            with pytest.raises(ag.AgError) as e:
                c.set_periodic(bad)
            assert e.value.code == ag.AG_EINVAL
        c.set_periodic(1.0)
        c.tree_build(_t(x), _t(v), _t(m), 16)
        w = torch.zeros((4096, 3), dtype=torch.float64, device=DEV)
        dx = torch.zeros_like(w)
        dm = torch.zeros(4096, dtype=torch.float64, device=DEV)
        with pytest.raises(ag.AgError) as e:
            c.grav_backward(None, w, 0.7, 1e-3, 1.0, dx, dm)
        assert e.value.code == ag.AG_ESTATE
        c.set_periodic(0.0)
        with pytest.raises(ag.AgError) as e:     # the tree was built in the box
            c.grav_backward(None, w, 0.7, 1e-3, 1.0, dx, dm)
        assert e.value.code == ag.AG_ESTATE
        c.tree_build(_t(x), _t(v), _t(m), 16)
        c.grav_backward(None, w, 0.7, 1e-3, 1.0, dx, dm)
        c.sync()


# ---- Ewald sums (g and T of all images; j stays nearest-image) ----------

def _tree_ewald(ag, box, x, v, m, theta, eps, ewald_open=None, active=None):
    with ag.Context(0) as c:
        c.set_periodic(box, ewald=True)
        if ewald_open is not None:
            c.set_option(ag.AG_OPT_EWALD_OPEN, ewald_open)
        c.tree_build(_t(x), _t(v), _t(m), 16)
        out = _outputs(len(m))
        ia = None if active is None else _t(active, torch.int32)
        c.grav_eval(ia, theta, eps, 1.0, *out)
        c.sync()
    return [o.cpu().numpy() for o in out]


def _uniform(n, seed=7):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, (n, 3)), rng.normal(size=(n, 3)), np.full(n, 1.0 / n)


@pytest.mark.parametrize("name", ["clumps", "uniform"])
def test_ewald_theta0(ag, orc, name):
    """theta = 0 and a correction walk opened down to 1/64 of the distance to
    the image points: the periodic direct sum up to FP32 pair terms and the
    table."""
    if name == "clumps":
        x, v, m = _clumps_in_box(4096, seed=9)
    else:
        x, v, m = _uniform(4096)
    a, j, T = _tree_ewald(ag, 1.0, x, v, m, 0.0, 1e-3, ewald_open=64)
    rows = np.random.default_rng(3).choice(len(m), 256, replace=False)
    ar, jr, Tr = orc.direct(x, v, m, 1e-3, 1.0, rows, box=1.0, ewald=True)
    # the images add a field of order G M / L^2 that the single images' sum
    # of |pair terms| leaves out: it joins the scale
    sa = orc.abs_scale(x, m, 1e-3, 1.0, rows, box=1.0) + m.sum()
    ea = np.linalg.norm(a[rows] - ar, axis=1) / sa
    et = tensor_rel_err(T[rows], Tr)
    print(f"\nEwald theta=0 {name}: g vs abs scale median {np.median(ea):.2e} max {ea.max():.2e}; "
          f"g relative median {np.median(rel_err(a[rows], ar)):.2e}; T relative median {np.median(et):.2e}")
    assert np.median(ea) <= 1e-6 and ea.max() <= 1e-4
    assert np.median(et) <= 1e-4
    # the jerk is the nearest-image one
    _, jn, _ = orc.direct(x, v, m, 1e-3, 1.0, rows, box=1.0)
    assert np.median(rel_err(j[rows], jn)) <= 1e-5


@pytest.mark.parametrize("name", ["clumps", "pancake", "uniform"])
def test_ewald_tree(ag, orc, name):
    if name == "clumps":
        x, v, m = _clumps_in_box(8192, seed=10)
        L, eps = 1.0, 1e-3
    elif name == "pancake":
        x, v, m = workloads.zeldovich_box(20, box=1.0)
        L, eps = 1.0, 1.0 / 20 / 8
    else:
        x, v, m = _uniform(8192)
        L, eps = 1.0, 1e-3
    a, j, T = _tree_ewald(ag, L, x, v, m, 0.7, eps)
    rows = np.random.default_rng(4).choice(len(m), 256, replace=False)
    ar, jr, Tr = orc.direct(x, v, m, eps, 1.0, rows, box=L, ewald=True)
    ea, et = rel_err(a[rows], ar), tensor_rel_err(T[rows], Tr)
    sa, sj, st = _scales(orc, x, v, m, eps, rows, L)
    # plus the images' field and tide, of order G M / L^2 and G M / L^3
    sa, st = sa + m.sum() / L**2, st + m.sum() / L**3
    w = np.array([1, 1, 1, 2, 2, 2], dtype=float)
    eas = np.linalg.norm(a[rows] - ar, axis=1) / sa
    ets = np.sqrt(((T[rows] - Tr) ** 2 * w).sum(1)) / st
    print(f"\nEwald tree {name}: relative g median {np.median(ea):.2e} p99 {np.percentile(ea, 99):.2e}, "
          f"T median {np.median(et):.2e} p99 {np.percentile(et, 99):.2e}; against the cancellation-free "
          f"sizes g {np.median(eas):.2e} / {np.percentile(eas, 99):.2e}, T {np.median(ets):.2e} / "
          f"{np.percentile(ets, 99):.2e}")
    if name == "clumps":
        assert np.median(ea) <= 1e-3 and np.percentile(ea, 99) <= 1e-2
        assert np.median(et) <= 5e-3 and np.percentile(et, 99) <= 5e-2
    else:
        assert np.median(eas) <= 1e-3 and np.percentile(eas, 99) <= 1e-2
        assert np.median(ets) <= 5e-3 and np.percentile(ets, 99) <= 5e-2


def test_ewald_lattice(ag, orc):
    """A perfect lattice is the uniform box: no force, and the tide of the
    mean density, (4 pi / 3) G M / L^3 per axis, off-diagonals zero.  The
    mean tide is exact up to rounding.  Per particle, the walk's g and T
    differ from these by the tree's truncation error, which scales with the
    cancellation-free size of the fields the two walks sum (the single image
    about the walk's image origin, of order the nearest-image size S, and the
    images' correction, of order G M / L^2, resp. G M / L^3) and, at
    quadrupole order, with theta^3: the tree bounds at theta = 0.7 (g median
    1e-3, T median 5e-3; 99th percentiles 1e-2, 5e-2, taken here as the
    maximum over the sample) times (theta / 0.7)^3."""
    k, L, theta = 24, 2.0, 0.5
    g = (np.arange(k) + 0.5) * L / k
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    n = len(x)
    m = np.full(n, 1.0 / n)
    eps = L / k / 8
    a, _, T = _tree_ewald(ag, L, x, np.zeros_like(x), m, theta, eps)
    c = 4 * np.pi / 3 / L**3
    rows = np.random.default_rng(5).choice(n, 64, replace=False)
    sa, _, st = _scales(orc, x, np.zeros_like(x), m, eps, rows, L)
    sa, st = sa + 1.0 / L**2, st + 1.0 / L**3
    ea = np.linalg.norm(a[rows], axis=1) / sa
    dT = T[rows].copy()
    dT[:, :3] -= c
    w = np.array([1, 1, 1, 2, 2, 2], dtype=float)
    et = np.sqrt((dT**2 * w).sum(1)) / st
    f = (theta / 0.7) ** 3
    print(f"\nEwald lattice: T diag mean {T[:, :3].mean():.6e} vs {c:.6e}; max |g| {np.abs(a).max():.2e}; "
          f"against the cancellation-free sizes g median {np.median(ea):.2e} max {ea.max():.2e}, "
          f"T median {np.median(et):.2e} max {et.max():.2e}; bounds x {f:.3f}")
    # the mean tide is the background's, exactly up to rounding
    assert abs(T[:, :3].mean() - c) <= 1e-5 * c
    assert np.median(ea) <= 1e-3 * f and ea.max() <= 1e-2 * f
    assert np.median(et) <= 5e-3 * f and et.max() <= 5e-2 * f


def test_ewald_arguments(ag):
    x, v, m, _ = workloads.clumps(1024, seed=4)
    with ag.Context(0) as c:
        with pytest.raises(ag.AgError) as e:
            c.set_periodic(0.0, ewald=True)
        assert e.value.code == ag.AG_EINVAL
        c.set_periodic(1.0, ewald=True)
        out = _outputs(1024)
        with pytest.raises(ag.AgError) as e:
            c.grav_direct(_t(x), _t(v), _t(m), None, 1e-3, 1.0, *out)
        assert e.value.code == ag.AG_ESTATE
        for bad in (0, 65):
            with pytest.raises(ag.AgError) as e:
                c.set_option(ag.AG_OPT_EWALD_OPEN, bad)
            assert e.value.code == ag.AG_EINVAL
