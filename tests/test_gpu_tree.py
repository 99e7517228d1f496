"""GPU parity: oct-tree build (topology invariants, node multipoles against the
oracle's brute-force moments) and the tree walk against the FP64 direct sum."""
import numpy as np
import pytest
import torch

import workloads
from conftest import rel_err, tensor_rel_err

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _t(a, dtype=None):
    return torch.tensor(a, device=DEV) if dtype is None else torch.tensor(a, dtype=dtype, device=DEV)


def _eval(ctx, x, v, m, theta, eps, G=1.0, active=None, n_leaf=16, build=True):
    n = len(m)
    if build:
        ctx.tree_build(_t(x), _t(v), _t(m), n_leaf)
    acc = torch.full((n, 3), float("nan"), dtype=torch.float64, device=DEV)
    jerk = torch.full((n, 3), float("nan"), dtype=torch.float64, device=DEV)
    tid = torch.full((n, 6), float("nan"), dtype=torch.float64, device=DEV)
    ia = None if active is None else _t(active, torch.int32)
    ctx.grav_eval(ia, theta, eps, G, acc, jerk, tid)
    ctx.sync()
    return acc.cpu().numpy(), jerk.cpu().numpy(), tid.cpu().numpy()


def _check_topology(link, mom, perm, n, n_leaf, x, v, m, orc, sample=300, cells=True):
    nn = link.shape[0]
    skip, start, cnt, lv = link[:, 0], link[:, 1], link[:, 2], link[:, 3]
    leaf = (lv & 0x100) != 0
    level = lv & 0xff
    # permutation
    assert np.array_equal(np.sort(perm), np.arange(n))
    # root covers everything; leaves tile [0, n) exactly once, in order
    assert start[0] == 0 and cnt[0] == n and skip[0] == nn
    ls = start[leaf]
    lc = cnt[leaf]
    assert np.all(lc >= 1)
    assert ls[0] == 0 and np.array_equal(ls[1:], (ls + lc)[:-1]) and ls[-1] + lc[-1] == n
    # leaves respect the capacity unless at the deepest level
    assert np.all((lc <= n_leaf) | (level[leaf] == 21))
    # every node's particles fit in a cell of its level: side / 2^level, with
    # side the root cube's (the largest extent of the whole set); not after a
    # refit, whose particles have moved since the cells were drawn
    if cells:
        side = (x.max(axis=0) - x.min(axis=0)).max() * (1 + 1e-9)
        ext = (mom[:, 22:25] - mom[:, 19:22]).max(axis=1)
        assert np.all(ext <= side * np.exp2(-level.astype(np.float64)))
    # pre-order: first child of an inner node is the next node, children tile the parent
    inner = np.nonzero(~leaf)[0]
    for i in inner[:2000]:
        ch = i + 1
        tot = 0
        pos = start[i]
        while ch < skip[i]:
            assert level[ch] > level[i] and start[ch] == pos
            pos += cnt[ch]
            tot += cnt[ch]
            ch = skip[ch]
        assert ch == skip[i] and tot == cnt[i]
    # node moments against brute force over the node's particles
    rng = np.random.default_rng(0)
    picks = np.concatenate([[0], rng.choice(nn, min(sample, nn), replace=False)])
    for i in picks:
        rows = perm[start[i]:start[i] + cnt[i]]
        ref = orc.moments(x, v, m, rows)
        got = mom[i]
        # natural sizes of the node: mass M, extent L, internal speed V; FP64
        # rounding of a centre of size |c| leaves |c| * 1e-16 offsets
        M = ref["M"]
        cx = max(1.0, np.abs(ref["com"]).max())
        ux = max(1.0, np.abs(ref["u"]).max())
        L = max((ref["hi"] - ref["lo"]).max(), 1e-15 * cx)
        V = max(np.abs(v[rows] - ref["u"]).max(), 1e-15 * ux)
        assert got[0] == pytest.approx(M, rel=1e-12)
        np.testing.assert_allclose(got[1:4], ref["com"], rtol=0, atol=1e-12 * cx)
        np.testing.assert_allclose(got[4:7], ref["u"], rtol=0, atol=1e-12 * ux)
        # 1e-28 M |c|^2: the floor left by centre-of-mass rounding (~1e-16 |c|)
        np.testing.assert_allclose(got[7:13], ref["Q"], rtol=0, atol=1e-9 * M * L * L + 1e-28 * M * cx * cx)
        np.testing.assert_allclose(got[13:19], ref["Qdot"], rtol=0,
                                   atol=1e-9 * M * L * V + 1e-28 * M * cx * max(ux, V))
        np.testing.assert_array_equal(got[19:22], ref["lo"])
        np.testing.assert_array_equal(got[22:25], ref["hi"])


@pytest.mark.parametrize("n,n_leaf,kind", [(1, 16, "plummer"), (17, 16, "plummer"), (5000, 16, "plummer"),
                                           (20000, 8, "sphere"), (30000, 32, "clumps")])
def test_tree_topology_and_moments(ctx, orc, n, n_leaf, kind):
    if kind == "plummer":
        x, v, m = workloads.plummer(n, seed=n)
    elif kind == "sphere":
        x, v, m = workloads.turbulent_sphere(n, seed=2, grid=32)
    else:
        x, v, m, _ = workloads.clumps(n, seed=3)
    m = m * np.random.default_rng(1).uniform(0.5, 1.5, n)
    ctx.tree_build(_t(x), _t(v), _t(m), n_leaf)
    link, mom, perm = (t.cpu().numpy() for t in ctx.tree_export())
    _check_topology(link, mom, perm, n, n_leaf, x, v, m, orc)


def test_tree_dense_cells(ctx, orc):
    """Cells far below the sorted key prefix holding more particles than a
    workgroup sorts in LDS (4000) and fewer (1500, 40): the tree is still the
    exact oct-tree of the full keys."""
    rng = np.random.default_rng(11)
    xp, vp, mp = workloads.plummer(8000, seed=11)
    balls = [rng.normal(scale=1e-7, size=(k, 3)) + rng.uniform(-1, 1, 3) for k in (4000, 1500, 40)]
    x = np.concatenate([xp] + balls)
    n = len(x)
    v = rng.normal(size=(n, 3))
    m = np.full(n, 1.0 / n)
    ctx.tree_build(_t(x), _t(v), _t(m), 16)
    link, mom, perm = (t.cpu().numpy() for t in ctx.tree_export())
    _check_topology(link, mom, perm, n, 16, x, v, m, orc, sample=500)
    a, _, _ = _eval(ctx, x, v, m, 0.6, 1e-3, build=False)
    rows = np.random.default_rng(12).choice(n, 512, replace=False)
    ar, _, _ = orc.direct(x, v, m, 1e-3, 1.0, rows)
    ea = rel_err(a[rows], ar)
    assert np.median(ea) < 1e-3 and np.percentile(ea, 99) < 1e-2


def test_tree_coincident_particles(ctx, orc):
    """More coincident particles than a leaf holds: the cell splits down to
    the deepest level and keeps them all in one leaf."""
    rng = np.random.default_rng(4)
    x = rng.normal(size=(500, 3))
    x[100:200] = x[7]
    v = rng.normal(size=(500, 3))
    m = np.full(500, 1 / 500)
    ctx.tree_build(_t(x), _t(v), _t(m), 8)
    link, mom, perm = (t.cpu().numpy() for t in ctx.tree_export())
    _check_topology(link, mom, perm, 500, 8, x, v, m, orc)
    a, j, t = _eval(ctx, x, v, m, 0.0, 0.05, build=False)
    ar, jr, tr = orc.direct(x, v, m, 0.05, 1.0)
    assert np.median(rel_err(a, ar)) < 1e-5


def test_tree_deterministic(ctx):
    x, v, m = workloads.turbulent_sphere(1 << 15, seed=2, grid=32)
    r1 = _eval(ctx, x, v, m, 0.7, 1e-3)
    l1 = ctx.tree_export()[0].cpu().numpy()
    r2 = _eval(ctx, x, v, m, 0.7, 1e-3)
    l2 = ctx.tree_export()[0].cpu().numpy()
    assert np.array_equal(l1, l2)
    for p, q in zip(r1, r2):
        assert np.array_equal(p, q)


@pytest.mark.parametrize("n", [100, 4096, 10007])
def test_walk_theta0_is_direct_sum(ctx, orc, n):
    """theta = 0 opens every node: the walk is the direct sum (FP32 pairs)."""
    x, v, m = workloads.plummer(n, seed=n)
    eps = 0.01
    a, j, t = _eval(ctx, x, v, m, 0.0, eps)
    ar, jr, tr = orc.direct(x, v, m, eps, 1.0)
    assert np.median(rel_err(a, ar)) <= 1e-5
    assert np.median(rel_err(j, jr)) <= 1e-5
    assert np.median(tensor_rel_err(t, tr)) <= 1e-5
    st = ctx.stats_read()
    assert st["n_pp"] > 0


@pytest.mark.parametrize("n_leaf", [1, 16, 64])
def test_walk_theta0_every_target_ragged(ctx, orc, n_leaf):
    """theta = 0 at ragged sizes (one target, partial tiles and groups, a
    few tiles): every target's g against the direct sum, measured against the
    cancellation-free size G sum_j m_j |f d|.  The walk holds coordinates in
    FP32 relative to the group centre, off by up to 2^-24 of the system size
    R, so a pair at the softening length carries up to ~2^-24 2R / eps
    relative error (5e-4 here, R <= 10, eps = 0.01; measured worst 5.3e-6);
    a missing or repeated pair moves a target by ~1/n of its scale or more,
    so the bound is 1e-4."""
    for n in (1, 2, 3, 63, 64, 65, 127, 1000, 4097):
        x, v, m = workloads.plummer(n, seed=100 + n)
        eps = 0.01
        a, j, t = _eval(ctx, x, v, m, 0.0, eps, n_leaf=n_leaf)
        ar, jr, tr = orc.direct(x, v, m, eps, 1.0)
        if n == 1:
            assert np.all(a == 0.0) and np.all(t == 0.0)
            continue
        sa = orc.abs_scale(x, m, eps, 1.0)
        e = np.linalg.norm(a - ar, axis=1) / sa
        assert e.max() <= 1e-4, (n, n_leaf, float(e.max()))


@pytest.mark.parametrize("split,pack", [(0, 0), (0, 1), (42, 1)])
def test_walk_group_split_and_pack(ag, ctx, orc, split, pack):
    """Groups of 33 .. 42 targets walked whole (AG_OPT_GROUP_SPLIT 0; the
    default walks them as two halves) and runs of children cut every 64
    targets (AG_OPT_GROUP_PACK): at theta = 0 every target still gets the
    direct sum (same bound as the default grouping, at ragged sizes); at
    theta = 0.7 the error against the oracle stays within the metric's bound
    and the group count differs from the default's; bad values are
    refused."""
    try:
        ctx.set_option(ag.AG_OPT_GROUP_SPLIT, split)
        ctx.set_option(ag.AG_OPT_GROUP_PACK, pack)
        for n in (40, 65, 1000, 4097):
            x, v, m = workloads.plummer(n, seed=300 + n)
            a, _, _ = _eval(ctx, x, v, m, 0.0, 0.01)
            ar, _, _ = orc.direct(x, v, m, 0.01, 1.0)
            e = np.linalg.norm(a - ar, axis=1) / orc.abs_scale(x, m, 0.01, 1.0)
            assert e.max() <= 1e-4, (n, float(e.max()))
        x, v, m = workloads.turbulent_sphere(1 << 15, seed=7, grid=32)
        rows = np.random.default_rng(3).choice(len(m), 256, replace=False)
        ar, _, _ = orc.direct(x, v, m, 1e-3, 1.0, rows)
        groups = {}
        for on in (False, True):   # against the default grouping (split 42, no packing)
            ctx.set_option(ag.AG_OPT_GROUP_SPLIT, split if on else 42)
            ctx.set_option(ag.AG_OPT_GROUP_PACK, pack if on else 0)
            ctx.stats_reset()
            a, _, _ = _eval(ctx, x, v, m, 0.7, 1e-3)
            st = ctx.stats_read()
            groups[on] = st["n_groups"]
            assert st["n_targets"] == len(m)
            e = rel_err(a[rows], ar)
            assert np.median(e) <= 1e-3 and np.percentile(e, 99) <= 1e-2, (on, np.median(e))
        assert groups[True] != groups[False]
        for bad in (-1, 1, 32, 65):
            with pytest.raises(ag.AgError):
                ctx.set_option(ag.AG_OPT_GROUP_SPLIT, bad)
        for bad in (-1, 2):
            with pytest.raises(ag.AgError):
                ctx.set_option(ag.AG_OPT_GROUP_PACK, bad)
    finally:
        ctx.set_option(ag.AG_OPT_GROUP_SPLIT, 42)
        ctx.set_option(ag.AG_OPT_GROUP_PACK, 0)


@pytest.mark.parametrize("theta", [0.5, 0.7])
def test_walk_accuracy_turbulent_sphere(ctx, orc, theta):
    """Uniform sphere with k^-4 velocities, N = 2^16, eps = 1e-3, on 4096
    sampled targets.  Acceleration: median relative error <= 1e-3, 99th
    percentile <= 1e-2.  Tidal tensor: the same expansion order, but T ~ 1/r^3
    weighs the nearest accepted nodes more than g ~ 1/r^2 does; it only sets
    dt ~ |T|^(-1/2) in power-of-two bins, so its bound is median <= 5e-3,
    99th percentile <= 5e-2.  Jerk: the node term carries the mean velocity
    and the quadrupole rate, one order lower in s/r than g (the next term is
    the octupole rate): median <= 1.5e-2, 99th percentile <= 1e-1."""
    n = 1 << 16
    x, v, m = workloads.turbulent_sphere(n, seed=2, grid=64)
    eps = 1e-3
    a, j, t = _eval(ctx, x, v, m, theta, eps)
    rows = np.random.default_rng(3).choice(n, 4096, replace=False)
    ar, jr, tr = orc.direct(x, v, m, eps, 1.0, rows)
    ea, ej, et = rel_err(a[rows], ar), rel_err(j[rows], jr), tensor_rel_err(t[rows], tr)
    stats = {k: (float(np.median(e)), float(np.percentile(e, 99))) for k, e in
             (("acc", ea), ("jerk", ej), ("tidal", et))}
    print(f"theta={theta}: {stats}")
    for k, (med, p99) in stats.items():
        lim = {"acc": (1e-3, 1e-2), "tidal": (5e-3, 5e-2), "jerk": (1.5e-2, 1e-1)}[k]
        assert med <= lim[0] and p99 <= lim[1], (k, med, p99)


def test_walk_plummer_clustered(ctx, orc):
    x, v, m, _ = workloads.clumps(1 << 16, seed=3)
    eps = 1e-3
    a, j, t = _eval(ctx, x, v, m, 0.7, eps)
    rows = np.random.default_rng(4).choice(len(m), 4096, replace=False)
    ar, jr, tr = orc.direct(x, v, m, eps, 1.0, rows)
    ea = rel_err(a[rows], ar)
    assert np.median(ea) <= 1e-3 and np.percentile(ea, 99) <= 1e-2


@pytest.mark.parametrize("frac", [0.003, 0.2, 0.77])
def test_walk_partial_active(ctx, orc, frac):
    n = 20011
    x, v, m = workloads.plummer(n, seed=5)
    act = np.random.default_rng(6).permutation(workloads.random_subset(n, frac, seed=7))
    a, j, t = _eval(ctx, x, v, m, 0.6, 0.01, active=act)
    other = np.setdiff1d(np.arange(n), act)
    assert np.all(np.isnan(a[other])) and np.all(np.isnan(j[other])) and np.all(np.isnan(t[other]))
    ar, jr, tr = orc.direct(x, v, m, 0.01, 1.0, act)
    ea = rel_err(a[act], ar)
    assert np.median(ea) <= 1e-3 and np.percentile(ea, 99) <= 1e-2
    st = ctx.stats_read()
    assert st["n_targets"] >= len(act)


def test_refit_after_drift(ctx, orc):
    """Refit with drifted positions and changed velocities (both read from
    the refit's own arrays): node moments, velocity moments included, and
    the forces match the oracle on the new state."""
    n = 30000
    x, v, m = workloads.plummer(n, seed=8)
    ctx.tree_build(_t(x), _t(v), _t(m), 16)
    x2 = x + 0.01 * v
    v2 = 1.3 * v + np.random.default_rng(9).normal(scale=0.05, size=v.shape)
    ctx.tree_refit(_t(x2), _t(v2), _t(m))
    link, mom, perm = (t.cpu().numpy() for t in ctx.tree_export())
    _check_topology(link, mom, perm, n, 16, x2, v2, m, orc, sample=100, cells=False)
    a, _, _ = _eval(ctx, x2, v2, m, 0.6, 0.01, build=False)
    rows = np.arange(0, n, 7)
    ar, _, _ = orc.direct(x2, v, m, 0.01, 1.0, rows)
    ea = rel_err(a[rows], ar)
    assert np.median(ea) <= 1e-3 and np.percentile(ea, 99) <= 1e-2


def test_batched_systems(ctx, orc):
    d = workloads.batched_plummer(nsys=12, seed=4, nmin=100, nmax=3000)
    x, v, m = d["x"], d["v"], d["m"]
    n = len(m)
    ctx.tree_build_batched(_t(x), _t(v), _t(m), _t(d["offsets"], torch.int64), 16)
    acc = torch.full((n, 3), float("nan"), dtype=torch.float64, device=DEV)
    jerk = torch.full_like(acc, float("nan"))
    tid = torch.full((n, 6), float("nan"), dtype=torch.float64, device=DEV)
    ctx.grav_eval_batched(_t(d["active"], torch.int32), 0.5, 0.01, 1.0, acc, jerk, tid)
    ctx.sync()
    a = acc.cpu().numpy()
    act = d["active"]
    other = np.setdiff1d(np.arange(n), act)
    assert np.all(np.isnan(a[other]))
    off = d["offsets"]
    for s in range(12):
        lo, hi = off[s], off[s + 1]
        rows = act[(act >= lo) & (act < hi)]
        ar, _, _ = orc.direct(x[lo:hi], v[lo:hi], m[lo:hi], 0.01, 1.0, rows - lo)
        ea = rel_err(a[rows], ar)
        assert np.median(ea) <= 1e-3 and np.percentile(ea, 99) <= 1e-2, s


def test_eval_errors(ag, orc):
    c = ag.Context(0)
    try:
        x, v, m = workloads.plummer(100, seed=1)
        acc = torch.zeros((100, 3), dtype=torch.float64, device=DEV)
        with pytest.raises(ag.AgError) as e:
            c.n = 100
            c.grav_eval(None, 0.5, 0.01, 1.0, acc, None, None)
        assert e.value.code == ag.AG_ESTATE
        c.tree_build(_t(x), _t(v), _t(m), 16)
        for th, ep in ((-0.1, 0.01), (0.5, 0.0), (0.5, -1.0)):
            with pytest.raises(ag.AgError) as e:
                c.grav_eval(None, th, ep, 1.0, acc, None, None)
            assert e.value.code == ag.AG_EINVAL
        # repeated and out-of-range active rows raise a device flag
        with pytest.raises(ag.AgError) as e:
            c.grav_eval(_t(np.array([1, 2, 2]), torch.int32), 0.5, 0.01, 1.0, acc, None, None)
            c.sync()
        assert e.value.code == ag.AG_EDEVICE
        with pytest.raises(ag.AgError) as e:
            c.grav_eval(_t(np.array([1, 100]), torch.int32), 0.5, 0.01, 1.0, acc, None, None)
            c.sync()
        assert e.value.code == ag.AG_EDEVICE
        # non-finite positions are reported
        xb = x.copy()
        xb[5, 1] = np.nan
        with pytest.raises(ag.AgError) as e:
            c.tree_build(_t(xb), _t(v), _t(m), 16)
            c.sync()
        assert e.value.code == ag.AG_ENONFINITE
        # still usable
        c.tree_build(_t(x), _t(v), _t(m), 16)
        c.grav_eval(None, 0.5, 0.01, 1.0, acc, None, None)
        c.sync()
        ar, _, _ = orc.direct(x, v, m, 0.01, 1.0)
        assert np.median(rel_err(acc.cpu().numpy(), ar)) < 1e-3
    finally:
        c.close()
