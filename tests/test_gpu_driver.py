"""GPU tests of the adaptive integrator (Sec. 2 scheme around the solver), the
kick-drift kernel, graph capture/replay and the launch options."""
import numpy as np
import pytest
import torch

import workloads
from conftest import rel_err

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _t(a, dtype=None):
    return torch.tensor(a, device=DEV) if dtype is None else torch.tensor(a, dtype=dtype, device=DEV)


def test_kick_drift_bit_exact(ctx):
    rng = np.random.default_rng(1)
    n = 10001
    x, v, a = rng.normal(size=(3, n, 3))
    tx, tv = _t(x), _t(v)
    ctx.kick_drift(tx, tv, _t(a), 0.125, 0.37)
    ctx.sync()
    v2 = v + a * 0.125
    x2 = x + v2 * 0.37
    assert np.array_equal(tv.cpu().numpy(), v2)
    assert np.array_equal(tx.cpu().numpy(), x2)


def test_select_stamps_t0(ctx, orc):
    rng = np.random.default_rng(2)
    n = 5000
    bins = rng.integers(0, 6, n).astype(np.int8)
    tf = rng.integers(0, 32, n).astype(np.int64)
    t0 = rng.uniform(0, 1, n)
    tt0 = _t(t0)
    tfd = _t(tf)
    act = torch.empty(n, dtype=torch.int32, device=DEV)
    cnt = torch.empty(1, dtype=torch.int64, device=DEV)
    ctx.adaptive_select(tfd, _t(bins), 1, 5, 0.5, act, cnt, t0=tt0, t=7.25)
    ctx.sync()
    _, mask, idx = orc.select(tf, bins, 1, 5, 0.5)
    got = tt0.cpu().numpy()
    assert np.all(got[idx] == 7.25)
    assert np.array_equal(got[mask == 0], t0[mask == 0])


def _clumps(n):
    x, v, m, _ = workloads.clumps(n, seed=3)
    return _t(x), _t(v), _t(m), (x, v, m)


def test_adaptive_counts_and_force_error(ag, orc):
    from paper_2010_13792_amd.driver import AdaptiveIntegrator
    n = 1 << 14
    tx, tv, tm, (x, v, m) = _clumps(n)
    steps = 12
    with ag.Context(0) as c:
        base = AdaptiveIntegrator(c, tx, tv, tm, q_f=0.0, theta=0.5, eps=1e-3)
        for _ in range(steps):
            assert base.step() == n          # q_f = 0: the every-step scheme
        ad = AdaptiveIntegrator(c, tx, tv, tm, q_f=0.5, theta=0.5, eps=1e-3)
        counts = [ad.step() for _ in range(steps)]
        c.sync()
        assert sum(counts) < steps * n
        # the deepest bin holds particles, and they are refreshed every step
        assert min(counts) > 0
        xs = ad.x.cpu().numpy()
        vs = ad.vpred.cpu().numpy()
        rows = np.random.default_rng(3).choice(n, 1024, replace=False)
        ar, _, _ = orc.direct(xs, vs, m, 1e-3, 1.0, rows)
        err = rel_err(ad.acc.cpu().numpy()[rows], ar)
        assert np.median(err) < 2e-3


def test_adaptive_relative_opening(ag, orc):
    """The integrator with the relative opening test: the fresh forces of the
    last step's active rows against the oracle's direct sum at the same
    positions, and more accurate than the geometric test alone."""
    from paper_2010_13792_amd.driver import AdaptiveIntegrator
    n = 1 << 14
    tx, tv, tm, (x, v, m) = _clumps(n)
    errs = {}
    with ag.Context(0) as c:
        for alpha in (0.0, 0.0025):
            ad = AdaptiveIntegrator(c, tx, tv, tm, q_f=0.5, theta=0.7, eps=1e-3, opening_alpha=alpha)
            for _ in range(6):
                k = ad.step()
            c.sync()
            rows = ad.active[:k].cpu().numpy().astype(np.int64)[:1024]
            ar, _, _ = orc.direct(ad.x.cpu().numpy(), ad.vpred.cpu().numpy(), m, 1e-3, 1.0, rows)
            errs[alpha] = rel_err(ad.a0.cpu().numpy()[rows], ar)
    assert np.percentile(errs[0.0025], 99) <= 2.5e-3
    assert np.percentile(errs[0.0025], 99) < np.percentile(errs[0.0], 99)


def test_adaptive_softening_integrator(ag, orc):
    """Lengths from the device each step (32nd neighbour): the fresh forces
    of the last step's active rows against the oracle's mean-kernel sum with
    the lengths the evaluation used, and a bit-exact resume."""
    from paper_2010_13792_amd.driver import AdaptiveIntegrator
    n = 1 << 13
    tx, tv, tm, (x, v, m) = _clumps(n)
    kw = dict(q_f=0.5, theta=0.6, eps=1e-3, soft_k=32)
    with ag.Context(0) as c:
        ad = AdaptiveIntegrator(c, tx, tv, tm, **kw)
        for _ in range(4):
            ad.step()
        h_used = ad.h.cpu().numpy().copy()      # set after the 4th step's tree: used by the 5th
        k = ad.step()
        c.sync()
        xs = ad.x.cpu().numpy()
        rows = ad.active[:k].cpu().numpy().astype(np.int64)[:1024]
        ar, _, _ = orc.direct_soft(xs, ad.vpred.cpu().numpy(), m, h_used, 1.0, rows)
        err = rel_err(ad.a0.cpu().numpy()[rows], ar)
        assert np.median(err) <= 1e-3 and np.percentile(err, 99) <= 1e-2
        # the lengths set after the last build are those of its positions
        np.testing.assert_array_equal(ad.h.cpu().numpy(), orc.neighbour_length(xs, 32))
        # resume
        a = AdaptiveIntegrator(c, tx, tv, tm, **kw)
        for _ in range(4):
            a.step()
        saved = a.state()
        ref = [a.step() for _ in range(2)]
        c.sync()
        ref_state = a.state()
        r = AdaptiveIntegrator(c, tx, tv, tm, **kw)
        r.restore(saved)
        got = [r.step() for _ in range(2)]
        c.sync()
        assert got == ref
        for key in ["x", "v", "acc", "h"]:
            assert torch.equal(r.state()[key], ref_state[key]), key


def _move(v, dev):
    if torch.is_tensor(v):
        return v.to(dev)
    if isinstance(v, tuple):
        return tuple(_move(a, dev) for a in v)
    return v




def test_pm_softening_integrator(ag, orc):
    """Price & Monaghan softening in the integrator (theta = 0, so the walk
    is the direct sum up to its FP32 coordinates): the fresh forces at the
    start and on the third step's active rows against the oracle's mean-kernel
    sum plus correction, with the lengths solved at those positions."""
    from paper_2010_13792_amd.driver import AdaptiveIntegrator
    n, n_ngb = 1200, 32.0
    tx, tv, tm, (x, v, m) = _clumps(n)
    with ag.Context(0) as c:
        ad = AdaptiveIntegrator(c, tx, tv, tm, q_f=0.5, theta=0.0, eps=1e-3, soft_pm=n_ngb)
        c.sync()
        for label, xs, vs, rows in [("start", x, v, np.arange(n))]:
            hr = orc.pm_lengths(xs, n_ngb)
            np.testing.assert_allclose(ad.h.cpu().numpy(), hr, rtol=1e-12)
            ar = orc.direct_soft(xs, vs, m, hr, 1.0, rows)[0] + orc.pm_correction(xs, m, hr, n_ngb, 1.0)[rows]
            err = rel_err(ad.a0.cpu().numpy()[rows], ar)
            print(f"pm integrator {label}: max rel err {err.max():.2e}", flush=True)
            assert np.max(err) <= 1e-4
        for _ in range(2):
            ad.step()
        k = ad.step()
        c.sync()
        assert k > 0
        xs, vs = ad.x.cpu().numpy(), ad.vpred.cpu().numpy()
        rows = ad.active[:k].cpu().numpy().astype(np.int64)
        hr = orc.pm_lengths(xs, n_ngb)
        np.testing.assert_allclose(ad.h.cpu().numpy(), hr, rtol=1e-12)
        ar = orc.direct_soft(xs, vs, m, hr, 1.0, rows)[0] + orc.pm_correction(xs, m, hr, n_ngb, 1.0)[rows]
        err = rel_err(ad.a0.cpu().numpy()[rows], ar)
        print(f"pm integrator step 3 ({k} active): max rel err {err.max():.2e}", flush=True)
        assert np.max(err) <= 1e-4


@pytest.mark.parametrize("predictor", ["jerk", "linear"])
def test_adaptive_resume_bit_exact(ag, predictor):
    from paper_2010_13792_amd.driver import AdaptiveIntegrator
    n = 1 << 13
    tx, tv, tm, _ = _clumps(n)
    kw = dict(q_f=0.25, theta=0.6, eps=1e-3, predictor=predictor)
    with ag.Context(0) as c:
        a = AdaptiveIntegrator(c, tx, tv, tm, **kw)
        for _ in range(6):
            a.step()
        c.sync()
        ref = a.state()
        b = AdaptiveIntegrator(c, tx, tv, tm, **kw)
        for _ in range(3):
            b.step()
        saved = {k: _move(v, "cpu") for k, v in b.state().items()}
        r = AdaptiveIntegrator(c, tx, tv, tm, **kw)
        r.restore({k: _move(v, DEV) for k, v in saved.items()})
        for _ in range(3):
            r.step()
        c.sync()
        got = r.state()
        for k in ["x", "v", "acc", "tf", "bins", "t0"]:
            assert torch.equal(got[k], ref[k]), k
        assert got["evaluations"] == ref["evaluations"]


def test_predictor_variants(ag, orc):
    """Between updates (global step a quarter of the shortest gravity bin,
    q_f = 1/4), holding the last force (the ablation of Sec. 4.1) leaves a
    larger force error than the jerk predictor (Eq. 6).  A polynomial
    through the last fresh forces (Sec. 2.2) needs as many logged forces as
    its order + 1: on the rows that have them, it beats holding the newest
    logged force of the same log at the same state."""
    from paper_2010_13792_amd.driver import AdaptiveIntegrator
    n = 1 << 14
    tx, tv, tm, (x, v, m) = _clumps(n)
    rows = np.random.default_rng(5).choice(n, 2048, replace=False)
    errs = {}
    with ag.Context(0) as c:
        for p in ["none", "jerk", "linear", "quadratic"]:
            # bins of this set span 4 to 2048 ticks: at q_f = 1/4, by step 30
            # rows of span <= 64 ticks hold >= 2 logged forces and rows of
            # span 16 to 64 are extrapolated (not refreshed) at that step
            ad = AdaptiveIntegrator(c, tx, tv, tm, q_f=0.25, theta=0.5, eps=1e-3, step_shift=2, predictor=p)
            counts = [ad.step() for _ in range(30)]
            c.sync()
            assert 0 < sum(counts) < 30 * n
            ar, _, _ = orc.direct(ad.x.cpu().numpy(), ad.vpred.cpu().numpy(), m, 1e-3, 1.0, rows)
            e = rel_err(ad.acc.cpu().numpy()[rows], ar)
            errs[p] = float(np.median(e))
            if ad.log is None:
                continue
            ha, ht, hn = ad.log
            hold = torch.empty_like(ad.acc)
            c.grav_predict_poly(ha, ht, hn, 0, ad.t, hold)
            c.sync()
            # rows whose log is full and whose force in use is extrapolated
            full = np.nonzero((hn.cpu().numpy() == ad.order + 1) & (ht[0].cpu().numpy() < ad.t))[0]
            assert full.size >= 256
            full = full[:1024]
            af, _, _ = orc.direct(ad.x.cpu().numpy(), ad.vpred.cpu().numpy(), m, 1e-3, 1.0, full)
            ep = np.median(rel_err(ad.acc.cpu().numpy()[full], af))
            e0 = np.median(rel_err(hold.cpu().numpy()[full], af))
            errs[f"{p} ({full.size} rows with a full log)"] = float(ep)
            errs[f"held ({full.size} rows with a full log)"] = float(e0)
            assert ep < 0.5 * e0
    print("median force error by predictor:", errs)
    assert errs["jerk"] < 0.2 * errs["none"]
    assert errs["jerk"] < 2e-3


def test_graph_replay_matches_eager(ag):
    d = workloads.batched_plummer(nsys=8, seed=9, nmin=500, nmax=4000)
    x, v, m = d["x"], d["v"], d["m"]
    n = len(m)
    tx, tv, tm = _t(x), _t(v), _t(m)
    toff = _t(d["offsets"], torch.int64)
    tact = _t(d["active"], torch.int32)
    acc = torch.zeros((n, 3), dtype=torch.float64, device=DEV)
    jerk, tid = torch.zeros_like(acc), torch.zeros((n, 6), dtype=torch.float64, device=DEV)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream), ag.Context(0, stream) as c:
        c.tree_build_batched(tx, tv, tm, toff, 16)
        c.grav_eval_batched(tact, 0.5, 0.01, 1.0, acc, jerk, tid)
        c.sync()
        eager = acc.clone()
        c.graph_begin()
        c.tree_build_batched(tx, tv, tm, toff, 16)
        c.grav_eval_batched(tact, 0.5, 0.01, 1.0, acc, jerk, tid)
        c.graph_end()
        for rep in range(3):
            acc.zero_()
            stream.synchronize()
            c.graph_replay()
            c.sync()
            assert torch.equal(acc, eager), rep
        # new positions in place, replay again: same as an eager run on them
        tx.mul_(1.5)
        c.graph_replay()
        c.sync()
        replayed = acc.clone()
        c.tree_build_batched(tx, tv, tm, toff, 16)
        c.grav_eval_batched(tact, 0.5, 0.01, 1.0, acc, jerk, tid)
        c.sync()
        assert torch.equal(acc, replayed)


def test_options(ag, ctx):
    x, v, m = workloads.plummer(3000, seed=4)
    res = []
    for waves, small in [(16, 2), (4, 2), (8, 8)]:
        ctx.set_option(ag.AG_OPT_WALK_WAVES_PER_CU, waves)
        ctx.set_option(ag.AG_OPT_SMALL_NODE, small)
        ctx.tree_build(_t(x), _t(v), _t(m), 16)
        acc = torch.zeros((3000, 3), dtype=torch.float64, device=DEV)
        ctx.grav_eval(None, 0.6, 0.01, 1.0, acc, None, None)
        ctx.sync()
        res.append(acc.cpu().numpy())
    ctx.set_option(ag.AG_OPT_WALK_WAVES_PER_CU, 16)
    ctx.set_option(ag.AG_OPT_SMALL_NODE, 2)
    # the number of resident waves only changes which wave walks which group
    assert np.array_equal(res[0], res[1])
    # summing small accepted nodes pairwise only changes the approximation
    assert np.median(rel_err(res[2], res[0])) < 1e-3
    with pytest.raises(ag.AgError):
        ctx.set_option(ag.AG_OPT_WALK_WAVES_PER_CU, 0)
    with pytest.raises(ag.AgError):
        ctx.set_option(99, 1)


@pytest.mark.gpu
def test_mac_offset_option(ag, ctx, orc):
    """The offset-aware opening test opens at least as many nodes and keeps
    the tree force within the tolerance of the oracle's direct sum; it is
    never less accurate in the median on a clustered set."""
    x, v, m, _ = workloads.clumps(20000, seed=8, nclump=8)
    n = len(m)
    rows = np.random.default_rng(1).choice(n, 512, replace=False)
    ar, _, _ = orc.direct(x, v, m, 1e-3, 1.0, rows)
    out = {}
    for off in (0, 1):
        ctx.set_option(ag.AG_OPT_MAC_OFFSET, off)
        ctx.tree_build(_t(x), _t(v), _t(m), 16)
        acc = torch.zeros((n, 3), dtype=torch.float64, device=DEV)
        ctx.stats_reset()
        ctx.grav_eval(None, 0.7, 1e-3, 1.0, acc, None, None)
        st = ctx.stats_read()
        out[off] = (rel_err(acc.cpu().numpy()[rows], ar), st["n_pp"] + st["n_pn"])
    ctx.set_option(ag.AG_OPT_MAC_OFFSET, 1)
    assert out[1][1] >= out[0][1]
    for off in (0, 1):
        assert np.median(out[off][0]) < 1e-3 and np.percentile(out[off][0], 99) < 1e-2
    assert np.median(out[1][0]) <= np.median(out[0][0])
    with pytest.raises(ag.AgError):
        ctx.set_option(ag.AG_OPT_MAC_OFFSET, 2)


@pytest.mark.gpu
def test_group_targets_option(ag, ctx, orc):
    """Groups of 64, 32 and 8 targets give the tree force within tolerance;
    smaller groups open fewer nodes per target (their boxes are smaller; a
    one-target group is the plain per-particle test, whose error at theta =
    0.7 is above the 1e-3 bound, so it is only checked for counts)."""
    x, v, m, _ = workloads.clumps(30000, seed=9, nclump=8)
    n = len(m)
    rows = np.random.default_rng(2).choice(n, 512, replace=False)
    ar, jr, _ = orc.direct(x, v, m, 1e-3, 1.0, rows)
    per_target = {}
    ctx.tree_build(_t(x), _t(v), _t(m), 16)
    for cap in (64, 32, 8, 1):
        ctx.set_option(ag.AG_OPT_GROUP_TARGETS, cap)
        acc = torch.zeros((n, 3), dtype=torch.float64, device=DEV)
        jerk = torch.zeros_like(acc)
        ctx.stats_reset()
        ctx.grav_eval(None, 0.7, 1e-3, 1.0, acc, jerk, None)
        st = ctx.stats_read()
        assert st["n_targets"] == n
        per_target[cap] = (st["n_pp"] + st["n_pn"]) / n
        if cap == 1:
            continue
        ea = rel_err(acc.cpu().numpy()[rows], ar)
        ej = rel_err(jerk.cpu().numpy()[rows], jr)
        assert np.median(ea) < 1e-3 and np.percentile(ea, 99) < 1e-2, cap
        assert np.median(ej) < 1.5e-2, cap
    ctx.set_option(ag.AG_OPT_GROUP_TARGETS, 64)
    assert per_target[1] <= per_target[32] <= per_target[64]
    with pytest.raises(ag.AgError):
        ctx.set_option(ag.AG_OPT_GROUP_TARGETS, 65)
