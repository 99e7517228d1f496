"""GPU parity: the no-predictor ablation, the force log and the polynomial
predictor (Sec. 2.2, the alternative to Eq. 6) against the oracle.  The
log is pure data movement (bit-exact); the predictor's Lagrange sums are
FP64 in both, compared within a bound set by the weights' absolute sum."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
EPS64 = 2.0 ** -52


def _t(a, dtype=None):
    return torch.tensor(a, device=DEV) if dtype is None else torch.tensor(a, device=DEV, dtype=dtype)


def _events(rng, n, steps):
    """Log events (time, unique rows in random order); some rows are never
    logged, and some are logged twice at one time."""
    never = rng.choice(n, n // 50, replace=False)
    ev = []
    t = 0.0
    for s in range(steps):
        t += float(rng.uniform(0.05, 0.5))
        rows = rng.choice(n, int(rng.integers(1, n + 1)), replace=False)
        rows = np.setdiff1d(rows, never)
        rng.shuffle(rows)
        ev.append((t, rows))
        if s == steps // 2:   # a second log at the same time for a few rows
            ev.append((t, rows[: max(1, rows.size // 10)]))
    return ev


def _run_log(ctx, orc, n, depth, ev, rng):
    ha_o = np.zeros((depth, n, 3))
    ht_o = np.zeros((depth, n))
    hn_o = np.zeros(n, dtype=np.int32)
    ha = torch.zeros((depth, n, 3), dtype=torch.float64, device=DEV)
    ht = torch.zeros((depth, n), dtype=torch.float64, device=DEV)
    hn = torch.zeros(n, dtype=torch.int32, device=DEV)
    for t, rows in ev:
        a0 = rng.normal(size=(n, 3)) * np.exp(rng.uniform(-5, 5, (n, 1)))
        orc.force_log(ha_o, ht_o, hn_o, rows, a0, t)
        ctx.force_log(_t(a0), t, ha, ht, hn, idx=_t(rows.astype(np.int32)))
    ctx.sync()
    return (ha, ht, hn), (ha_o, ht_o, hn_o)


@pytest.mark.parametrize("n,depth", [(1, 1), (300, 2), (5001, 4)])
def test_force_log_bit_exact(ctx, orc, n, depth):
    rng = np.random.default_rng(n + depth)
    ev = _events(rng, n, 7)
    (ha, ht, hn), (ha_o, ht_o, hn_o) = _run_log(ctx, orc, n, depth, ev, rng)
    assert np.array_equal(hn.cpu().numpy(), hn_o)
    assert np.array_equal(ht.cpu().numpy(), ht_o)
    assert np.array_equal(ha.cpu().numpy(), ha_o)


def _check_poly(ctx, orc, log_gpu, log_orc, order, t, mask=None, rows=None):
    ha, ht, hn = log_gpu
    ha_o, ht_o, hn_o = log_orc
    n = hn.shape[0]
    fill = 12345.0
    out = torch.full((n, 3), fill, dtype=torch.float64, device=DEV)
    ctx.grav_predict_poly(ha, ht, hn, order, t, out, mask=None if mask is None else _t(mask))
    ctx.sync()
    got = out.cpu().numpy()
    if rows is None:
        rows = np.arange(n)
    sub = (ha_o[:, rows], ht_o[:, rows], hn_o[rows])
    ref = orc.predict_poly(*sub, order, t)
    wsum = orc.predict_poly_weight_sum(sub[1], sub[2], order, t)
    g = got[rows]
    on = np.ones(rows.size, dtype=bool) if mask is None else mask[rows] == 1
    logged = hn_o[rows] > 0
    use = on & logged
    # each weight carries <= 2 (order + 1) roundings, the sum order + 1 more
    scale = np.abs(ha_o[:, rows]).max(axis=(0, 2))
    tol = 4 * (order + 2) ** 2 * EPS64 * wsum * scale
    err = np.abs(g - ref).max(axis=1)
    assert np.all(err[use] <= tol[use]), (np.max(err[use] / np.maximum(tol[use], 1e-300)), order)
    if order == 0:
        assert np.array_equal(g[use], ref[use])
    assert np.all(g[~use] == fill)
    return use.sum()


@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_predict_poly_parity(ctx, orc, order):
    rng = np.random.default_rng(40 + order)
    n, depth = 20011, 4
    ev = _events(rng, n, 6)
    log_gpu, log_orc = _run_log(ctx, orc, n, depth, ev, rng)
    t_last = ev[-1][0]
    for t in (t_last, t_last + 0.01, t_last + 0.7):
        assert _check_poly(ctx, orc, log_gpu, log_orc, order, t) > n // 2
    mask = (rng.uniform(size=n) < 0.5).astype(np.uint8)
    _check_poly(ctx, orc, log_gpu, log_orc, order, t_last + 0.3, mask=mask)


def test_predict_poly_full_size_sampled(ctx, orc):
    """N = 2^22 (the clustered adaptive workload's size), linear predictor,
    checked on 4096 sampled rows."""
    rng = np.random.default_rng(9)
    n, depth = 1 << 22, 2
    ha = torch.zeros((depth, n, 3), dtype=torch.float64, device=DEV)
    ht = torch.zeros((depth, n), dtype=torch.float64, device=DEV)
    hn = torch.zeros(n, dtype=torch.int32, device=DEV)
    gen = torch.Generator(device=DEV).manual_seed(9)
    logs = []
    for t in (0.25, 0.5):
        a0 = torch.randn((n, 3), dtype=torch.float64, device=DEV, generator=gen)
        ctx.force_log(a0, t, ha, ht, hn)
        logs.append(a0)
    rows = np.sort(rng.choice(n, 4096, replace=False))
    # the oracle rebuilds the log of the sampled rows from the same inputs
    ha_o = np.zeros((depth, rows.size, 3))
    ht_o = np.zeros((depth, rows.size))
    hn_o = np.zeros(rows.size, dtype=np.int32)
    rr = torch.tensor(rows, device=DEV)
    for t, a0 in zip((0.25, 0.5), logs):
        orc.force_log(ha_o, ht_o, hn_o, np.arange(rows.size), a0[rr].cpu().numpy(), t)
    out = torch.zeros((n, 3), dtype=torch.float64, device=DEV)
    ctx.grav_predict_poly(ha, ht, hn, 1, 0.625, out)
    ctx.sync()
    ref = orc.predict_poly(ha_o, ht_o, hn_o, 1, 0.625)
    got = out[rr].cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=0, atol=64 * EPS64 * np.abs(ha_o).max())
    assert np.array_equal(hn.cpu().numpy(), np.full(n, 2, dtype=np.int32))


def test_no_predictor(ctx):
    """jerk = NULL: the force of the last evaluation, on the masked rows."""
    rng = np.random.default_rng(11)
    n = 4099
    a0 = rng.normal(size=(n, 3))
    mask = (rng.uniform(size=n) < 0.5).astype(np.uint8)
    out = torch.full((n, 3), 7.0, dtype=torch.float64, device=DEV)
    ctx.grav_predict(_t(a0), None, None, 3.0, out, mask=_t(mask))
    ctx.sync()
    got = out.cpu().numpy()
    assert np.array_equal(got[mask == 1], a0[mask == 1])
    assert np.all(got[mask == 0] == 7.0)


def test_predictor_argument_errors(ag, ctx):
    n = 10
    ha = torch.zeros((2, n, 3), dtype=torch.float64, device=DEV)
    ht = torch.zeros((2, n), dtype=torch.float64, device=DEV)
    hn = torch.zeros(n, dtype=torch.int32, device=DEV)
    a0 = torch.zeros((n, 3), dtype=torch.float64, device=DEV)
    for order in (-1, 2):
        with pytest.raises(ag.AgError) as e:
            ctx.grav_predict_poly(ha, ht, hn, order, 1.0, a0)
        assert e.value.code == ag.AG_EINVAL
    with pytest.raises(ag.AgError) as e:
        ctx.force_log(a0, float("nan"), ha, ht, hn)
    assert e.value.code == ag.AG_EINVAL
    deep = torch.zeros((5, n, 3), dtype=torch.float64, device=DEV)
    with pytest.raises(ag.AgError) as e:
        ctx.force_log(a0, 1.0, deep, torch.zeros((5, n), dtype=torch.float64, device=DEV), hn)
    assert e.value.code == ag.AG_EINVAL
    with pytest.raises(ag.AgError) as e:
        ctx.grav_predict(a0, a0, None, 1.0, a0)   # a jerk needs t0
    assert e.value.code == ag.AG_EINVAL
    # a row out of range is skipped and reported at the next sync
    ctx.force_log(a0, 1.0, ha, ht, hn, idx=torch.tensor([0, 3, n], dtype=torch.int32, device=DEV))
    with pytest.raises(ag.AgError) as e:
        ctx.sync()
    assert e.value.code == ag.AG_EDEVICE
    assert hn.cpu().numpy().tolist() == [1, 0, 0, 1] + [0] * (n - 4)
