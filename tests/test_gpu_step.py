"""GPU parity: tidal timestep and bins (Eq. 7), force-age bookkeeping
(Eq. 3, Eq. 4) and the predictor (Eq. 6).  Integer decisions are bit-exact
against the oracle on identical inputs."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _tensors(n, rng):
    T = rng.normal(size=(n, 6)) * np.exp(rng.uniform(-14, 14, (n, 1)))
    T[::97] = 0.0
    return T


@pytest.mark.parametrize("n", [1, 255, 4097, 100003])
def test_timestep_bins_bit_exact(ctx, orc, n):
    rng = np.random.default_rng(n)
    T = _tensors(n, rng)
    eta, dt_max, k_max = 0.01, 0.37, 40
    td = torch.tensor(T, device=DEV)
    dt = torch.empty(n, dtype=torch.float64, device=DEV)
    b = torch.empty(n, dtype=torch.int8, device=DEV)
    ctx.grav_timestep(td, eta, dt_max, k_max, dt, b)
    ctx.sync()
    dtr, br = orc.timestep(T, eta, dt_max, k_max)
    assert np.array_equal(b.cpu().numpy(), br)
    d = dt.cpu().numpy()
    fin = np.isfinite(dtr)
    assert np.array_equal(np.isfinite(d), fin)
    np.testing.assert_allclose(d[fin], dtr[fin], rtol=4e-16 * 8)


def test_timestep_bin_edges(ctx, orc):
    """Exact powers of 16 in Q stay in their bin; one ulp more goes deeper."""
    rows = []
    for k in range(12):
        t = 0.5 * 4.0**k
        tn = np.nextafter(t, np.inf)
        rows += [[0, 0, 0, t, t, t], [0, 0, 0, tn, tn, tn]]
    T = np.array(rows)
    td = torch.tensor(T, device=DEV)
    dt = torch.empty(len(T), dtype=torch.float64, device=DEV)
    b = torch.empty(len(T), dtype=torch.int8, device=DEV)
    ctx.grav_timestep(td, 0.5, 1.0, 40, dt, b)
    ctx.sync()
    got = b.cpu().numpy()
    assert got.tolist() == [k + e for k in range(12) for e in (0, 1)]
    assert np.array_equal(got, orc.timestep(T, 0.5, 1.0, 40)[1])


def test_timestep_subset_and_nonfinite(ctx, orc):
    rng = np.random.default_rng(5)
    n = 1000
    T = _tensors(n, rng)
    T[3, 0] = np.nan
    T[4, 2] = np.inf
    idx = np.sort(rng.choice(n, 300, replace=False)).astype(np.int32)
    idx = np.union1d(idx, [3, 4]).astype(np.int32)
    td = torch.tensor(T, device=DEV)
    dt = torch.full((n,), -1.0, dtype=torch.float64, device=DEV)
    b = torch.full((n,), -1, dtype=torch.int8, device=DEV)
    ctx.grav_timestep(td, 0.01, 2.0, 25, dt, b, idx=torch.tensor(idx, device=DEV))
    ctx.sync()
    bb = b.cpu().numpy()
    _, br = orc.timestep(T, 0.01, 2.0, 25)
    assert np.array_equal(bb[idx], br[idx])
    rest = np.setdiff1d(np.arange(n), idx)
    assert np.all(bb[rest] == -1) and np.all(dt.cpu().numpy()[rest] == -1.0)
    assert bb[3] == 25 and bb[4] == 25


@pytest.mark.parametrize("n,q", [(1, 0.5), (5000, 0.0), (5000, 0.125), (70001, 0.5), (70001, 1.0),
                                 (70001, 1.5)])
def test_select_bit_exact_over_steps(ctx, orc, n, q):
    rng = np.random.default_rng(n + int(q * 8))
    K = 6
    bins = rng.integers(0, K + 3, n).astype(np.int8)
    tf = rng.integers(0, 2 ** K, n).astype(np.int64)
    tfd = torch.tensor(tf, device=DEV)
    bd = torch.tensor(bins, device=DEV)
    act = torch.empty(n, dtype=torch.int32, device=DEV)
    cnt = torch.empty(1, dtype=torch.int64, device=DEV)
    tf_ref = tf.copy()
    for step in range(5):
        step_ticks = 1 + (step % 2)
        ctx.adaptive_select(tfd, bd, step_ticks, K, q, act, cnt)
        ctx.sync()
        tf_ref, _, idx_ref = orc.select(tf_ref, bins, step_ticks, K, q)
        k = int(cnt.item())
        assert k == idx_ref.size
        assert np.array_equal(act[:k].cpu().numpy(), idx_ref)
        assert np.array_equal(tfd.cpu().numpy(), tf_ref)


def test_predictor_bit_exact(ctx, orc):
    rng = np.random.default_rng(7)
    n = 50001
    a0 = rng.normal(size=(n, 3))
    j = rng.normal(size=(n, 3)) * 10
    t0 = rng.uniform(0, 1, n)
    t = 1.375
    out = torch.empty((n, 3), dtype=torch.float64, device=DEV)
    ctx.grav_predict(torch.tensor(a0, device=DEV), torch.tensor(j, device=DEV),
                     torch.tensor(t0, device=DEV), t, out)
    ctx.sync()
    assert np.array_equal(out.cpu().numpy(), orc.predict(a0, j, t0, t))


def test_predictor_mask_and_alias(ctx, orc):
    rng = np.random.default_rng(8)
    n = 777
    a0 = rng.normal(size=(n, 3))
    j = rng.normal(size=(n, 3))
    t0 = rng.uniform(0, 1, n)
    mask = (rng.uniform(size=n) < 0.5).astype(np.uint8)
    buf = torch.tensor(a0, device=DEV)
    ctx.grav_predict(buf, torch.tensor(j, device=DEV), torch.tensor(t0, device=DEV), 2.0, buf,
                     mask=torch.tensor(mask, device=DEV))
    ctx.sync()
    ref = orc.predict(a0, j, t0, 2.0)
    got = buf.cpu().numpy()
    assert np.array_equal(got[mask == 1], ref[mask == 1])
    assert np.array_equal(got[mask == 0], a0[mask == 0])
