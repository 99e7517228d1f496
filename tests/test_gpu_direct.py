"""GPU parity: direct summation (FP64 and FP32 pairs) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import workloads
from conftest import rel_err, tensor_rel_err

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _run_direct(ag, ctx, x, v, m, eps, G, prec, active=None):
    n = len(m)
    tx, tv, tm = (torch.tensor(a, device=DEV) for a in (x, v, m))
    acc = torch.full((n, 3), float("nan"), dtype=torch.float64, device=DEV)
    jerk = torch.full((n, 3), float("nan"), dtype=torch.float64, device=DEV)
    tid = torch.full((n, 6), float("nan"), dtype=torch.float64, device=DEV)
    ia = None if active is None else torch.tensor(active, dtype=torch.int32, device=DEV)
    ctx.grav_direct(tx, tv, tm, ia, eps, G, acc, jerk, tid, precision=prec)
    ctx.sync()
    return acc.cpu().numpy(), jerk.cpu().numpy(), tid.cpu().numpy()


def _abs_scales(x, v, m, eps, rows):
    """Cancellation-free sizes sum_j m_j |term_j| of g, j and S at `rows`."""
    import oracle
    sa = oracle.abs_scale(x, m, eps, 1.0, rows)
    sj = np.empty(len(rows))
    st = np.empty(len(rows))
    f_of = lambda r: oracle.kernel(r, eps)
    for t, i in enumerate(rows):
        d = x - x[i]
        nu = v - v[i]
        r = np.linalg.norm(d, axis=1)
        f, D, _ = f_of(r)
        mm = m.copy()
        mm[i] = 0.0
        jt = f[:, None] * nu + (D * np.sum(d * nu, 1))[:, None] * d
        sj[t] = np.sum(mm * np.linalg.norm(jt, axis=1))
        st[t] = np.sum(mm * (3 * np.abs(f) + np.abs(D) * r * r))
    return sa, sj, st


def test_direct_fp64_plummer_4096(ag, ctx, orc):
    """Plummer sphere, N = 4096, eps = 0.01, all particles: the FP64 path agrees
    with the oracle to 1e-12 (median relative, and max against the
    cancellation-free scale sum_j m_j |f d|)."""
    x, v, m = workloads.plummer(4096, seed=1)
    eps, G = 0.01, 1.0
    a, j, t = _run_direct(ag, ctx, x, v, m, eps, G, ag.AG_FP64)
    ar, jr, tr = orc.direct(x, v, m, eps, G)
    ea, ej, et = rel_err(a, ar), rel_err(j, jr), tensor_rel_err(t, tr)
    assert np.median(ea) <= 1e-12 and np.median(ej) <= 1e-12 and np.median(et) <= 1e-12
    rows = np.arange(0, 4096, 37)
    sa, sj, st = _abs_scales(x, v, m, eps, rows)
    assert np.max(np.linalg.norm(a[rows] - ar[rows], axis=1) / sa) <= 1e-12
    assert np.max(np.linalg.norm(j[rows] - jr[rows], axis=1) / sj) <= 1e-12
    assert np.max(np.abs(t[rows] - tr[rows]).max(1) / st) <= 1e-12


def test_direct_fp32_pairs_plummer_4096(ag, ctx, orc):
    x, v, m = workloads.plummer(4096, seed=1)
    eps, G = 0.01, 1.0
    a, j, t = _run_direct(ag, ctx, x, v, m, eps, G, ag.AG_FP32_PAIRS)
    ar, jr, tr = orc.direct(x, v, m, eps, G)
    assert np.median(rel_err(a, ar)) <= 1e-5
    assert np.median(rel_err(j, jr)) <= 1e-5
    assert np.median(tensor_rel_err(t, tr)) <= 1e-5


@pytest.mark.parametrize("n,frac", [(1, 1.0), (2, 1.0), (257, 1.0), (1000, 0.3), (3001, 0.01)])
def test_direct_ragged_and_subsets(ag, ctx, orc, n, frac):
    """Ragged sizes (not multiples of the target tile or the staged source tile),
    small target sets split over workgroups, partial active sets
    in random order; rows not listed stay untouched."""
    x, v, m = workloads.plummer(n, seed=n)
    m = m * np.random.default_rng(n).uniform(0.5, 1.5, n)
    eps, G = 0.05, 0.7
    act = workloads.random_subset(n, frac, seed=n + 1)
    act = np.random.default_rng(n + 2).permutation(act)
    for prec, tol in ((ag.AG_FP64, 1e-12), (ag.AG_FP32_PAIRS, 1e-4)):
        a, j, t = _run_direct(ag, ctx, x, v, m, eps, G, prec, act)
        ar, jr, tr = orc.direct(x, v, m, eps, G, act)
        other = np.setdiff1d(np.arange(n), act)
        assert np.all(np.isnan(a[other])) and np.all(np.isnan(t[other]))
        if n == 1:
            assert np.all(a[act] == 0) and np.all(t[act] == 0)
            continue
        assert np.median(rel_err(a[act], ar)) <= tol
        assert np.median(rel_err(j[act], jr)) <= tol
        assert np.median(tensor_rel_err(t[act], tr)) <= tol


@pytest.mark.parametrize("n", [9000, 20000, 40000])
def test_direct_wide_target_sets(ag, ctx, orc, n):
    """Every row a target at sizes where each workgroup holds 16 to 64
    targets (4, 2 or 1 lane groups per wave; FP64 launches half as many
    workgroups as FP32 pairs, so the two take different shapes): sampled
    rows against the oracle, in both precisions, with a ragged last tile."""
    x, v, m = workloads.plummer(n, seed=n)
    eps, G = 0.01, 1.0
    rows = np.random.default_rng(n).choice(n, 64, replace=False)
    rows = np.concatenate([rows, [0, n - 1]])
    ar, jr, tr = orc.direct(x, v, m, eps, G, rows)
    for prec, tol in ((ag.AG_FP64, 1e-12), (ag.AG_FP32_PAIRS, 1e-5)):
        a, j, t = _run_direct(ag, ctx, x, v, m, eps, G, prec)
        assert np.all(np.isfinite(a)) and np.all(np.isfinite(t))
        assert np.median(rel_err(a[rows], ar)) <= tol
        assert np.median(rel_err(j[rows], jr)) <= tol
        assert np.median(tensor_rel_err(t[rows], tr)) <= tol


def test_direct_coincident_and_softened(ag, ctx, orc):
    """Coincident particles and pairs inside the softening length."""
    rng = np.random.default_rng(9)
    x = rng.uniform(-0.05, 0.05, (300, 3))
    x[10] = x[11]
    v = rng.normal(size=(300, 3))
    m = rng.uniform(0.5, 1.5, 300)
    eps = 0.1
    a, j, t = _run_direct(ag, ctx, x, v, m, eps, 1.0, ag.AG_FP64)
    ar, jr, tr = orc.direct(x, v, m, eps, 1.0)
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(t))
    np.testing.assert_allclose(a, ar, rtol=1e-11, atol=1e-11 * np.abs(ar).max())
    np.testing.assert_allclose(j, jr, rtol=1e-11, atol=1e-11 * np.abs(jr).max())
    np.testing.assert_allclose(t, tr, rtol=1e-11, atol=1e-11 * np.abs(tr).max())


def test_direct_deterministic(ag, ctx):
    x, v, m = workloads.plummer(2048, seed=3)
    r1 = _run_direct(ag, ctx, x, v, m, 0.01, 1.0, ag.AG_FP64)
    r2 = _run_direct(ag, ctx, x, v, m, 0.01, 1.0, ag.AG_FP64)
    for p, q in zip(r1, r2):
        assert np.array_equal(p, q)


def test_direct_bad_index_flag(ag, ctx):
    x, v, m = workloads.plummer(64, seed=3)
    with pytest.raises(ag.AgError) as e:
        _run_direct(ag, ctx, x, v, m, 0.01, 1.0, ag.AG_FP64, np.array([0, 5, 64]))
    assert e.value.code == ag.AG_EDEVICE
    # the context stays usable
    _run_direct(ag, ctx, x, v, m, 0.01, 1.0, ag.AG_FP64)


def test_direct_argument_errors(ag, ctx):
    x, v, m = workloads.plummer(16, seed=3)
    for eps in (0.0, -1.0, float("nan")):
        with pytest.raises(ag.AgError) as e:
            _run_direct(ag, ctx, x, v, m, eps, 1.0, ag.AG_FP64)
        assert e.value.code == ag.AG_EINVAL
    with pytest.raises(ag.AgError) as e:
        _run_direct(ag, ctx, x, v, m, 0.1, 1.0, 7)
    assert e.value.code == ag.AG_EINVAL
