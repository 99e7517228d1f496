"""GPU edge cases of the tree path: positions far from the origin (the walk's
FP32 coordinates are taken relative to each group, so a large common offset
must cost no accuracy), a single particle, and a two-body system whose
field has a closed form; the memory limit's AG_ENOMEM path."""
import numpy as np
import pytest
import torch

import workloads
from conftest import rel_err

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _t(a, dtype=None):
    return torch.tensor(a, device=DEV) if dtype is None else torch.tensor(a, dtype=dtype, device=DEV)


def _eval(ag, x, v, m, theta, eps, G=1.0):
    n = len(m)
    out = [torch.full((n, k), float("nan"), dtype=torch.float64, device=DEV) for k in (3, 3, 6)]
    with ag.Context(0) as c:
        c.tree_build(_t(x), _t(v), _t(m), 16)
        c.grav_eval(None, theta, eps, G, *out)
        c.sync()
    return [o.cpu().numpy() for o in out]


def test_far_offset(ag, orc):
    x, v, m, _ = workloads.clumps(1 << 14, seed=51)
    shift = np.array([1.0e4, -2.5e4, 3.0e4])
    rows = np.random.default_rng(52).choice(len(m), 1024, replace=False)
    for xs in (x, x + shift):
        a, j, T = _eval(ag, xs, v, m, 0.7, 1e-3)
        ar, _, _ = orc.direct(xs, v, m, 1e-3, 1.0, rows)
        e = rel_err(a[rows], ar)
        print(f"offset {xs[0] - x[0]}: median {np.median(e):.2e} p99 {np.percentile(e, 99):.2e}", flush=True)
        assert np.median(e) <= 1e-3 and np.percentile(e, 99) <= 1e-2


def test_single_particle(ag):
    a, j, T = _eval(ag, np.array([[0.3, -0.2, 5.0]]), np.array([[1.0, 0.0, 0.0]]), np.array([2.0]), 0.7, 1e-3)
    assert np.all(a == 0.0) and np.all(j == 0.0) and np.all(T == 0.0)


def test_two_bodies_closed_form(ag):
    x = np.array([[0.1, 0.2, 0.3], [0.4, -0.2, 0.7]])
    v = np.array([[0.0, 1.0, 0.0], [0.5, 0.0, -0.25]])
    m = np.array([1.0, 2.0])
    G = 1.7
    a, j, T = _eval(ag, x, v, m, 0.7, 1e-3, G)
    for i, k in ((0, 1), (1, 0)):
        d = x[k] - x[i]
        nu = v[k] - v[i]
        r = np.linalg.norm(d)
        ga = G * m[k] * d / r**3
        gj = G * m[k] * (nu / r**3 - 3.0 * np.dot(d, nu) * d / r**5)
        Tf = -G * m[k] * (np.eye(3) / r**3 - 3.0 * np.outer(d, d) / r**5)
        gT = np.array([Tf[0, 0], Tf[1, 1], Tf[2, 2], Tf[0, 1], Tf[0, 2], Tf[1, 2]])
        assert np.allclose(a[i], ga, rtol=1e-6, atol=0)
        assert np.allclose(j[i], gj, rtol=1e-5, atol=1e-6 * np.abs(gj).max())
        assert np.allclose(T[i], gT, rtol=1e-5, atol=1e-6 * np.abs(gT).max())


def test_memory_limit_gives_enomem_and_recovers(ag):
    """AG_ENOMEM forced by the context's memory limit: a build that would
    grow the buffers past it fails before freeing or launching anything and
    leaves no tree (an evaluation then gives AG_ESTATE); with the limit
    lifted the same context builds and evaluates bit for bit as a fresh
    one."""
    n = 20000
    x, v, m = workloads.plummer(n, seed=12)
    tx, tv, tm = _t(x), _t(v), _t(m)
    with pytest.raises(ag.AgError) as bad:
        with ag.Context(0) as c:
            c.set_option(ag.AG_OPT_MEM_LIMIT, -1)
    assert bad.value.code == ag.AG_EINVAL
    with ag.Context(0) as c:
        c.set_option(ag.AG_OPT_MEM_LIMIT, 1 << 20)   # far below what 20000 particles need
        with pytest.raises(ag.AgError) as e:
            c.tree_build(tx, tv, tm, 16)
        assert e.value.code == ag.AG_ENOMEM
        acc = torch.zeros((n, 3), dtype=torch.float64, device=DEV)
        rows = torch.arange(n, dtype=torch.int32, device=DEV)
        with pytest.raises(ag.AgError) as e2:
            c.grav_eval(rows, 0.7, 1e-3, 1.0, acc, None, None)
        assert e2.value.code == ag.AG_ESTATE
        c.set_option(ag.AG_OPT_MEM_LIMIT, 0)
        c.tree_build(tx, tv, tm, 16)
        c.grav_eval(None, 0.7, 1e-3, 1.0, acc, None, None)
        c.sync()
    ref = torch.zeros_like(acc)
    with ag.Context(0) as c:
        c.tree_build(tx, tv, tm, 16)
        c.grav_eval(None, 0.7, 1e-3, 1.0, ref, None, None)
        c.sync()
    assert torch.equal(acc, ref)
