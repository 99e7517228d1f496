"""GPU parity of the neighbour lengths (distance to the k-th nearest other
particle, the length adaptive softening follows) with the oracle's brute
force: both take d^2 = (dx^2 + dy^2) + dz^2 in FP64 with each operation
rounded once, so the lengths agree bit for bit.  Clumped and uniform
particles, a cubic lattice (many equal distances), coincident particles,
k = n - 1, the largest k, and sampled targets at 2^20 particles."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _t(a, dtype=None):
    return torch.tensor(a, device=DEV) if dtype is None else torch.tensor(a, dtype=dtype, device=DEV)


def _lengths(ag, x, k, n_leaf=16, box=0.0):
    n = x.shape[0]
    v = np.zeros((n, 3))
    m = np.full(n, 1.0 / n)
    with ag.Context(0) as c:
        if box:
            c.set_periodic(box)
        c.tree_build(_t(x), _t(v), _t(m), n_leaf)
        h = c.neighbour_lengths(k)
        hs = c.neighbour_lengths(k, scale=0.7)
        c.sync()
    h = h.cpu().numpy()
    # the scale multiplies each length once, in FP64
    np.testing.assert_array_equal(hs.cpu().numpy(), 0.7 * h)
    return h


@pytest.mark.parametrize("k", [1, 7, 32, 64])
def test_clumps_exact(ag, orc, k):
    x, _, _, _ = workloads.clumps(6001, seed=11)
    h = _lengths(ag, x, k)
    hr = orc.neighbour_length(x, k)
    print(f"clumps n=6001 k={k}: mismatches {int(np.sum(h != hr))}", flush=True)
    np.testing.assert_array_equal(h, hr)


@pytest.mark.parametrize("n_leaf", [1, 16, 64])
def test_uniform_leaf_sizes(ag, orc, n_leaf):
    rng = np.random.default_rng(12)
    x = rng.uniform(-1.0, 1.0, (4099, 3))
    np.testing.assert_array_equal(_lengths(ag, x, 16, n_leaf), orc.neighbour_length(x, 16))


def test_lattice_ties(ag, orc):
    # spacing 1/8: the 6 face neighbours tie, then the 12 edge neighbours
    g = np.arange(10) / 8.0
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    for k in (1, 6, 7, 18, 19):
        h = _lengths(ag, x, k)
        np.testing.assert_array_equal(h, orc.neighbour_length(x, k))
    interior = np.all((x > 0) & (x < 9 / 8.0), axis=1)
    h6 = _lengths(ag, x, 6)
    assert np.all(h6[interior] == 0.125)


def test_coincident_and_small(ag, orc):
    rng = np.random.default_rng(13)
    base = rng.normal(size=(300, 3))
    x = np.concatenate([base, base[:100], base[:50]])   # up to triples
    for k in (1, 2, 3, 40):
        for n_leaf in (1, 16):   # one per leaf: the copies share the deepest cells
            np.testing.assert_array_equal(_lengths(ag, x, k, n_leaf), orc.neighbour_length(x, k))
    assert np.all(_lengths(ag, x, 2)[:50] == 0.0)
    y = rng.normal(size=(65, 3))                         # k = n - 1: the farthest
    np.testing.assert_array_equal(_lengths(ag, y, 64), orc.neighbour_length(y, 64))
    z = rng.normal(size=(2, 3))
    h = _lengths(ag, z, 1)
    assert h[0] == h[1] == orc.neighbour_length(z, 1)[0]
    w = np.tile(rng.normal(size=(1, 3)), (100, 1))        # all coincident
    assert np.all(_lengths(ag, w, 40) == 0.0)


@pytest.fixture(scope="module")
def sphere_2p20():
    return workloads.turbulent_sphere(1 << 20, seed=2)[0]


@pytest.mark.parametrize("k", [16, 32, 64])
def test_full_size_sampled(ag, orc, sphere_2p20, k):
    x = sphere_2p20
    n = len(x)
    h = _lengths(ag, x, k)
    rows = np.random.default_rng(14 + k).choice(n, 256, replace=False)
    np.testing.assert_array_equal(h[rows], orc.neighbour_length(x, k, targets=rows, chunk=32))
    assert np.all(np.isfinite(h)) and np.all(h > 0)


def test_independent_of_grouping(ag):
    """The lengths do not depend on how the targets are grouped (one target
    per wave up to 64, ragged group sizes in between)."""
    x, _, _, _ = workloads.clumps(6001, seed=23)
    n = len(x)
    out = []
    for gt in (64, 17, 5, 1):
        with ag.Context(0) as c:
            c.set_option(ag.AG_OPT_GROUP_TARGETS, gt)
            c.tree_build(_t(x), _t(np.zeros((n, 3))), _t(np.full(n, 1.0 / n)), 16)
            h = c.neighbour_lengths(20)
            c.sync()
        out.append(h.cpu().numpy())
    for h in out[1:]:
        np.testing.assert_array_equal(h, out[0])


# ---- periodic trees: nearest images ------------------------------------------
@pytest.mark.parametrize("k", [1, 16, 32, 64])
def test_periodic_clumps_exact(ag, orc, k):
    x, _, _, _ = workloads.clumps(6001, seed=21)
    x = np.mod(x, 1.0)            # clumps cut by the faces
    h = _lengths(ag, x, k, box=1.0)
    np.testing.assert_array_equal(h, orc.neighbour_length(x, k, box=1.0))


def test_periodic_uniform_and_box_size(ag, orc):
    rng = np.random.default_rng(22)
    for L in (1.0, 2.5):
        x = rng.uniform(0.0, L, (5003, 3))
        for n_leaf in (1, 16):
            np.testing.assert_array_equal(_lengths(ag, x, 24, n_leaf, box=L), orc.neighbour_length(x, 24, box=L))


def test_periodic_lattice(ag, orc):
    a = 1.0 / 8                    # exact, so every difference is
    g = np.arange(8) * a
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    for k in (6, 18, 26):
        h = _lengths(ag, x, k, box=1.0)
        np.testing.assert_array_equal(h, orc.neighbour_length(x, k, box=1.0))
    assert np.all(_lengths(ag, x, 6, box=1.0) == a)   # the corners too


def test_arguments(ag):
    x, v, m, _ = workloads.clumps(2048, seed=4)
    with ag.Context(0) as c:
        with pytest.raises(ag.AgError) as e:
            c.neighbour_lengths(8, out=torch.empty(2048, dtype=torch.float64, device=DEV))
        assert e.value.code == ag.AG_ESTATE                # no tree yet
        c.tree_build(_t(x), _t(v), _t(m), 16)
        for bad in (0, 65, -3):
            with pytest.raises(ag.AgError) as e:
                c.neighbour_lengths(bad)
            assert e.value.code == ag.AG_EINVAL
        for bad in (0.0, -1.0, float("inf"), float("nan")):
            with pytest.raises(ag.AgError) as e:
                c.neighbour_lengths(8, scale=bad)
            assert e.value.code == ag.AG_EINVAL
        c.set_periodic(0.0)
        off = _t([0, 1000, 2048], torch.int64)
        c.tree_build_batched(_t(x), _t(v), _t(m), off, 16)
        with pytest.raises(ag.AgError) as e:
            c.neighbour_lengths(8)
        assert e.value.code == ag.AG_ESTATE
        y = np.random.default_rng(1).normal(size=(10, 3))
        c.tree_build(_t(y), _t(np.zeros((10, 3))), _t(np.ones(10)), 16)
        with pytest.raises(ag.AgError) as e:
            c.neighbour_lengths(10)
        assert e.value.code == ag.AG_EINVAL
        c.sync()
