"""The allocation-free direct sum (ag_grav_direct_noalloc) against
ag_grav_direct: the same kernels on library-held scratch, so the results are
bit-identical; two calls in a row that both split their sources over
workgroups (small listed target sets), the second with a smaller input (the
shared scratch is reused), then every row of a set that fills the device
without a split; in both precisions; and its argument checks."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _t(a, dtype=None):
    return torch.tensor(a, device=DEV) if dtype is None else torch.tensor(a, dtype=dtype, device=DEV)


def _outputs(n):
    return [torch.full((n, k), float("nan"), dtype=torch.float64, device=DEV) for k in (3, 3, 6)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_direct(ag, prec):
    p = ag.AG_FP64 if prec == "fp64" else ag.AG_FP32_PAIRS
    # both of the first two split their sources in either precision (250 and
    # 84 tiles of 4 targets), the second is smaller; the third splits nothing
    cases = [(20000, np.random.default_rng(1).permutation(20000)[:1000]),
             (1500, np.random.default_rng(2).permutation(1500)[:333]), (4096, None)]
    with ag.Context(0) as c:
        for n, act in cases:
            x, v, m = workloads.plummer(n, seed=n)
            tx, tv, tm = _t(x), _t(v), _t(m)
            ia = None if act is None else _t(act.astype(np.int32), torch.int32)
            ref, got = _outputs(n), _outputs(n)
            c.grav_direct(tx, tv, tm, ia, 0.01, 1.3, *ref, precision=p)
            c.grav_direct(tx, tv, tm, ia, 0.01, 1.3, *got, precision=p, noalloc=True)
            c.sync()
            for r, g in zip(ref, got):
                assert torch.equal(torch.isnan(r), torch.isnan(g))
                assert torch.equal(torch.nan_to_num(r), torch.nan_to_num(g)), (n, prec)
            if act is not None:   # rows not listed stay untouched
                other = np.setdiff1d(np.arange(n), act)
                assert torch.all(torch.isnan(got[0][_t(other)]))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,k", [(2048, 1), (2048, 1023), (2048, 2047), (65536, 3), (65536, 1024), (65536, 2047),
                                 (1 << 20, 511), (1 << 20, 2047), (1 << 20, 2048)])
def test_noalloc_refuses_no_size(ag, n, k, prec):
    """Target sets on both sides of the split thresholds (the sources are
    split over workgroups below 1024 targets in FP64 and below 2048 with FP32
    pairs, and the scratch holds the split sums), up to 2^20 sources: the
    fixed scratch always suffices, and the results equal the allocating entry
    point's bit for bit."""
    p = ag.AG_FP64 if prec == "fp64" else ag.AG_FP32_PAIRS
    x, v, m = workloads.plummer(n, seed=k)
    act = np.random.default_rng(k).choice(n, k, replace=False).astype(np.int32)
    tx, tv, tm, ia = _t(x), _t(v), _t(m), _t(act, torch.int32)
    with ag.Context(0) as c:
        ref, got = _outputs(n), _outputs(n)
        c.grav_direct(tx, tv, tm, ia, 0.01, 1.0, *ref, precision=p)
        c.grav_direct(tx, tv, tm, ia, 0.01, 1.0, *got, precision=p, noalloc=True)
        c.sync()
    for r, g in zip(ref, got):
        assert torch.equal(torch.nan_to_num(r), torch.nan_to_num(g)), (n, k)
    assert torch.all(torch.isfinite(got[0][ia.long()]))


def test_noalloc_arguments(ag):
    x, v, m = workloads.plummer(64, seed=3)
    with ag.Context(0) as c:
        out = _outputs(64)
        for eps in (0.0, float("nan")):
            with pytest.raises(ag.AgError) as e:
                c.grav_direct(_t(x), _t(v), _t(m), None, eps, 1.0, *out, noalloc=True)
            assert e.value.code == ag.AG_EINVAL
        with pytest.raises(ag.AgError) as e:
            c.grav_direct(_t(x), _t(v), _t(m), _t(np.array([0, 5, 64]), torch.int32), 0.01, 1.0, *out, noalloc=True)
            c.sync()
        assert e.value.code == ag.AG_EDEVICE
        c.grav_direct(_t(x), _t(v), _t(m), None, 0.01, 1.0, *out, noalloc=True)   # still usable
        c.sync()
        assert torch.all(torch.isfinite(out[0]))
