"""Host-side argument checks of the adaptive integrator (no GPU: they run
before the integrator touches its context)."""
import pytest
import torch

from paper_2010_13792_amd.driver import AdaptiveIntegrator, PREDICTORS


def _x():
    return torch.zeros((4, 3), dtype=torch.float64)


@pytest.mark.parametrize("kw", [dict(predictor="cubic-spline"), dict(opening_alpha=-0.1),
                                dict(opening_alpha=float("nan")), dict(soft_k=-1), dict(soft_k=8, soft_scale=0.0),
                                dict(soft_pm=8.0), dict(soft_pm=-1.0), dict(soft_pm=32.0, soft_k=16)])
def test_rejects_bad_arguments(kw):
    with pytest.raises(ValueError):
        AdaptiveIntegrator(None, _x(), _x(), torch.ones(4, dtype=torch.float64), q_f=0.5, theta=0.7, eps=1e-3, **kw)


def test_predictor_names():
    assert set(PREDICTORS) == {"jerk", "none", "linear", "quadratic"}
