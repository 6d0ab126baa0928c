"""Pins of the host-side R-hat / ESS estimators against closed forms.

AR(1) chains x_t = rho x_{t-1} + sqrt(1 - rho^2) e_t (stationary start) have
integrated autocorrelation time (1 + rho)/(1 - rho), so ESS -> n M (1 - rho)/(1 + rho).
iid chains give R-hat -> 1; chains with shifted means give R-hat > 1.
"""
import numpy as np
import pytest

from paper_2002_01184_amd import diagnostics as dg


def _ar1(n, M, rho, seed):
    rng = np.random.default_rng(seed)
    e = rng.normal(size=(n, M))
    x = np.empty((n, M))
    x[0] = e[0]
    s = np.sqrt(1 - rho * rho)
    for t in range(1, n):
        x[t] = rho * x[t - 1] + s * e[t]
    return x


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9, -0.3])
def test_ess_ar1_closed_form(rho):
    n, M = 4000, 40
    x = _ar1(n, M, rho, seed=int(100 * (rho + 1)))
    expected = n * M * (1 - rho) / (1 + rho)
    got = dg.ess(x)
    assert abs(got / expected - 1) < 0.1, (got, expected)
    assert abs(dg.ess_bulk(x) / expected - 1) < 0.12


def test_rhat_iid_is_one_and_shift_detected():
    x = _ar1(2000, 32, 0.3, seed=1)
    assert dg.rhat(x) < 1.01
    y = x.copy()
    y[:, :16] += 0.5
    # classic between/within formula on the unsplit chains
    n = y.shape[0]
    B = n * y.mean(0).var(ddof=1)
    W = y.var(0, ddof=1).mean()
    expected = np.sqrt(((n - 1) / n * W + B / n) / W)
    assert dg._rhat_basic(y) == pytest.approx(expected, rel=1e-12)
    # population value for half the chains shifted by 0.5 sd: sqrt(1 + 0.5^2 / 4)
    assert dg.rhat(y) == pytest.approx(np.sqrt(1 + 0.25 / 4), abs=0.01)
    # a trend within chains is caught by splitting
    z = x + np.linspace(0, 2, x.shape[0])[:, None]
    assert dg.rhat(z) > 1.05


def test_summarize_shapes():
    x = _ar1(200, 8, 0.2, seed=3)
    s = np.stack([x, 2 * x], axis=-1)
    out = dg.summarize(s)
    assert out["ess_bulk"].shape == (2,) and out["max_rhat"] < 1.05
    assert out["ess_bulk"][0] == pytest.approx(out["ess_bulk"][1])   # rank-based: scale-free


def test_torch_estimators_equal_numpy():
    import torch
    x = _ar1(600, 12, 0.6, seed=9)
    x[:, :3] += 0.2
    s = np.stack([x, x ** 2, np.round(x, 1)], axis=-1)          # includes ties
    a = dg.summarize(s)
    b = dg.t_summarize(torch.from_numpy(s))
    assert np.allclose(a["ess_bulk"], b["ess_bulk"], rtol=1e-9)
    assert np.allclose(a["rhat"], b["rhat"], rtol=1e-12)


def _half_moments(x):
    """x [R, C, D] -> two-pass mean / m2 [2, C, D] of the halves r < R//2 and r >= R//2."""
    h = x.shape[0] // 2
    parts = [x[:h], x[h:]]
    mean = np.stack([p.mean(0) for p in parts])
    m2 = np.stack([((p - p.mean(0)) ** 2).sum(0) for p in parts])
    return mean, m2


def test_split_rhat_from_moments_equals_split_rhat_of_samples():
    rng = np.random.default_rng(5)
    x = _ar1(600, 12, 0.6, seed=3)[:, :, None] + rng.normal(0, 0.05, size=(1, 12, 1))
    x = np.concatenate([x, 2 * x + 1], axis=2)                     # two coordinates
    mean, m2 = _half_moments(x)
    got = dg.moments_rhat(mean, m2, x.shape[0])
    for d in range(2):
        assert got[d] == pytest.approx(dg._rhat_basic(dg._split(x[:, :, d])), rel=1e-12)
    # a shifted chain raises it
    y = x.copy()
    y[:, 0] += 3.0
    assert np.all(dg.moments_rhat(*_half_moments(y), x.shape[0]) > 1.05)


@pytest.mark.parametrize("rho", [0.0, 0.7])
def test_batch_means_ess_ar1(rho):
    n, M, blen = 20000, 16, 400
    x = _ar1(n, M, rho, seed=11)[:, :, None]
    mean, m2 = _half_moments(x)
    bsum = x.reshape(n // blen, blen, M, 1).sum(1)
    got = dg.moments_ess_batch(mean, m2, bsum, n, blen)[0]
    expected = n * M * (1 - rho) / (1 + rho)
    assert abs(got / expected - 1) < 0.15, (got, expected)
    # the pooled within-chain variance recombined from the halves is the sample variance
    h = n // 2
    d = mean[1] - mean[0]
    m2c = m2[0] + m2[1] + d * d * h * (n - h) / n
    assert np.allclose(m2c / (n - 1), x.var(0, ddof=1), rtol=1e-10)
