"""Pins of the oracle's replica exchange (paper Sec. 2.2, case study REMC).

Replica k targets p(x)^beta_k, i.e. beta_k times the log-probability (the
paper's replica target function multiplies the log-probability by the
inverse temperature).  Pins:
  * the tempered leapfrog on a Gaussian is the per-eigenmode closed form with
    precision beta * a;
  * a tempered N(0, 1) chain samples N(0, 1/beta);
  * with equal temperatures every proposed exchange is accepted, so the step
    is the exact pair permutation of its parity class;
  * the exchange acceptance of fixed states equals min(1, exp((beta_a - beta_b)
    (l(x_b) - l(x_a)))) in frequency, and is 1 in the favourable direction;
  * a full run keeps every replica at its own tempered distribution
    (variance 1/beta_k on N(0, 1)) -- an exchange rule with the wrong sign moves
    wide states to the cold replica and fails this.
"""
import numpy as np
import pytest

import oracle
from oracle import Target

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _mode_map(a, eps, L):
    M = np.array([[1 - eps ** 2 * a / 2, eps], [-eps * a * (1 - eps ** 2 * a / 4), 1 - eps ** 2 * a / 2]])
    c = 1 - eps ** 2 * a / 2
    th = np.arccos(c)
    return np.cos(L * th) * np.eye(2) + np.sin(L * th) / np.sin(th) * (M - c * np.eye(2))


def test_tempered_leapfrog_is_closed_form_with_scaled_precision():
    D, eps, L, beta = 5, 0.4, 9, 0.3
    a = np.linspace(0.5, 6.0, D)
    tg = Target(oracle.GAUSS_DIAG, D, prec=a).tempered(beta)
    rng = np.random.default_rng(7)
    x0, p0 = rng.normal(size=D), rng.normal(size=D)
    xL, pL, lpL, gL = oracle.leapfrog(tg, eps, L, x0, p0)
    for i in range(D):
        yL, qL = _mode_map(beta * a[i], eps, L) @ np.array([x0[i], p0[i]])
        assert xL[i] == pytest.approx(yL, rel=1e-12, abs=1e-14)
        assert pL[i] == pytest.approx(qL, rel=1e-12, abs=1e-14)
    assert lpL == pytest.approx(-0.5 * beta * np.sum(a * xL ** 2), rel=1e-12)
    assert np.allclose(gL, -beta * a * xL, rtol=1e-13, atol=0)


def test_tempered_standard_normal_has_variance_one_over_beta():
    beta = 0.25
    tg = Target(oracle.STD_NORMAL, 1).tempered(beta)
    r = oracle.sample_chain(tg, 3, 11, np.zeros((200, 1)), 1.5, 100, 400)
    v = r["samples"].var()
    # 80000 draws, integrated autocorrelation of x^2 a few transitions: SE of var ~ 1.5%
    assert v == pytest.approx(1.0 / beta, rel=0.08)


def test_equal_temperatures_swap_every_proposed_pair():
    K, M, D = 5, 3, 2
    tg = Target(oracle.STD_NORMAL, D)
    x = np.random.default_rng(1).normal(size=(K * M, D))
    for t in (0, 1):
        r = oracle.remc_swap(tg, [0.7] * K, 3, t, x)
        expect = x.copy()
        for k in range(t % 2, K - 1, 2):
            expect[k * M:(k + 1) * M], expect[(k + 1) * M:(k + 2) * M] = \
                x[(k + 1) * M:(k + 2) * M].copy(), x[k * M:(k + 1) * M].copy()
        assert np.array_equal(r["x"], expect)
        paired = np.zeros(K * M, bool)
        for k in range(t % 2, K - 1, 2):
            paired[k * M:(k + 2) * M] = True
        assert np.array_equal(r["swapped"], paired)
        # the cached values belong to each chain's own replica after the exchange
        lp, g = oracle.logp_grad(tg.tempered(0.7), r["x"])
        assert np.allclose(r["logp"], lp, rtol=0, atol=0) and np.allclose(r["g"], g, rtol=0, atol=0)


def test_exchange_acceptance_frequency_matches_ratio():
    M = 40000
    betas = [1.0, 0.5]
    tg = Target(oracle.STD_NORMAL, 1)
    xa, xb = 0.0, 1.5                                  # l(xa) = 0, l(xb) = -1.125
    x = np.concatenate([np.full((M, 1), xa), np.full((M, 1), xb)])
    r = oracle.remc_swap(tg, betas, 5, 0, x)
    p = np.exp((betas[0] - betas[1]) * (-0.5 * xb ** 2 + 0.5 * xa ** 2))   # 0.5698
    frac = r["swapped"][:M].mean()
    assert abs(frac - p) < 4 * np.sqrt(p * (1 - p) / M)
    assert np.array_equal(r["swapped"][:M], r["swapped"][M:])
    moved = r["swapped"][:M]
    assert np.all(r["x"][:M][moved] == xb) and np.all(r["x"][M:][moved] == xa)
    assert np.all(r["x"][:M][~moved] == xa)
    # favourable direction (the wide state at the hot replica already): always accepted
    r2 = oracle.remc_swap(tg, betas, 5, 0, np.concatenate([np.full((M, 1), xb), np.full((M, 1), xa)]))
    assert r2["swapped"].all()
    # odd swap index with two replicas: no pair
    r3 = oracle.remc_swap(tg, betas, 5, 1, x)
    assert not r3["swapped"].any() and np.array_equal(r3["x"], x)


def test_replicas_keep_their_tempered_distributions():
    betas = [1.0, 0.5, 0.25, 0.125]
    M = 100
    tg = Target(oracle.STD_NORMAL, 1)
    r = oracle.remc_sample_chain(tg, betas, 3, 0, np.zeros((4 * M, 1)), 1.5, 100, 600)
    s = r["samples"]
    for k, b in enumerate(betas):
        v = s[:, k * M:(k + 1) * M].var()
        assert v == pytest.approx(1.0 / b, rel=0.06), (k, v)
        assert abs(s[:, k * M:(k + 1) * M].mean()) < 0.1 / np.sqrt(b)
    assert 0.3 < r["swapped"].mean() < 0.9


def test_remc_with_one_replica_is_plain_sample_chain():
    tg = Target(oracle.GAUSS_DIAG, 3, prec=np.array([0.5, 1.0, 2.0]))
    x0 = np.random.default_rng(3).uniform(-2, 2, size=(20, 3))
    a = oracle.remc_sample_chain(tg, [1.0], 4, 9, x0, 0.3, 30, 40, adapt=True)
    b = oracle.sample_chain(tg, 4, 9, x0, 0.3, 30, 40, adapt=True)
    assert np.array_equal(a["samples"], b["samples"])
    assert np.array_equal(a["is_accepted"], b["is_accepted"])
    assert not a["swapped"].any()
    assert np.array_equal(a["final_eps"], b["final_eps"])
