"""Pins of the oracle's multiplicative step-size adaptation (the paper's
SimpleStepSizeAdaptation example of the wrapper pattern, Sec. 4.1): after each
burn-in transition the step size is multiplied by (1 + rate) when the accept
statistic min(1, exp(-dH)) exceeds the target and divided by (1 + rate)
otherwise; it keeps its last value after the burn-in.

  * a chain whose accept statistic is always 0 (NaN state) ends the burn-in at
    eps0 / (1 + rate)^B, one with statistic always 1 (flat target: dH = 0
    exactly) at eps0 (1 + rate)^B;
  * the rule is a stochastic approximation of the step size at which half of
    the accept statistics exceed the target, so after a long burn-in the kept
    transitions have about half of their statistics above the target;
  * dual averaging is unchanged by the new argument.
"""
import numpy as np
import pytest

import oracle
from oracle import Target

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def test_rule_single_steps():
    assert oracle.simple_adapt(0.5, 0.9, 0.8, 0.02) == 0.5 * 1.02
    assert oracle.simple_adapt(0.5, 0.8, 0.8, 0.02) == 0.5 / 1.02     # equality shrinks
    assert oracle.simple_adapt(0.5, 0.0, 0.8, 0.02) == 0.5 / 1.02


def test_always_reject_and_always_accept_closed_forms():
    B, r, e0 = 60, 0.03, 0.4
    tg = Target(oracle.STD_NORMAL, 2)
    x0 = np.array([[np.nan, 0.0], [np.nan, 1.0]])
    o = oracle.sample_chain(tg, 3, 1, x0, e0, B, 2, adapt="simple", rate=r)
    assert np.allclose(o["final_eps"], e0 / (1 + r) ** B, rtol=1e-13, atol=0)
    assert not o["is_accepted"].any()
    flat = Target(oracle.GAUSS_DIAG, 3, prec=np.zeros(3))
    o = oracle.sample_chain(flat, 3, 1, np.ones((4, 3)), e0, B, 2, adapt="simple", rate=r)
    assert np.allclose(o["final_eps"], e0 * (1 + r) ** B, rtol=1e-13, atol=0)
    assert np.all(o["log_accept_ratio"] == 0.0)
    # kept transitions use the last adapted value, unchanged
    assert np.all(o["step_size"] == o["final_eps"][None, :])


def test_balances_at_the_median_accept_statistic():
    D, C, delta = 10, 200, 0.8
    tg = Target(oracle.STD_NORMAL, D)
    x0 = np.random.default_rng(0).normal(size=(C, D))
    o = oracle.sample_chain(tg, 5, 3, x0, 1.0, 1500, 400, adapt="simple", target_accept=delta, rate=0.01)
    alpha = np.exp(np.minimum(0.0, o["log_accept_ratio"]))
    frac = np.mean(alpha > delta)
    assert 0.4 < frac < 0.6, frac
    # the same chains under dual averaging reach a mean statistic near the target instead
    d = oracle.sample_chain(tg, 5, 3, x0, 1.0, 1500, 400, adapt=True, target_accept=delta)
    assert abs(np.exp(np.minimum(0.0, d["log_accept_ratio"])).mean() - delta) < 0.05


def test_dual_averaging_path_is_unchanged_by_the_rate_argument():
    tg = Target(oracle.STD_NORMAL, 3)
    x0 = np.random.default_rng(1).normal(size=(8, 3))
    a = oracle.sample_chain(tg, 4, 2, x0, 0.5, 50, 20, adapt=True, rate=0.01)
    b = oracle.sample_chain(tg, 4, 2, x0, 0.5, 50, 20, adapt="dual_averaging", rate=0.5)
    assert np.array_equal(a["samples"], b["samples"]) and np.array_equal(a["final_eps"], b["final_eps"])
