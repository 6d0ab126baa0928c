"""Pins of the oracle's No-U-Turn sampler (paper Sec. 2.3; Hoffman & Gelman
2014, Algorithm 3).

  * max_depth 0 never moves; max_depth 1 is one leapfrog step of size v eps
    (v from the direction uniform) accepted exactly when the slice variable
    admits the new point -- recomputed here from the leapfrog, the momentum and
    the Philox blocks, independently of the tree code;
  * the trajectory never exceeds 2^depth - 1 leapfrog steps and, on a 1-D
    Gaussian with a small step, stops near half an orbit (U-turn);
  * stationary moments: N(0, 1), a correlated 2-D Gaussian (rho 0.9) and an
    ill-conditioned diagonal Gaussian, within Monte Carlo error.
"""
import numpy as np
import pytest

import oracle
from oracle import Target

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _u52(seed, chain, t, block, tag):
    w = oracle.philox(np.array([[chain, t, block, tag]], dtype=np.uint32),
                      (seed & 0xFFFFFFFF, seed >> 32))[0].astype(np.uint64)
    k = float(w[0] >> np.uint64(6)) * 67108864.0 + float(w[1] >> np.uint64(6))
    return (k + 0.5) * 2.0 ** -52


def test_depth_zero_never_moves():
    tg = Target(oracle.STD_NORMAL, 3)
    x = np.array([0.3, -1.0, 2.0])
    r = oracle.nuts_transition(tg, 5, 2, 7, 0.4, 0, x)
    assert np.array_equal(r["x"], x) and r["depth"] == 0 and r["n_leapfrog"] == 0 and not r["moved"]


@pytest.mark.parametrize("kind", ["dense", "logreg"])
def test_depth_one_is_a_sliced_single_leapfrog_step(kind):
    rng = np.random.default_rng(0)
    if kind == "dense":
        A = rng.normal(size=(4, 4))
        tg = Target(oracle.GAUSS_DENSE, 4, prec=A @ A.T + np.eye(4))
    else:
        tg = Target(oracle.LOGREG, 4, X=rng.normal(size=(40, 4)), y=(rng.uniform(size=40) < 0.5).astype(float))
    seed, eps = 9, 0.45
    moved = 0
    for chain in range(40):
        for t in range(3):
            x = rng.normal(size=4)
            lp0, g0 = oracle.logp_grad(tg, x)
            p0 = oracle.momentum(seed, chain + 1, t, 4)[chain]
            v = -1.0 if _u52(seed, chain, t, 0, oracle.TAG_NUTS_DIR) < 0.5 else 1.0
            x1, p1, lp1, _ = oracle.leapfrog(tg, v * eps, 1, x, p0)
            H0 = -lp0 + 0.5 * p0 @ p0
            H1 = -lp1 + 0.5 * p1 @ p1
            log_u = np.log(_u52(seed, chain, t, 0, oracle.TAG_NUTS_SLICE)) - H0
            take = (log_u <= -H1) and (log_u < 1000 - H1)
            r = oracle.nuts_transition(tg, seed, chain, t, eps, 1, x)
            assert r["depth"] == 1 and r["n_leapfrog"] == 1
            assert r["moved"] == take
            assert np.allclose(r["x"], x1 if take else x, rtol=0, atol=1e-15)
            moved += take
    assert 0 < moved < 120


def test_trajectory_length_and_u_turn():
    tg = Target(oracle.STD_NORMAL, 1)
    r = oracle.nuts_sample_chain(tg, 3, np.ones((64, 1)), 0.02, 5, 20, max_depth=12)
    d, nl = r["depth"], r["n_leapfrog"]
    assert np.all(nl <= 2 ** d - 1)
    # the orbit of N(0, 1) has period 2 pi: a trajectory stops by the U-turn
    # criterion within half an orbit of its span (pi / 0.02 ~ 157 steps), so none
    # reaches a full orbit and the longest are about half of one
    assert nl.max() <= 2 * np.pi / 0.02 and d.max() <= 9
    assert 0.8 * np.pi / 0.02 < np.percentile(nl, 95) < 1.2 * np.pi / 0.02


@pytest.mark.parametrize("case", ["std1", "corr2", "diag6"])
def test_stationary_moments(case):
    if case == "std1":
        tg, cov, eps = Target(oracle.STD_NORMAL, 1), np.eye(1), 0.5
    elif case == "corr2":
        cov = np.array([[1.0, 0.9], [0.9, 1.0]])
        tg, eps = Target(oracle.GAUSS_DENSE, 2, prec=np.linalg.inv(cov)), 0.2
    else:
        lam = np.logspace(-1, 1, 6)
        tg, cov, eps = Target(oracle.GAUSS_DIAG, 6, prec=1 / lam), np.diag(lam), 0.2
    D = cov.shape[0]
    x0 = np.random.default_rng(1).normal(size=(200, D)) @ np.linalg.cholesky(cov).T
    r = oracle.nuts_sample_chain(tg, 11, x0, eps, 50, 500, max_depth=8)
    s = r["samples"].reshape(-1, D)
    # 100000 draws, NUTS draws nearly independent: 4-sigma bounds
    assert np.all(np.abs(s.mean(0)) < 4 * np.sqrt(np.diag(cov) / 1e4))
    assert np.allclose(np.cov(s.T).reshape(D, D), cov, atol=0.04 * np.max(np.diag(cov)))


# ------------------------------------------------- step-size adaptation --
# Hoffman & Gelman (2014) Algorithm 6: the statistic that drives the step size
# is the mean of min(1, exp(H0 - H)) over the leaves of the last doubling.
# On N(0, I) leapfrog conserves r.r/2 + (1 - eps^2/4) x.x/2 exactly, so a
# leaf's energy error is (eps^2 / 8)(|x|^2 - |x0|^2): the statistic follows
# from the leaves' positions alone, without the oracle's energy code.

@pytest.mark.parametrize("eps", [0.3, 0.9, 1.6])
def test_accept_stat_is_the_last_doublings_mean_in_closed_form(eps):
    D = 3
    tg = Target(oracle.STD_NORMAL, D)
    rng = np.random.default_rng(11)
    checked = 0
    for t in range(40):
        x0 = rng.normal(size=D) * 1.5
        r = oracle.nuts_transition(tg, 9, t % 5, t, eps, 6, x0, record_leaves=True)
        assert r["leaf_x"].shape == (r["n_leapfrog"], D)
        if r["n_leapfrog"] == 0:
            continue
        last = r["leaf_j"] == r["depth"] - 1
        assert last.any() and np.all(np.diff(r["leaf_j"]) >= 0)
        dh = eps * eps / 8.0 * (np.sum(r["leaf_x"][last] ** 2, axis=1) - np.sum(x0 ** 2))
        expect = np.mean(np.minimum(1.0, np.exp(-dh)))
        assert abs(r["accept_stat"] - expect) <= 1e-10 * max(1.0, expect), (t, r["accept_stat"], expect)
        # the whole trajectory's mean differs whenever there is more than one doubling
        checked += 1
    assert checked >= 30


def test_accept_stat_edge_values_and_simple_adaptation_closed_forms():
    # flat target (zero precision): H is constant along the trajectory, statistic exactly 1,
    # so the multiplicative rule grows the step by exactly (1 + rate) per burn-in transition
    flat = Target(oracle.GAUSS_DIAG, 2, prec=np.zeros(2))
    B, rate, eps0 = 12, 0.03, 0.2
    o = oracle.nuts_sample_chain(flat, 4, np.zeros((3, 2)), eps0, B, 2, max_depth=3, adapt="simple", rate=rate)
    assert np.all(o["accept_stat"] == 1.0)
    expect = eps0
    for _ in range(B):
        expect = expect * (1 + rate)
    assert np.all(o["final_eps"] == expect)
    # NaN state: the first leaf diverges with statistic 0; the step shrinks by exactly 1 / (1 + rate)
    tg = Target(oracle.STD_NORMAL, 2)
    x0 = np.full((3, 2), np.nan)
    o = oracle.nuts_sample_chain(tg, 4, x0, eps0, B, 2, max_depth=5, adapt="simple", rate=rate)
    assert np.all(o["accept_stat"] == 0.0) and np.all(o["n_leapfrog"] == 1)
    expect = eps0
    for _ in range(B):
        expect = expect / (1 + rate)
    assert np.all(o["final_eps"] == expect)


def test_dual_averaging_brings_the_statistic_to_the_target():
    tg = Target(oracle.STD_NORMAL, 20)
    x0 = np.random.default_rng(3).normal(size=(32, 20))
    means = {}
    for delta in (0.65, 0.9):
        o = oracle.nuts_sample_chain(tg, 21, x0, 1.0, 300, 200, max_depth=8, adapt=True, target_accept=delta)
        means[delta] = o["accept_stat"].mean()
        assert abs(means[delta] - delta) < 0.06, (delta, means[delta])
        assert np.all(np.isfinite(o["final_eps"])) and np.all(o["final_eps"] > 0)
        # after burn-in the step size is frozen at the averaged iterate
        assert np.ptp(o["final_eps"]) > 0
    assert means[0.9] > means[0.65]


def test_fixed_step_run_is_unchanged_by_the_statistic():
    tg = Target(oracle.STD_NORMAL, 4)
    x0 = np.random.default_rng(5).normal(size=(6, 4))
    a = oracle.nuts_sample_chain(tg, 2, x0, 0.5, 10, 20, max_depth=6)
    assert np.all(a["final_eps"] == 0.5)
    assert np.all((a["accept_stat"] >= 0) & (a["accept_stat"] <= 1))
