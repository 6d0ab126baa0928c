"""Pins of the oracle's No-U-Turn sampler (paper Sec. 3.2; Hoffman & Gelman
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
