"""Pins of the oracle's HMC transition against closed forms, invariants and
brute force (nothing here re-types the oracle's own code).

* Leapfrog on a quadratic target is linear.  Per eigenmode a of the precision,
  one kick-drift-kick step is M = [[1 - e^2 a/2, e], [-e a (1 - e^2 a/4), 1 - e^2 a/2]]
  and M^L = cos(L th) I + sin(L th)/sin(th) (M - cos(th) I) with cos th = 1 - e^2 a/2.
  For the paper's example (N(0,1), step 1.5, 3 steps) M^3 is dyadic:
  [[47/128, -45/32], [315/512, 47/128]].
* The integrator conserves the shadow energy a (1 - e^2 a/4) y^2 + p^2 per mode, so
  dH = sum_modes (e^2 a^2 / 8) (y_L^2 - y_0^2).
* From x0 = 0 the first transition of the example has dH = c p0^2 with
  c = (9/32)(45/32)^2 and mean acceptance (1 + 2c)^-1/2 = 0.688043.
* In stationarity the example's mean acceptance is 0.760231 and the lag-1
  autocorrelation of x is 0.354968 (2-D quadrature, recomputed below).
* Reversibility, O(e^2) energy error, volume preservation, finite-difference
  gradients, a logistic model with X = 0 reducing to its prior, posterior
  moments by quadrature, Gaussian moments, and batch semantics.
"""
import numpy as np
import pytest

import oracle
from oracle import Target


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# ------------------------------------------------------- closed forms --
def test_leapfrog_paper_example_is_dyadic_map():
    tg = Target(oracle.STD_NORMAL, 1)
    rng = np.random.default_rng(0)
    for _ in range(200):
        x0, p0 = rng.normal(size=2) * 3
        x3, p3, lp, g = oracle.leapfrog(tg, 1.5, 3, [x0], [p0])
        assert x3[0] == pytest.approx(47 / 128 * x0 - 45 / 32 * p0, rel=1e-14, abs=1e-14)
        assert p3[0] == pytest.approx(315 / 512 * x0 + 47 / 128 * p0, rel=1e-14, abs=1e-14)
        assert lp == pytest.approx(-0.5 * x3[0] ** 2, rel=1e-14)
        assert g[0] == -x3[0]


def _mode_map(a, eps, L):
    """Closed-form L-step leapfrog matrix for one mode of precision a."""
    M = np.array([[1 - eps ** 2 * a / 2, eps], [-eps * a * (1 - eps ** 2 * a / 4), 1 - eps ** 2 * a / 2]])
    c = 1 - eps ** 2 * a / 2
    th = np.arccos(c)
    return np.cos(L * th) * np.eye(2) + np.sin(L * th) / np.sin(th) * (M - c * np.eye(2))


def _spd(D, seed, lo=0.3, hi=5.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(D, D)))
    a = np.exp(rng.uniform(np.log(lo), np.log(hi), D))
    return Q, a, (Q * a) @ Q.T


@pytest.mark.parametrize("kind", ["diag", "dense"])
def test_leapfrog_gaussian_matches_eigen_closed_form(kind):
    D, eps, L = 6, 0.37, 11
    if kind == "dense":
        Q, a, P = _spd(D, 1)
        tg = Target(oracle.GAUSS_DENSE, D, prec=P)
    else:
        Q, a = np.eye(D), np.linspace(0.2, 4.0, D)
        tg = Target(oracle.GAUSS_DIAG, D, prec=a)
    rng = np.random.default_rng(2)
    x0, p0 = rng.normal(size=D), rng.normal(size=D)
    xL, pL, lpL, gL = oracle.leapfrog(tg, eps, L, x0, p0)
    y0, q0 = Q.T @ x0, Q.T @ p0
    yL = np.empty(D)
    qL = np.empty(D)
    for i in range(D):
        yL[i], qL[i] = _mode_map(a[i], eps, L) @ np.array([y0[i], q0[i]])
    assert _rel(xL, Q @ yL) < 1e-12
    assert _rel(pL, Q @ qL) < 1e-12
    assert lpL == pytest.approx(-0.5 * np.sum(a * yL ** 2), rel=1e-12)


@pytest.mark.parametrize("kind", ["std", "dense"])
def test_delta_h_matches_shadow_energy_closed_form(kind):
    if kind == "std":
        D, eps, L = 1, 1.5, 3
        Q, a = np.eye(1), np.ones(1)
        tg = Target(oracle.STD_NORMAL, 1)
    else:
        D, eps, L = 5, 0.3, 7
        Q, a, P = _spd(D, 3)
        tg = Target(oracle.GAUSS_DENSE, D, prec=P)
    C = 64
    x0 = np.random.default_rng(4).normal(size=(C, D))
    out = oracle.step(tg, L, seed=9, t=5, eps=eps, x=x0)
    p0 = oracle.momentum(9, C, 5, D)           # the momenta the transition drew
    for c in range(C):
        y0, q0 = Q.T @ x0[c], Q.T @ p0[c]
        yL = np.array([(_mode_map(a[i], eps, L) @ [y0[i], q0[i]])[0] for i in range(D)])
        dh = np.sum(eps ** 2 * a ** 2 / 8 * (yL ** 2 - y0 ** 2))
        assert out["delta_h"][c] == pytest.approx(dh, rel=1e-9, abs=1e-12)
        if kind == "std":
            assert out["delta_h"][c] == pytest.approx(9 / 32 * (yL[0] ** 2 - y0[0] ** 2), rel=1e-9, abs=1e-12)


def test_first_transition_acceptance_from_zero():
    C = 40000
    tg = Target(oracle.STD_NORMAL, 1)
    out = oracle.step(tg, 3, seed=0, t=0, eps=1.5, x=np.zeros((C, 1)))
    c = 9 / 32 * (45 / 32) ** 2
    assert c == 0.556182861328125
    p0 = oracle.momentum(0, C, 0, 1)[:, 0]
    assert np.allclose(out["delta_h"], c * p0 ** 2, rtol=1e-12, atol=1e-15)
    alpha = np.exp(np.minimum(0, out["log_accept_ratio"]))
    expected = (1 + 2 * c) ** -0.5            # = 0.688043
    se = np.std(alpha) / np.sqrt(C)
    assert abs(alpha.mean() - expected) < 4 * se
    acc = out["accepted"].mean()
    assert abs(acc - expected) < 4 * np.sqrt(expected * (1 - expected) / C)


def _stationary_quadrature(h=0.005):
    g = np.arange(-9, 9 + h / 2, h)
    w = np.exp(-0.5 * g * g) / np.sqrt(2 * np.pi) * h
    acc = lag = 0.0
    for i0 in range(0, len(g), 400):
        x0, wx = g[i0:i0 + 400, None], w[i0:i0 + 400, None]
        x3 = 47 / 128 * x0 - 45 / 32 * g[None, :]
        a = np.minimum(1, np.exp(-9 / 32 * (x3 * x3 - x0 * x0)))
        acc += np.sum(wx * w[None, :] * a)
        lag += np.sum(wx * w[None, :] * (a * x0 * x3 + (1 - a) * x0 * x0))
    return acc, lag


def test_paper_example_stationary_acceptance_and_autocorrelation():
    acc_q, lag_q = _stationary_quadrature()
    assert acc_q == pytest.approx(0.760231, abs=2e-6)
    assert lag_q == pytest.approx(0.354968, abs=2e-6)
    C, T = 20000, 20
    tg = Target(oracle.STD_NORMAL, 1)
    x0 = np.random.default_rng(5).normal(size=(C, 1))      # a stationary start
    out = oracle.sample_chain(tg, 3, seed=1, x0=x0, eps0=1.5, num_burnin=0, num_results=T)
    xs = np.concatenate([x0[None], out["samples"]], 0)[:, :, 0]     # [T+1, C]
    alpha = np.exp(np.minimum(0, out["log_accept_ratio"]))
    # chains are independent; transitions within a chain are correlated: use chain means
    per_chain = alpha.mean(0)
    assert abs(per_chain.mean() - acc_q) < 4 * per_chain.std() / np.sqrt(C)
    prod = (xs[1:] * xs[:-1]).mean(0)
    assert abs(prod.mean() - lag_q) < 4 * prod.std() / np.sqrt(C)
    # and the paper's example configuration itself: 100 chains x 100 kept draws
    ex = oracle.sample_chain(tg, 3, seed=0, x0=np.zeros((100, 1)), eps0=1.5, num_burnin=300,
                             num_results=100)
    s = ex["samples"].ravel()
    assert abs(s.mean()) < 0.058 and abs(s.var() - 1) < 0.077
    assert abs(ex["is_accepted"].mean() - 0.760) < 0.03
    assert np.all(ex["step_size"] == 1.5)


# ---------------------------------------------------------- invariants --
def _logreg_target(N=40, D=3, seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(N, D))
    w = rng.normal(size=D)
    y = (rng.uniform(size=N) < 1 / (1 + np.exp(-X @ w))).astype(float)
    return Target(oracle.LOGREG, D, X=X, y=y, prior_scale=scale)


def test_reversibility_logreg_and_dense():
    for tg in [_logreg_target(), Target(oracle.GAUSS_DENSE, 5, prec=_spd(5, 7)[2])]:
        rng = np.random.default_rng(8)
        x0, p0 = rng.normal(size=tg.dim) * 0.5, rng.normal(size=tg.dim)
        xL, pL, _, _ = oracle.leapfrog(tg, 0.1, 25, x0, p0)
        xb, pb, _, _ = oracle.leapfrog(tg, 0.1, 25, xL, -pL)
        assert np.max(np.abs(xb - x0)) < 1e-12 * 50
        assert np.max(np.abs(-pb - p0)) < 1e-12 * 50


def _delta_h(tg, x0, p0, eps, L):
    lp0, _ = oracle.logp_grad(tg, x0)
    xL, pL, lpL, _ = oracle.leapfrog(tg, eps, L, x0, p0)
    return (-lpL + 0.5 * pL @ pL) - (-lp0 + 0.5 * p0 @ p0)


def test_energy_error_is_second_order():
    tg = _logreg_target(N=60, D=4, seed=1)
    rng = np.random.default_rng(2)
    ratios = []
    for _ in range(5):
        x0, p0 = rng.normal(size=4) * 0.3, rng.normal(size=4)
        d1 = _delta_h(tg, x0, p0, 0.02, 20)
        d2 = _delta_h(tg, x0, p0, 0.01, 40)
        ratios.append(d1 / d2)
    assert np.all(np.abs(np.array(ratios) - 4) < 0.4), ratios


def test_volume_preservation():
    tg = _logreg_target(N=30, D=2, seed=3)
    z0 = np.array([0.3, -0.2, 0.7, 0.1])
    h = 1e-5

    def flow(z):
        xL, pL, _, _ = oracle.leapfrog(tg, 0.15, 9, z[:2], z[2:])
        return np.concatenate([xL, pL])
    J = np.empty((4, 4))
    for j in range(4):
        e = np.zeros(4)
        e[j] = h
        J[:, j] = (flow(z0 + e) - flow(z0 - e)) / (2 * h)
    assert abs(np.linalg.det(J) - 1) < 1e-6


@pytest.mark.parametrize("which", ["logreg", "dense", "diag", "std"])
def test_gradient_matches_finite_differences(which):
    D = 4
    if which == "logreg":
        tg = _logreg_target(N=50, D=D, seed=4, scale=1.7)
    elif which == "dense":
        tg = Target(oracle.GAUSS_DENSE, D, prec=_spd(D, 9)[2])
    elif which == "diag":
        tg = Target(oracle.GAUSS_DIAG, D, prec=np.array([0.5, 1.0, 3.0, 10.0]))
    else:
        tg = Target(oracle.STD_NORMAL, D)
    x = np.random.default_rng(5).normal(size=D)
    _, g = oracle.logp_grad(tg, x)
    h = 1e-6
    fd = np.empty(D)
    for i in range(D):
        e = np.zeros(D)
        e[i] = h
        fd[i] = (oracle.logp_grad(tg, x + e)[0] - oracle.logp_grad(tg, x - e)[0]) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-7)


def test_logreg_with_zero_design_is_its_prior():
    N, D, s = 17, 3, 2.0
    tg = Target(oracle.LOGREG, D, X=np.zeros((N, D)), y=np.ones(N), prior_scale=s)
    x = np.array([0.3, -1.2, 2.0])
    lp, g = oracle.logp_grad(tg, x)
    lp0, _ = oracle.logp_grad(tg, np.zeros(D))
    assert lp - lp0 == pytest.approx(-0.5 * x @ x / s ** 2, rel=1e-14)
    assert np.allclose(g, -x / s ** 2, rtol=1e-14)
    assert lp0 == pytest.approx(-N * np.log(2), rel=1e-14)   # softplus(0) = log 2 per row


@pytest.mark.slow
def test_logreg_posterior_moments_match_quadrature():
    # D = 1: the posterior by brute-force quadrature on a grid
    rng = np.random.default_rng(6)
    N = 25
    X = rng.normal(size=(N, 1))
    y = (rng.uniform(size=N) < 1 / (1 + np.exp(-1.3 * X[:, 0]))).astype(float)
    tg = Target(oracle.LOGREG, 1, X=X, y=y)
    grid = np.linspace(-8, 8, 40001)
    z = grid[:, None] * X[None, :, 0]
    logpost = np.sum(y * z - np.logaddexp(0, z), 1) - 0.5 * grid ** 2
    w = np.exp(logpost - logpost.max())
    w /= w.sum()
    m_q = np.sum(w * grid)
    v_q = np.sum(w * (grid - m_q) ** 2)
    C = 4000
    out = oracle.sample_chain(tg, 5, seed=3, x0=np.zeros((C, 1)), eps0=0.3, num_burnin=50,
                              num_results=50)
    s = out["samples"][:, :, 0]
    chain_means = s.mean(0)
    assert abs(chain_means.mean() - m_q) < 5 * chain_means.std() / np.sqrt(C)
    v = s.var()
    assert abs(v - v_q) / v_q < 0.05


@pytest.mark.slow
def test_gaussian_sample_variances_along_eigenvectors():
    D = 4
    Q, a, P = _spd(D, 11, lo=0.5, hi=4.0)
    tg = Target(oracle.GAUSS_DENSE, D, prec=P)
    C = 4000
    x0 = np.random.default_rng(7).normal(size=(C, D))
    out = oracle.sample_chain(tg, 6, seed=2, x0=x0, eps0=0.25, num_burnin=20, num_results=40)
    y = out["samples"].reshape(-1, D) @ Q
    assert np.all(np.abs(y.mean(0)) < 5 * np.sqrt(1 / a / (C * 10)))
    assert np.allclose(y.var(0), 1 / a, rtol=0.06)


def test_batch_semantics_chains_are_independent():
    # Changing one chain's state leaves every other chain's results bitwise unchanged.
    tg = _logreg_target(N=20, D=3, seed=1)
    x = np.random.default_rng(3).normal(size=(8, 3))
    a = oracle.step(tg, 4, seed=5, t=2, eps=0.2, x=x)
    x2 = x.copy()
    x2[3] += 1.0
    b = oracle.step(tg, 4, seed=5, t=2, eps=0.2, x=x2)
    keep = np.arange(8) != 3
    for k in ["x", "logp", "x_prop", "p_prop", "delta_h", "accepted"]:
        assert np.array_equal(a[k][keep], b[k][keep]), k
    # and per-chain evaluation equals batched evaluation
    lp, g = oracle.logp_grad(tg, x)
    for c in range(8):
        lpc, gc = oracle.logp_grad(tg, x[c])
        assert lpc == lp[c] and np.array_equal(gc, g[c])


def test_rejected_chains_keep_state_bitwise_and_nan_rejects():
    tg = Target(oracle.STD_NORMAL, 2)
    x = np.array([[0.5, -0.5], [np.nan, 0.0], [1e200, 1.0]])
    out = oracle.step(tg, 3, seed=0, t=0, eps=1.5, x=x)
    assert not out["accepted"][1] and out["log_accept_ratio"][1] == -np.inf
    assert not out["accepted"][2]
    rej = ~out["accepted"]
    assert np.array_equal(out["x"][rej], x[rej], equal_nan=True)


# ------------------------------------------------------- driver + adapt --
def test_sample_chain_equals_iterated_steps():
    # burn-in transitions are not stored; sample r is the state after transition burnin + r
    tg = _logreg_target(N=30, D=3, seed=2)
    C, L, B, R = 16, 4, 3, 5
    x0 = np.random.default_rng(9).normal(size=(C, 3)) * 0.3
    out = oracle.sample_chain(tg, L, seed=4, x0=x0, eps0=0.2, num_burnin=B, num_results=R)
    x, lp, g = x0, None, None
    kept = []
    for t in range(B + R):
        st = oracle.step(tg, L, seed=4, t=t, eps=0.2, x=x, logp=lp, g=g)
        x, lp, g = st["x"], st["logp"], st["g"]
        if t >= B:
            kept.append(x)
            assert np.array_equal(out["is_accepted"][t - B], st["accepted"])
            assert np.array_equal(out["target_log_prob"][t - B], st["logp"])
    assert np.array_equal(out["samples"], np.stack(kept))
    assert np.array_equal(out["final_x"], x)


def test_dual_averaging_fixed_point_and_direction():
    eps0 = 0.1
    mu = np.log(10 * eps0)
    le, hb, leb, mu_o = oracle.dual_avg_run(eps0, [0.8] * 5000)
    assert mu_o == pytest.approx(mu)
    assert np.all(hb == 0) and np.allclose(le, mu, rtol=0, atol=1e-15)
    assert abs(leb[-1] - mu) < 1e-6 and abs(leb[0] - mu) < 1e-15   # first weight is 1^-kappa = 1
    le1, _, _, _ = oracle.dual_avg_run(eps0, [1.0] * 20)     # always accepting -> grow
    le0, _, _, _ = oracle.dual_avg_run(eps0, [0.0] * 20)     # never accepting -> shrink
    assert np.all(le1 > mu) and np.all(le0 < mu)
    # H-bar is the (t0-shrunk) running mean of (delta - alpha): alpha = 0.3 for m=1..M
    _, hb3, _, _ = oracle.dual_avg_run(eps0, [0.3] * 7)
    assert hb3[-1] == pytest.approx(0.5 * 7 / (7 + 10), rel=1e-13)


def test_dual_averaging_first_iterates_by_hand():
    # Hoffman & Gelman (2014) eq. 6 with gamma 0.05, t0 10, kappa 0.75, delta 0.8, eps0 = 0.5 (mu = log 5,
    # not 0) and scripted statistics 0.2, 0.9, 0.5. The values below were simplified by hand:
    #   Hbar_1 = 0.6/11, Hbar_2 = 0.5/12, Hbar_3 = 0.8/13 (Hbar_m = sum_i (delta - alpha_i) / (m + t0)),
    #   log eps_m = log 5 - 20 sqrt(m) Hbar_m = log 5 - 12/11, log 5 - 5 sqrt(2)/6, log 5 - 16 sqrt(3)/13,
    #   log ebar_1 = log eps_1 (first weight 1^-kappa = 1), then the weight of the new iterate is m^-kappa.
    le, hb, leb, mu = oracle.dual_avg_run(0.5, [0.2, 0.9, 0.5])
    l5 = np.log(5.0)
    assert mu == pytest.approx(l5, rel=1e-15)
    assert hb == pytest.approx([0.6 / 11, 0.5 / 12, 0.8 / 13], rel=1e-14)
    e1, e2, e3 = l5 - 12 / 11, l5 - 5 * np.sqrt(2) / 6, l5 - 16 * np.sqrt(3) / 13
    assert le == pytest.approx([e1, e2, e3], rel=1e-14)
    w2, w3 = 2.0 ** -0.75, 3.0 ** -0.75
    b2 = w2 * e2 + (1 - w2) * e1
    assert leb == pytest.approx([e1, b2, w3 * e3 + (1 - w3) * b2], rel=1e-14)
    # numerically: log ebar = 0.51849..., 0.53167..., 0.38339... (iterates move, so a swapped weight shows)
    assert leb[1] != pytest.approx(w2 * e1 + (1 - w2) * e2, rel=1e-3)


def test_dual_averaging_iterate_average_special_cases():
    # kappa = 1: the averaged iterate is the arithmetic (Polyak) mean of log eps_1..m;
    # kappa = 0: it is the last iterate; any kappa in (0, 1]: a convex combination with weights
    # w_i = i^-kappa prod_{j>i} (1 - j^-kappa), which sum to 1 (the unrolled recursion).
    rng = np.random.default_rng(17)
    alphas = rng.uniform(0, 1, size=60)
    eps0 = 0.37
    le, hb, leb, _ = oracle.dual_avg_run(eps0, alphas, kappa=1.0)
    m = np.arange(1, 61)
    assert leb == pytest.approx(np.cumsum(le) / m, rel=1e-12, abs=1e-13)
    # Hbar_m is the t0-shrunk running mean of (delta - alpha)
    assert hb == pytest.approx(np.cumsum(0.8 - alphas) / (m + 10.0), rel=1e-12, abs=1e-15)
    le0, _, leb0, _ = oracle.dual_avg_run(eps0, alphas, kappa=0.0)
    assert np.array_equal(leb0, le0)
    le7, _, leb7, _ = oracle.dual_avg_run(eps0, alphas, kappa=0.75)
    M = 60
    w = np.array([i ** -0.75 * np.prod([1 - j ** -0.75 for j in range(i + 1, M + 1)]) for i in range(1, M + 1)])
    assert w.sum() == pytest.approx(1.0, rel=1e-13)
    assert leb7[-1] == pytest.approx(np.dot(w, le7), rel=1e-12)
    # the log step sizes themselves vary by O(1) here, so these identities are not vacuous
    assert np.ptp(le7) > 1.0


def test_dual_averaging_reaches_target_acceptance():
    tg = Target(oracle.GAUSS_DIAG, 10, prec=np.linspace(1, 25, 10))
    C = 200
    x0 = np.random.default_rng(1).uniform(-2, 2, size=(C, 10))
    out = oracle.sample_chain(tg, 10, seed=0, x0=x0, eps0=0.01, num_burnin=400, num_results=300,
                              adapt=True)
    alpha = np.exp(np.minimum(0, out["log_accept_ratio"]))
    assert abs(alpha.mean() - 0.8) < 0.05
    # step size frozen after burn-in, per chain
    assert np.all(out["step_size"] == out["step_size"][0:1])
    assert np.allclose(out["final_eps"], out["step_size"][-1])


def test_step_on_selected_chains_equals_step_on_all():
    # step_chains runs chosen chain ids only (for full-size workloads); the streams are
    # keyed by chain id, so it equals the all-chain step on those rows, bitwise
    tg = _logreg_target(N=40, D=5, seed=8)
    x = np.random.default_rng(3).normal(size=(23, 5)) * 0.4
    full = oracle.step(tg, 4, seed=6, t=9, eps=0.1, x=x)
    ids = [0, 4, 5, 22]
    sub = oracle.step_chains(tg, 4, 6, 9, 0.1, x[ids], ids, nthreads=3)
    for k in ("x", "logp", "g", "x_prop", "p_prop", "logp_prop", "delta_h", "log_accept_ratio", "accepted"):
        assert np.array_equal(full[k][ids], sub[k]), k
