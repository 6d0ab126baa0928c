"""Pins of the oracle's transformed kernel (paper Sec. 4.1,
TransformedTransitionKernel) with the diagonal affine bijector
x = shift + scale * z: the chain runs on z against the pulled-back target
l(shift + scale z) and its samples are pushed forward.

  * on a Gaussian with precision P the pulled-back target has precision
    S P S (S = diag(scale)), so the z-space leapfrog is the per-eigenmode closed
    form of S P S; with scale = 1/sqrt(diag P) on a diagonal Gaussian every mode
    has precision 1;
  * the shift does not change the x-space chain (the dynamics are
    translation invariant);
  * scale 1 and shift 0 give the untransformed chain bit for bit;
  * pushed-forward samples of N(0, diag(lambda)) have variances lambda.
"""
import numpy as np
import pytest

import oracle
from oracle import Target


def _mode_map(a, eps, L):
    M = np.array([[1 - eps ** 2 * a / 2, eps], [-eps * a * (1 - eps ** 2 * a / 4), 1 - eps ** 2 * a / 2]])
    c = 1 - eps ** 2 * a / 2
    th = np.arccos(c)
    return np.cos(L * th) * np.eye(2) + np.sin(L * th) / np.sin(th) * (M - c * np.eye(2))


def test_pulled_back_dense_gaussian_is_closed_form_of_SPS():
    D, eps, L = 5, 0.3, 8
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.normal(size=(D, D)))
    P = (Q * np.linspace(0.5, 4.0, D)) @ Q.T
    s = np.linspace(0.6, 1.4, D)
    tz = Target(oracle.GAUSS_DENSE, D, prec=P).transformed(s, shift=rng.normal(size=D) * 0 + 0.0)
    A = (s[:, None] * P) * s[None, :]
    a, V = np.linalg.eigh(A)
    z0, p0 = rng.normal(size=D), rng.normal(size=D)
    zL, pL, lpL, gL = oracle.leapfrog(tz, eps, L, z0, p0)
    y0, q0 = V.T @ z0, V.T @ p0
    yq = np.array([_mode_map(a[i], eps, L) @ np.array([y0[i], q0[i]]) for i in range(D)])
    assert np.allclose(zL, V @ yq[:, 0], rtol=1e-11, atol=1e-12)
    assert np.allclose(pL, V @ yq[:, 1], rtol=1e-11, atol=1e-12)
    assert np.allclose(gL, -A @ zL, rtol=1e-11, atol=1e-12)


def test_whitening_scale_gives_unit_modes():
    lam = np.array([0.01, 1.0, 100.0])
    tz = Target(oracle.GAUSS_DIAG, 3, prec=1 / lam).transformed(np.sqrt(lam))
    z0, p0 = np.array([0.3, -1.0, 2.0]), np.array([1.0, 0.5, -0.7])
    zL, pL, _, _ = oracle.leapfrog(tz, 0.4, 7, z0, p0)
    for i in range(3):
        y, q = _mode_map(1.0, 0.4, 7) @ np.array([z0[i], p0[i]])
        assert zL[i] == pytest.approx(y, rel=1e-12, abs=1e-14) and pL[i] == pytest.approx(q, rel=1e-12, abs=1e-14)


def test_shift_does_not_change_the_x_chain():
    tg = Target(oracle.LOGREG, 2, X=np.random.default_rng(0).normal(size=(30, 2)),
                y=(np.arange(30) % 2).astype(float))
    x0 = np.random.default_rng(1).uniform(-1, 1, size=(6, 2))
    a = oracle.transformed_sample_chain(tg, [0.5, 2.0], None, 4, 3, x0, 0.2, 10, 20)
    b = oracle.transformed_sample_chain(tg, [0.5, 2.0], [0.25, -0.75], 4, 3, x0, 0.2, 10, 20)
    assert np.array_equal(a["is_accepted"], b["is_accepted"])
    assert np.allclose(a["samples"], b["samples"], rtol=0, atol=1e-12)


def test_unit_scale_is_the_untransformed_chain():
    tg = Target(oracle.GAUSS_DIAG, 4, prec=np.array([0.5, 1.0, 2.0, 4.0]))
    x0 = np.random.default_rng(2).uniform(-2, 2, size=(10, 4))
    a = oracle.transformed_sample_chain(tg, np.ones(4), None, 5, 7, x0, 0.3, 20, 30, adapt=True)
    b = oracle.sample_chain(tg, 5, 7, x0, 0.3, 20, 30, adapt=True)
    assert np.array_equal(a["samples"], b["samples"]) and np.array_equal(a["final_eps"], b["final_eps"])


def test_pushed_forward_variances():
    lam = np.logspace(-2, 2, 6)
    tg = Target(oracle.GAUSS_DIAG, 6, prec=1 / lam)
    x0 = np.random.default_rng(3).normal(size=(200, 6)) * np.sqrt(lam)
    r = oracle.transformed_sample_chain(tg, np.sqrt(lam), None, 5, 1, x0, 0.3, 50, 300)   # angle ~pi/2
    v = r["samples"].reshape(-1, 6).var(0)
    assert np.allclose(v / lam, 1.0, atol=0.05)
