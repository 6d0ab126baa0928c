"""GPU parity of the transformed kernel (paper Sec. 4.1, TransformedTransitionKernel
with the diagonal affine bijector x = shift + scale * z) against the oracle,
which runs plain HMC on z against the pulled-back target and pushes the
samples forward.  The plain form runs in x with scale multiplying the step in
every drift and kick; the fused Gaussian kernels run in z = x / scale against
the pulled-back precision.

Bars as for the plain transition: the paper's FP64 example agrees with the
oracle to 1e-12 with identical decisions over a whole run; FP32 one-step
proposals within 1e-5 (compared in x; the momentum is z's on both sides) with
>= 99.9% of decisions agreeing; scale 1 is bitwise the untransformed chain.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import gpu_available, oracle_target, rel_err_rows, to_np

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_2002_01184_amd import hmc  # noqa: E402


@pytest.mark.parametrize("form", [hmc.HMC_FORM_PLAIN, hmc.HMC_FORM_GRAPH, hmc.HMC_FORM_FUSED])
def test_paper_example_transformed_run_matches_oracle(form):
    w = W.std_normal_1d()
    s = hmc.sampler_for(w, form=form)
    s.set_transform_scale([0.7])
    g = s.sample_chain(100, 300)
    s.close()
    o = oracle.transformed_sample_chain(oracle_target(w), [0.7], [0.3], w.num_leapfrog_steps, w.seed, w.x0,
                                        w.step_size, 300, 100)
    assert np.array_equal(to_np(g["is_accepted"]).astype(bool), o["is_accepted"])
    assert np.max(np.abs(to_np(g["samples"]) - o["samples"])) <= 1e-12


def _cases():
    return {
        "gauss_diag_101": W.gauss_diag(dim=101, num_chains=40, L=6, step_size=0.08),
        "gauss_dense_37": W.gauss_dense(dim=37, num_chains=45, L=7, step_size=0.1, seed=3),
        "logreg_77x3": W.logreg(77, 3, 33, L=4, step_size=0.2, seed=5),
        "logreg_1000x25": W.logreg(1000, 25, 64, L=10, step_size=0.05),
        "std_normal_7d": W.std_normal_1d(num_chains=60, dim=7, state_dtype="f32", L=5, step_size=0.4),
    }


def _form_cases():
    return [(name, form) for name in _cases() for form in ("plain", "fused")]


@pytest.mark.parametrize("name,form", _form_cases())
def test_transformed_one_step_parity(name, form):
    w = _cases()[name]
    scale = np.linspace(0.5, 1.5, w.dim)
    s = hmc.sampler_for(w, form=hmc.HMC_FORM_PLAIN if form == "plain" else hmc.HMC_FORM_FUSED)
    assert hmc.hmc_effective_form(s.ctx) == (hmc.HMC_FORM_PLAIN if form == "plain" else hmc.HMC_FORM_FUSED)
    s.set_transform_scale(scale)
    tz = oracle_target(w).transformed(scale)
    rng = np.random.default_rng(7)
    x = w.x0.copy()
    errs, agree = [], []
    for t in range(3):
        s.set_state(torch.from_numpy(np.ascontiguousarray(x)).cuda(), None, t)
        gp = {k: to_np(v) for k, v in s.step(want_proposal=True).items()}
        o = oracle.step(tz, w.num_leapfrog_steps, s.config.seed, t, w.step_size, x.astype(np.float64) / scale)
        errs.append(rel_err_rows(gp["proposed_state"], o["x_prop"] * scale))
        errs.append(rel_err_rows(gp["proposed_momentum"], o["p_prop"]))
        agree.append(gp["is_accepted"].astype(bool) == o["accepted"])
        x = (x + 0.2 * rng.standard_normal(x.shape)).astype(x.dtype)
    s.close()
    e = np.concatenate(errs)
    assert e.max() <= 1e-5, e.max()
    assert np.concatenate(agree).mean() >= 0.999


def _unit_cases():
    return {
        "logreg_plain": (W.logreg(300, 12, 48, L=6, step_size=0.05, seed=2), hmc.HMC_FORM_PLAIN),
        "dense_fused": (W.gauss_dense(dim=37, num_chains=45, L=7, step_size=0.1, seed=3), hmc.HMC_FORM_FUSED),
        "diag_fused": (W.gauss_diag(dim=101, num_chains=40, L=6, step_size=0.08), hmc.HMC_FORM_FUSED),
        "std_fp64_fused": (W.std_normal_1d(), hmc.HMC_FORM_FUSED),
        "logreg_fused": (W.logreg(300, 12, 48, L=6, step_size=0.05, seed=2), hmc.HMC_FORM_FUSED),
    }


@pytest.mark.parametrize("name", list(_unit_cases()))
def test_unit_scale_is_bitwise_the_untransformed_run(name):
    w, form = _unit_cases()[name]
    a = hmc.sampler_for(w, form=form)
    ra = a.sample_chain(8, 6, adapt=True)
    xa = a.get_state()[0]
    a.close()
    b = hmc.sampler_for(w, form=form)
    b.set_transform_scale(np.ones(w.dim))
    rb = b.sample_chain(8, 6, adapt=True)
    xb = b.get_state()[0]
    b.close()
    for k in ("samples", "is_accepted", "log_accept_ratio", "step_size"):
        assert torch.equal(ra[k], rb[k]), k
    assert torch.equal(xa, xb)


@pytest.mark.parametrize("form", [hmc.HMC_FORM_PLAIN, hmc.HMC_FORM_FUSED])
def test_whitening_speeds_up_an_ill_conditioned_gaussian(form):
    # variances 1e-2 .. 1e2: with scale = sqrt(lambda) every mode has unit precision in z
    w = W.gauss_diag(dim=50, num_chains=512, L=5, step_size=0.3, burnin=50, results=200)
    lam = w.extra["lam"]
    s = hmc.sampler_for(w, form=form)
    s.set_transform_scale(np.sqrt(lam))
    g = s.sample_chain(200, 50)
    s.close()
    v = to_np(g["samples"]).reshape(-1, 50).var(0)
    assert np.allclose(v / lam, 1.0, atol=0.08)


def test_transform_errors():
    w = W.logreg(200, 9, 96, L=5, step_size=0.05, seed=4)
    p = hmc.sampler_for(w, form=hmc.HMC_FORM_PLAIN)
    with pytest.raises(hmc.HMCError, match="finite and > 0"):
        p.set_transform_scale(-np.ones(9))
    p.close()


def test_fused_transformed_logistic_agrees_with_plain_in_distribution():
    # whole transformed runs of the fused (z-space) and plain (x-space) logistic kernels
    w = W.logreg(200, 5, 256, L=8, step_size=0.1, seed=12)
    scale = np.array([0.5, 2.0, 1.0, 0.8, 1.5])
    out = {}
    for form in (hmc.HMC_FORM_PLAIN, hmc.HMC_FORM_FUSED):
        s = hmc.sampler_for(w, form=form)
        assert hmc.hmc_effective_form(s.ctx) == form
        s.set_transform_scale(scale)
        out[form] = to_np(s.sample_chain(200, 100, adapt=True)["samples"]).reshape(-1, 5)
        s.close()
    m_p, m_f = out[hmc.HMC_FORM_PLAIN].mean(0), out[hmc.HMC_FORM_FUSED].mean(0)
    sd = out[hmc.HMC_FORM_PLAIN].std(0)
    assert np.all(np.abs(m_f - m_p) < 0.1 * sd + 1e-3), (m_p, m_f, sd)
    assert np.allclose(out[hmc.HMC_FORM_FUSED].std(0), sd, rtol=0.1)
