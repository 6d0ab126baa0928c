"""The plain form's merged transition on the element-wise targets (N(0, I),
diagonal Gaussian) and the dense Gaussian.

A transition is L launches: the first also draws the momentum, forms H0 and
makes the first half kick; the last also forms H at the trajectory's end,
takes the Metropolis decision and writes the accepted state, gradient and
log-probability (a rejected chain keeps them bitwise).  One-step parity with
the FP64 oracle across the launch shapes -- element-wise: lanes per chain
(1, 4, 16, 64), slots per lane of the last step (up to 32, D = 2048), vector
and scalar row access; dense: 1 to 8 tiles of 16 dims, a ragged last chain
tile -- for L = 1 (first and last step in one launch), L = 2 (no middle
step), and the shapes outside the merged kernels (element-wise L = 1 or
D > 2048, dense D > 128) that run one kernel per phase.
"""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import decision_report, gpu_available, one_step, rel_err_rows, to_np

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_2002_01184_amd import hmc  # noqa: E402


def _state(w, seed):
    # a draw near the target's own scale (1.3 standard deviations per mode)
    rng = np.random.default_rng(seed)
    dt = np.float64 if w.state_dtype == "f64" else np.float32
    z = rng.standard_normal((w.num_chains, w.dim)) * 1.3
    if w.kind == W.GAUSS_DIAG:
        z = z * np.sqrt(w.extra["lam"])
    elif w.kind == W.GAUSS_DENSE:
        z = (z * np.sqrt(w.extra["lam"])) @ w.extra["Q"].T
    return np.ascontiguousarray(z.astype(dt))


CASES = {
    # name: (workload, tolerance on the proposal)
    "f32_D1000_vec4_G64_NE16": (W.gauss_diag(dim=1000, num_chains=96, L=4, step_size=0.05), 1e-5),
    "f64_D6_vec2_G4_NE2": (W.std_normal_1d(num_chains=200, dim=6, state_dtype="f64", L=3, step_size=0.5), 1e-12),
    "f64_D1_G1": (W.std_normal_1d(num_chains=300, dim=1, state_dtype="f64", L=3, step_size=1.5), 1e-12),
    "f32_D13_G4_NE4": (W.gauss_diag(dim=13, num_chains=150, L=5, step_size=0.08), 1e-5),
    "f32_D64_G16_NE4_L2": (W.gauss_diag(dim=64, num_chains=130, L=2, step_size=0.1), 1e-5),
    "f32_D2048_G64_NE32": (W.gauss_diag(dim=2048, num_chains=40, L=3, step_size=0.04), 1e-5),
    "f64_D2047_G64_NE32": (W.gauss_diag(dim=2047, num_chains=33, L=3, step_size=0.04, state_dtype="f64"), 1e-12),
    "f32_D2049_per_phase": (W.gauss_diag(dim=2049, num_chains=20, L=3, step_size=0.04), 1e-5),
    "f64_D3_L1_per_phase": (W.std_normal_1d(num_chains=100, dim=3, state_dtype="f64", L=1, step_size=0.9), 1e-12),
    "dense_D100_NT7": (W.gauss_dense(dim=100, num_chains=70, L=6, step_size=0.1, seed=2), 1e-5),
    "dense_D16_NT1_L1": (W.gauss_dense(dim=16, num_chains=33, L=1, step_size=0.2, seed=3), 1e-5),
    "dense_D128_NT8_L2": (W.gauss_dense(dim=128, num_chains=48, L=2, step_size=0.08, seed=4), 1e-5),
    "dense_D5_NT1": (W.gauss_dense(dim=5, num_chains=17, L=4, step_size=0.1, seed=5), 1e-5),
    "dense_D129_per_phase": (W.gauss_dense(dim=129, num_chains=20, L=3, step_size=0.08, seed=6), 1e-5),
}


@pytest.mark.parametrize("name", list(CASES))
def test_one_step_parity_and_select(name):
    w, tol = CASES[name]
    s = hmc.sampler_for(w, form=hmc.HMC_FORM_PLAIN)
    errs, agree_all = [], []
    for k, t in enumerate([0, 5, 777]):
        xs = _state(w, 10 + k)
        g, o = one_step(w, s, xs, t)
        e = np.maximum(rel_err_rows(g["proposed_state"], o["x_prop"]),
                       rel_err_rows(g["proposed_momentum"], o["p_prop"]))
        errs.append(e)
        agree, margins, dh_err = decision_report(g, o, w.seed, t)
        agree_all.append(agree)
        if len(margins):
            assert np.all(margins <= 10 * np.max(dh_err) + 1e-12)
        xg = to_np(s.get_state()[0])
        acc = g["is_accepted"].astype(bool)
        assert np.array_equal(xg[~acc], xs[~acc])          # rejected: untouched
        assert np.array_equal(xg[acc], g["proposed_state"][acc])
    e = np.concatenate(errs)
    print(f"{name}: proposal rel err p50={np.median(e):.2e} max={e.max():.2e}; agree {np.mean(agree_all):.5f}")
    assert e.max() <= tol
    assert np.mean(agree_all) >= (1.0 if w.state_dtype == "f64" else 0.999)
    s.close()


@pytest.mark.parametrize("name", ["f32_D1000_vec4_G64_NE16", "f64_D6_vec2_G4_NE2", "f32_D64_G16_NE4_L2",
                                  "dense_D100_NT7", "dense_D16_NT1_L1"])
def test_run_keeps_gradient_and_logp_of_the_kept_state(name):
    # after a run with rejections, the cached gradient and logp are those of the
    # current state: one more transition from the fetched state on a fresh
    # sampler (which recomputes them) gives bitwise the same result
    w, _ = CASES[name]
    s = hmc.sampler_for(w, form=hmc.HMC_FORM_PLAIN)
    x0 = torch.from_numpy(_state(w, 3)).to(s.device)
    s.set_state(x0, None, 0)
    out = s.sample_chain(6, 0)
    acc = to_np(out["is_accepted"]).astype(bool)
    assert acc.any() and not acc.all()
    a = s.step()
    x, e, t = s.get_state()
    s.close()
    s2 = hmc.sampler_for(w, form=hmc.HMC_FORM_PLAIN)
    s2.set_state(torch.from_numpy(to_np(out["samples"][-1])).to(s2.device), e, t - 1)
    b = s2.step()
    assert torch.equal(a["is_accepted"], b["is_accepted"])
    assert torch.equal(a["log_accept_ratio"], b["log_accept_ratio"])
    assert torch.equal(x, s2.get_state()[0])
    s2.close()


@pytest.mark.parametrize("case", ["diag", "dense"])
def test_plain_and_graph_forms_bitwise_equal(case):
    w = (W.gauss_diag(dim=300, num_chains=257, L=4, step_size=0.07, adapt=True) if case == "diag"
         else W.gauss_dense(dim=50, num_chains=100, L=5, step_size=0.1, adapt=True))
    outs = []
    for form in [hmc.HMC_FORM_PLAIN, hmc.HMC_FORM_GRAPH]:
        s = hmc.sampler_for(w, form=form)
        outs.append(s.sample_chain(5, 5, adapt=True))
        s.close()
    for k in ["samples", "is_accepted", "log_accept_ratio", "step_size", "target_log_prob"]:
        assert torch.equal(outs[0][k], outs[1][k]), k
