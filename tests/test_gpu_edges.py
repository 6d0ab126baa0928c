"""Edge and degenerate cases of the transition through the C ABI, against the
FP64 oracle (one-step mode, the bars of the parity tests: proposal error
<= 1e-5 in FP32 with >= 99.9% of decisions agreeing, 1e-12 in FP64):

  * one chain; a single leapfrog step (L = 1); one-dimensional FP32 states;
  * chain counts that leave a ragged last tile in every fused kernel (the
    4-chain logistic tile, the 16-chain dense tile, element-wise lane groups)
    and dimensions that leave ragged 4-dim blocks;
  * the largest shapes each fused kernel takes (logistic D = 32, N = 1024;
    dense D = 128; element-wise D = 2048);
  * runs with no kept draws (burn-in only) and with no transitions at all.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import decision_report, gpu_available, one_step, oracle_target, rel_err_rows, to_np

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_2002_01184_amd import hmc  # noqa: E402

FORMS = {"plain": hmc.HMC_FORM_PLAIN, "auto": hmc.HMC_FORM_AUTO}


def _edge_cases():
    return {
        "one_chain_logreg": W.logreg(300, 7, 1, L=6, step_size=0.05, seed=8),
        "one_chain_dense": W.gauss_dense(dim=20, num_chains=1, L=5, step_size=0.1, seed=2),
        "one_chain_diag": W.gauss_diag(dim=9, num_chains=1, L=4, step_size=0.1),
        "single_leapfrog_logreg": W.logreg(200, 5, 40, L=1, step_size=0.1, seed=3),
        "single_leapfrog_dense": W.gauss_dense(dim=16, num_chains=20, L=1, step_size=0.2, seed=4),
        "one_dim_fp32": W.std_normal_1d(num_chains=33, dim=1, state_dtype="f32", L=3, step_size=0.7),
        "ragged_logreg_tile": W.logreg(150, 6, 5, L=4, step_size=0.08, seed=6),
        "ragged_dense_tile": W.gauss_dense(dim=17, num_chains=17, L=4, step_size=0.1, seed=5),
        "ragged_elem_dims": W.gauss_diag(dim=257, num_chains=3, L=4, step_size=0.05),
        "max_logreg_fused": W.logreg(1024, 32, 12, L=3, step_size=0.02, seed=7),
        "max_dense_fused": W.gauss_dense(dim=128, num_chains=20, L=3, step_size=0.05, seed=9),
        "max_elem_fused": W.gauss_diag(dim=2048, num_chains=6, L=3, step_size=0.05),
    }


CASES = _edge_cases()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("form", ["plain", "auto"])
def test_edge_one_step_parity(name, form):
    w = CASES[name]
    s = hmc.sampler_for(w, form=FORMS[form])
    errs, agree_all = [], []
    for t, xs in ((0, w.x0), (5, (0.5 * w.x0).astype(w.x0.dtype))):
        g, o = one_step(w, s, np.ascontiguousarray(xs), t)
        errs.append(np.maximum(rel_err_rows(g["proposed_state"], o["x_prop"]),
                               rel_err_rows(g["proposed_momentum"], o["p_prop"])))
        agree, margins, dh_err = decision_report(g, o, w.seed, t)
        agree_all.append(agree)
        if len(margins):
            assert np.all(margins <= 10 * np.max(dh_err) + 1e-12)
    s.close()
    assert np.concatenate(errs).max() <= 1e-5
    assert np.mean(agree_all) >= 0.999


def test_fused_limits_are_the_fused_kernels():
    # the maximum shapes above do run on the fused kernels under the automatic form
    for name in ("max_logreg_fused", "max_dense_fused", "max_elem_fused"):
        s = hmc.sampler_for(CASES[name], form=hmc.HMC_FORM_AUTO)
        assert hmc.hmc_effective_form(s.ctx) == hmc.HMC_FORM_FUSED, name
        s.close()


@pytest.mark.parametrize("form", ["plain", "auto"])
def test_burn_in_only_and_empty_runs(form):
    w = W.gauss_dense(dim=12, num_chains=24, L=5, step_size=0.15, seed=3)
    s = hmc.sampler_for(w, form=FORMS[form])
    out = s.sample_chain(0, 7)                 # burn-in only: nothing kept, the state advances
    assert out["samples"].shape == (0, 24, 12)
    x, _, t = s.get_state()
    assert t == 7
    o = oracle.sample_chain(oracle_target(w), w.num_leapfrog_steps, w.seed, w.x0.astype(np.float64), w.step_size,
                            0, 7)
    assert np.max(rel_err_rows(to_np(x), o["samples"][-1])) <= 1e-5
    s.sample_chain(0, 0)                       # no transitions: nothing changes
    x2, _, t2 = s.get_state()
    assert t2 == 7 and torch.equal(x, x2)
    s.close()


def test_fp64_one_chain_full_run():
    w = W.std_normal_1d(num_chains=1)
    s = hmc.sampler_for(w, form=hmc.HMC_FORM_AUTO)
    g = s.sample_chain(50, 20)
    s.close()
    o = oracle.sample_chain(oracle_target(w), w.num_leapfrog_steps, w.seed, w.x0, w.step_size, 20, 50)
    assert np.array_equal(to_np(g["is_accepted"]).astype(bool), o["is_accepted"])
    assert np.max(np.abs(to_np(g["samples"]) - o["samples"])) <= 1e-12
