"""GPU checks of the mixed-precision form: BF16 X and theta on MFMA with FP32
accumulation for the two gradient contractions, and an FP32-accurate
log-probability (theta split into three BF16 terms, softplus summed in FP64)
for dH.  The gradient error is a property of BF16 and is stated, not bound to
the FP32 tolerance; the log-probability that enters the accept test is bound.
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


def _bf16_case(N, D, C, seed=2, L=6, eps=0.004):
    return W.logreg(N, D, C, L=L, step_size=eps, bf16=True, init=0.05, seed=seed)


# shapes of every instantiation (32-dim k-steps 1, 2, 4, 6, 8, 12, 16) and of the padding
# (N not a multiple of 32 rows, D not a multiple of 32 or of 8)
@pytest.mark.parametrize("N,D,C", [(3000, 40, 300), (777, 25, 130), (4096, 256, 256), (3000, 64, 300), (2056, 128, 520),
                                   (1000, 190, 200), (3001, 300, 130), (2000, 512, 128), (1500, 417, 70)])
def test_bf16_form_one_step(N, D, C):
    w = _bf16_case(N, D, C)
    s = hmc.sampler_for(w, grad_bf16=True)
    assert s.form == "plain"
    g, o = one_step(w, s, np.ascontiguousarray(w.x0), 3)
    ex = rel_err_rows(g["proposed_state"], o["x_prop"])
    agree, margins, dh_err = decision_report(g, o, w.seed, 3)
    # the log-probability of the post-decision state is the accurate one
    xg, _, _ = s.get_state()
    lp_o, _ = oracle.logp_grad(oracle_target(w), to_np(xg).astype(np.float64))
    lp_err = np.abs(g["target_log_prob"] - lp_o) / np.abs(lp_o)
    print(f"bf16 N={N} D={D} C={C}: proposal rel err p50={np.median(ex):.2e} p99={np.quantile(ex, 0.99):.2e}; "
          f"logp rel err max {lp_err.max():.2e}; dH abs err p50 {np.median(dh_err):.2e}; decisions agree {agree:.4f}")
    assert np.quantile(ex, 0.99) < 2e-2
    assert lp_err.max() < 2e-6
    assert agree >= 0.97
    s.close()


def test_bf16_and_fp32_forms_agree_to_bf16_precision():
    w = _bf16_case(2000, 64, 256, seed=4)
    outs = []
    for bf in (False, True):
        s = hmc.sampler_for(w, grad_bf16=bf)
        outs.append(s.step(want_proposal=True))
        s.close()
    a, b = to_np(outs[0]["proposed_state"]), to_np(outs[1]["proposed_state"])
    e = rel_err_rows(b, a)
    print(f"bf16 vs fp32 gradient trajectories: rel diff p50={np.median(e):.2e} max={e.max():.2e}")
    assert np.quantile(e, 0.99) < 2e-2


def test_bf16_full_size_logreg_100000x512_sampled_chains():
    # the largest logistic shape of the served stream, every chain on the GPU, the oracle on
    # chains spread over the 128-chain tiles
    w = W.logreg(100000, 512, 1024, L=10, step_size=0.003, bf16=True, init=0.05, seed=7)
    s = hmc.sampler_for(w, grad_bf16=True)
    out = s.step(want_proposal=True)
    g = {k: to_np(v) for k, v in out.items()}
    xg, _, _ = s.get_state()
    s.close()
    chains = [0, 1, 127, 128, 513, 1023]
    o = oracle.step_chains(oracle_target(w), w.num_leapfrog_steps, w.seed, 0, w.step_size,
                           w.x0[chains].astype(np.float64), chains)
    ex = rel_err_rows(g["proposed_state"][chains], o["x_prop"])
    lp_o, _ = oracle.logp_grad(oracle_target(w), to_np(xg)[chains].astype(np.float64))
    lp_err = np.abs(g["target_log_prob"][chains] - lp_o) / np.abs(lp_o)
    print(f"logreg_100000x512 bf16, chains {chains}: proposal rel err p50={np.median(ex):.2e} max={ex.max():.2e}; "
          f"logp rel err max {lp_err.max():.2e}")
    assert np.max(ex) < 2e-2 and lp_err.max() < 2e-6


def test_bf16_full_size_logreg_100000x256_first_chains():
    # the large configuration at full size (8192 chains) in its launch configuration;
    # the oracle runs the first 16 chains (same chain ids, same Philox streams)
    w = W.cfg_logreg_100000x256()
    s = hmc.sampler_for(w, grad_bf16=True)
    out = s.step(want_proposal=True)
    g = {k: to_np(v) for k, v in out.items()}
    xg, _, _ = s.get_state()
    s.close()
    k = 16
    o = oracle.step(oracle_target(w), w.num_leapfrog_steps, w.seed, 0, w.step_size, w.x0[:k].astype(np.float64))
    ex = rel_err_rows(g["proposed_state"][:k], o["x_prop"])
    lp_o, _ = oracle.logp_grad(oracle_target(w), to_np(xg)[:k].astype(np.float64))
    lp_err = np.abs(g["target_log_prob"][:k] - lp_o) / np.abs(lp_o)
    print(f"logreg_100000x256 bf16, first {k} chains: proposal rel err p50={np.median(ex):.2e} max={ex.max():.2e}; "
          f"logp rel err max {lp_err.max():.2e}; accepted {g['is_accepted'][:k].mean():.2f} vs oracle "
          f"{o['accepted'].mean():.2f}")
    assert np.max(ex) < 2e-2 and lp_err.max() < 2e-6
