"""GPU parity of the FP32-gradient logistic-regression path (split-N MFMA
contractions, paper Sec. 2.1 with the batch semantics of Sec. 2) at the widths
every instantiation covers, against the FP64 oracle.

  * D = 9, 100, 200, 250, 257, 384 and 512 (1 to 32 tiles of 16 dims: every
    instantiation of the step kernel, 16-byte and element-wise stage loads of
    FP32 and BF16 X, the largest beyond 64 KB of LDS; chain counts that leave
    the last 64-chain tile ragged, row counts not a multiple of 16), every
    chain against the oracle;
  * the 100000 x 256 workload (BF16-stored X, 8192 chains, L = 10) in its
    FP32-gradient form, every chain on the GPU, the oracle on sampled chains
    spread over the chain tiles;
  * the largest logistic shape of the served stream, 100000 x 512, likewise.

Bar (one-step mode, both sides start transition t from the same state): per
chain ||x_L - x_L^ref|| / ||x_L^ref|| and the same for p_L at most 1e-5;
decisions agree, any disagreement lying where |log u + dH| is within the dH
difference.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import decision_report, gpu_available, oracle_target, rel_err_rows, to_np

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_2002_01184_amd import hmc  # noqa: E402


def _gpu_step(w, s, x_state, t):
    xs = torch.from_numpy(np.ascontiguousarray(x_state)).to(s.device)
    s.set_state(xs, None, t)
    g = s.step(want_proposal=True)
    return {k: to_np(v) for k, v in g.items()}


def _check(name, g, o, chains, seed, t):
    ex = rel_err_rows(g["proposed_state"][chains], o["x_prop"])
    ep = rel_err_rows(g["proposed_momentum"][chains], o["p_prop"])
    e = np.maximum(ex, ep)
    ga = g["is_accepted"][chains].astype(bool)
    agree = float(np.mean(ga == o["accepted"]))
    u = oracle.accept_uniform(seed, max(chains) + 1, t)[chains]
    margin = np.abs(np.log(u) + o["delta_h"])
    dh_err = np.abs(g["delta_h"][chains] - o["delta_h"])
    bad = ga != o["accepted"]
    print(f"{name}: {len(chains)} chains, proposal rel err p50={np.median(e):.2e} p99={np.quantile(e, 0.99):.2e} "
          f"max={e.max():.2e}; dH abs err max {dh_err.max():.2e}; decisions agree {agree:.4f}")
    assert e.max() <= 1e-5, e.max()
    assert np.all(margin[bad] <= dh_err[bad]), (margin[bad], dh_err[bad])
    return agree


@pytest.mark.parametrize("N,D,C,bf16x", [(2000, 100, 200, False), (2500, 200, 150, True), (2000, 257, 200, False),
                                         (3000, 384, 130, True), (4000, 512, 300, False), (1200, 100, 70, True),
                                         (900, 250, 66, False), (37, 9, 5, False)])
def test_fp32_logreg_wide_dims_every_chain(N, D, C, bf16x):
    w = W.logreg(N, D, C, L=6, step_size=0.01, bf16=bf16x, init=0.1, seed=D)
    s = hmc.sampler_for(w, form=hmc.HMC_FORM_PLAIN)
    t = 5
    g = _gpu_step(w, s, w.x0, t)
    s.close()
    o = oracle.step(oracle_target(w), w.num_leapfrog_steps, w.seed, t, w.step_size, w.x0.astype(np.float64))
    agree = _check(f"logreg {N}x{D} {'bf16' if bf16x else 'f32'} X", g, o, list(range(C)), w.seed, t)
    assert agree >= 0.999


def test_fp32_logreg_wide_dims_graph_form():
    w = W.logreg(1500, 300, 64, L=5, step_size=0.01, init=0.1, seed=33)
    s = hmc.sampler_for(w, form=hmc.HMC_FORM_GRAPH)
    g = _gpu_step(w, s, w.x0, 2)
    s.close()
    o = oracle.step(oracle_target(w), w.num_leapfrog_steps, w.seed, 2, w.step_size, w.x0.astype(np.float64))
    _check("logreg 1500x300 graph", g, o, list(range(64)), w.seed, 2)


def _sampled(C):
    # chains at wave and tile edges (16 chains per wave, 64 per tile), in the middle and at the end
    return sorted({0, 1, 15, 16, 17, 63, 64, 255, 256, C // 2 - 1, C // 2, C // 2 + 7, C - 17, C - 16, C - 2, C - 1})


def test_fp32_path_logreg_100000x256_sampled_chains():
    w = W.cfg_logreg_100000x256()
    s = hmc.sampler_for(w, grad_bf16=False)
    assert s.form == "plain"
    t = 3
    g = _gpu_step(w, s, w.x0, t)
    s.close()
    chains = _sampled(w.num_chains)
    o = oracle.step_chains(oracle_target(w), w.num_leapfrog_steps, w.seed, t, w.step_size,
                           w.x0[chains].astype(np.float64), chains)
    _check("logreg 100000x256 FP32 path, 8192 chains", g, o, chains, w.seed, t)


def test_fp32_path_logreg_100000x512_sampled_chains():
    w = W.logreg(100000, 512, 1024, L=10, step_size=0.003, bf16=True, init=0.05, seed=7)
    s = hmc.sampler_for(w, grad_bf16=False)
    t = 1
    g = _gpu_step(w, s, w.x0, t)
    s.close()
    chains = _sampled(w.num_chains)
    o = oracle.step_chains(oracle_target(w), w.num_leapfrog_steps, w.seed, t, w.step_size,
                           w.x0[chains].astype(np.float64), chains)
    _check("logreg 100000x512 FP32 path, 1024 chains", g, o, chains, w.seed, t)
