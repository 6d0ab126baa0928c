"""The allocation-free entry point hmc_sample_chain_noalloc, called through the
C ABI, against hmc_init + hmc_sample_chain + hmc_get_state on the same inputs:
samples, traces, final states and step sizes bit for bit (same kernels, same
order of arithmetic).  Each case makes two calls in a row, the second on a
smaller input, so the second runs in a scratch that still holds the first
call's contents."""
import ctypes

import numpy as np
import pytest

import workloads as W
from gpu_helpers import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_2002_01184_amd import hmc  # noqa: E402

KEYS = ("samples", "step_size", "is_accepted", "log_accept_ratio", "target_log_prob")


def _reference(w, form, adapt):
    s = hmc.sampler_for(w, form=form)
    out = s.sample_chain(w.num_results, w.num_burnin, adapt=adapt)
    x, e, t = s.get_state()
    torch.cuda.synchronize()
    res = {k: out[k].clone() for k in KEYS}
    res["final_x"], res["final_eps"] = x.clone(), e.clone()
    eff = s.form
    s.close()
    return res, eff


def _noalloc(w, form, adapt):
    # the same target and config structs the Sampler builds (its workspace is not used)
    s = hmc.sampler_for(w, form=hmc.HMC_FORM_PLAIN)
    s.close()
    dev = s.device
    C, D, R = s.C, s.D, w.num_results
    cfg = hmc.hmc_config(s.config.num_chains, s.config.num_leapfrog_steps, s.config.state_dtype,
                         s.config.grad_dtype, form, s.config.seed)
    init = s.keep[-1]
    out = dict(samples=torch.full((R, C, D), float("nan"), dtype=s.dtype, device=dev),
               step_size=torch.zeros(R, C, dtype=torch.float64, device=dev),
               is_accepted=torch.full((R, C), 7, dtype=torch.uint8, device=dev),
               log_accept_ratio=torch.zeros(R, C, dtype=torch.float64, device=dev),
               target_log_prob=torch.zeros(R, C, dtype=torch.float64, device=dev),
               final_x=torch.full((C, D), float("nan"), dtype=s.dtype, device=dev),
               final_eps=torch.zeros(C, dtype=torch.float64, device=dev))
    tr = hmc.hmc_trace(*[hmc._ptr(out[k]) for k in KEYS[1:]])
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    print(f"noalloc call: {w.name} C={C} D={D} R={R} burn-in={w.num_burnin} form={form}", flush=True)
    hmc.hmc_sample_chain_noalloc(s.target, cfg, hmc._ptr(init), [w.step_size], R, w.num_burnin,
                                 hmc.make_adapt(adapt), hmc._ptr(out["samples"]), tr, hmc._ptr(out["final_x"]),
                                 hmc._ptr(out["final_eps"]), stream)
    return out


PAIRS = {
    "logreg_fused": (lambda: W.logreg(1000, 25, 1024, L=10, step_size=0.05, burnin=40, results=30),
                     lambda: W.logreg(500, 25, 300, L=10, step_size=0.05, burnin=20, results=25, seed=3),
                     hmc.HMC_FORM_AUTO, True, "fused"),
    "dense_plain": (lambda: W.gauss_dense(100, 4096, L=20, step_size=0.1, burnin=10, results=10),
                    lambda: W.gauss_dense(37, 45, L=7, step_size=0.1, burnin=12, results=9, seed=3),
                    hmc.HMC_FORM_PLAIN, True, "plain"),
    "paper_fp64": (lambda: W.std_normal_1d(),
                   lambda: W.std_normal_1d(num_chains=10, burnin=30, results=20, seed=5),
                   hmc.HMC_FORM_AUTO, False, "fused"),
    "logreg_plain_1000x60": (lambda: W.logreg(1000, 60, 512, L=6, step_size=0.02, burnin=15, results=10),
                             lambda: W.logreg(700, 40, 64, L=6, step_size=0.02, burnin=5, results=7, seed=2),
                             hmc.HMC_FORM_PLAIN, True, "plain"),
}


@pytest.mark.parametrize("name", list(PAIRS))
def test_noalloc_equals_workspace_entry_point_twice(name):
    big, small, form, adapt, eff = PAIRS[name]
    for w in (big(), small()):          # second call: smaller input in the same scratch
        ref, ref_form = _reference(w, form, adapt)
        assert ref_form == eff
        got = _noalloc(w, form, adapt)
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(got[k], ref[k]), (name, w.name, k)


def test_noalloc_rejects_what_does_not_fit():
    w = W.cfg_logreg_100000x256()
    w.num_chains = 8192
    s_target = hmc.hmc_target(w.kind, 0, w.dim, None, ctypes.c_void_p(1 << 20), hmc.HMC_BF16, 0, w.X.shape[0],
                              ctypes.c_void_p(1 << 20), 1.0)
    cfg = hmc.hmc_config(8192, 10, hmc.HMC_F32, hmc.HMC_BF16, hmc.HMC_FORM_AUTO, 0)
    with pytest.raises(hmc.HMCError) as e:
        hmc.hmc_sample_chain_noalloc(s_target, cfg, ctypes.c_void_p(1 << 20), [0.005], 10, 10, None, None, None,
                                     None, None, None)
    assert e.value.status == hmc.HMC_E_NOMEM and "exceeds" in str(e.value)
    cfg = hmc.hmc_config(64, 10, hmc.HMC_F32, hmc.HMC_F32, hmc.HMC_FORM_GRAPH, 0)
    small = hmc.hmc_target(hmc.HMC_TGT_STD_NORMAL, 0, 3, None, None, hmc.HMC_F32, 0, 0, None, 1.0)
    with pytest.raises(hmc.HMCError) as e:
        hmc.hmc_sample_chain_noalloc(small, cfg, ctypes.c_void_p(1 << 20), [0.1], 10, 10, None, None, None,
                                     None, None, None)
    assert e.value.status == hmc.HMC_E_UNSUPPORTED
