"""The library's kernel timer (measurement support for the benchmark): events
around every launch of a context's dominant kernel, on its own stream."""
import pytest

import workloads as W
from gpu_helpers import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2002_01184_amd import hmc  # noqa: E402


@pytest.mark.parametrize("case,form,grad_bf16,name", [
    ("logreg_bf16", hmc.HMC_FORM_PLAIN, True, "k_lr16_grad"),
    ("logreg_f32", hmc.HMC_FORM_PLAIN, False, "k_lr32_step"),
    ("dense", hmc.HMC_FORM_PLAIN, False, "k_dense_step"),
    ("diag", hmc.HMC_FORM_PLAIN, False, "k_elem_first/mid/last"),
    ("dense", hmc.HMC_FORM_FUSED, False, "fused transition kernel"),
])
def test_kernel_timer_counts_the_dominant_launches(case, form, grad_bf16, name):
    w = {"logreg_bf16": W.logreg(2048, 64, 256, L=4, step_size=0.01, bf16=True, init=0.1),
         "logreg_f32": W.logreg(1000, 25, 256, L=4, step_size=0.05),
         "dense": W.gauss_dense(37, 64, L=5, step_size=0.1),
         "diag": W.gauss_diag(dim=50, num_chains=128, L=6, step_size=0.05)}[case]
    s = hmc.sampler_for(w, form=form, grad_bf16=grad_bf16)
    R, B = 3, 2
    hmc.hmc_kernel_timer_start(s.ctx, 1000)
    s.sample_chain(R, B, adapt=True)
    ms, n, got = hmc.hmc_kernel_timer_read(s.ctx)
    expect = 1 if form == hmc.HMC_FORM_FUSED else (R + B) * w.num_leapfrog_steps
    assert got == name and n == expect and ms > 0
    # a cap below the launch count records the first launches only; reading stops the timer
    hmc.hmc_kernel_timer_start(s.ctx, 2)
    s.sample_chain(R, B)
    assert hmc.hmc_kernel_timer_read(s.ctx)[1] == min(2, expect)
    with pytest.raises(hmc.HMCError):
        hmc.hmc_kernel_timer_read(s.ctx)
    s.close()


@pytest.mark.parametrize("form", [hmc.HMC_FORM_FUSED, hmc.HMC_FORM_PLAIN])
def test_kernel_timer_skips_the_bootstrap(form):
    # resetting the chains (set_state recomputes logp and gradient) inside the timed
    # region must not add launches: the bench resets before every timed step
    import numpy as np
    import torch
    w = W.logreg(1000, 25, 256, L=3, step_size=0.05)
    s = hmc.sampler_for(w, form=form)
    x0 = torch.from_numpy(np.ascontiguousarray(w.x0)).to(s.device)
    hmc.hmc_kernel_timer_start(s.ctx, 100)
    for _ in range(2):
        s.set_state(x0, None, 0)
        s.sample_chain(2, 1)
    ms, n, name = hmc.hmc_kernel_timer_read(s.ctx)
    if form == hmc.HMC_FORM_FUSED:
        assert (n, name) == (2, "fused transition kernel")
    else:
        assert (n, name) == (2 * 3 * 3, "k_lr32_step")
    s.close()
