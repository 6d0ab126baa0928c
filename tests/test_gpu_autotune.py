"""Autotuner: trials restore the chain state exactly, and the chosen launch
configuration samples the same chain as any other (within FP32 rounding of
the arithmetic order; bitwise for the same choice)."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import decision_report, gpu_available, one_step, rel_err_rows

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_2002_01184_amd import hmc  # noqa: E402

CASES = {
    "logreg_1000x25": (W.logreg(1000, 25, 512, L=5, step_size=0.05, seed=21), False),
    "logreg_3000x40": (W.logreg(3000, 40, 200, L=4, step_size=0.01, seed=22, init=0.3), False),
    "logreg_2000x64_bf16": (W.logreg(2000, 64, 256, L=4, step_size=0.004, bf16=True, init=0.05, seed=23), True),
    "gauss_diag_300": (W.gauss_diag(dim=300, num_chains=256, L=6, step_size=0.05, seed=24), False),
    "gauss_dense_60": (W.gauss_dense(dim=60, num_chains=96, L=6, step_size=0.1, seed=25), False),
}


@pytest.mark.parametrize("name", list(CASES))
def test_autotune_restores_state(name):
    w, bf = CASES[name]
    a = hmc.sampler_for(w, grad_bf16=bf)
    rep = a.autotune(2)
    print(f"{name}: {rep.strip().splitlines()[-1]} ({len(rep.splitlines()) - 1} candidates)")
    _, _, t = a.get_state()
    assert t == 0
    out_a = a.sample_chain(6, 4, adapt=True)
    form_a = a.form
    a.close()
    b = hmc.sampler_for(w, grad_bf16=bf)
    rep_b = b.autotune(2)                  # cached: applies the same choice without trials
    assert rep_b.startswith("cached")
    assert b.form == form_a
    out_b = b.sample_chain(6, 4, adapt=True)
    b.close()
    for k in ["samples", "is_accepted", "step_size"]:
        assert torch.equal(out_a[k], out_b[k]), k


def test_autotuned_sampler_matches_oracle():
    w, _ = CASES["logreg_3000x40"]
    s = hmc.sampler_for(w)
    s.autotune(2)
    g, o = one_step(w, s, np.ascontiguousarray(w.x0), 5)
    e = rel_err_rows(g["proposed_state"], o["x_prop"])
    agree, _, _ = decision_report(g, o, w.seed, 5)
    assert e.max() <= 1e-5 and agree >= 0.999
    s.close()
