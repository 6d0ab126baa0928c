"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: FP64 state (the paper's 1-D example) agrees with the oracle to 1e-12
relative with identical decisions; FP32 state: per-step proposal relative error
<= 1e-5 per chain (one-step mode: both sides start transition t from the same
state) and >= 99.9% of accept decisions agreeing, every disagreement lying
where |log u + dH| is within the dH difference.
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

FORMS = {"plain": hmc.HMC_FORM_PLAIN, "graph": hmc.HMC_FORM_GRAPH, "auto": hmc.HMC_FORM_AUTO}


def _cases():
    return {
        "std_normal_7d": W.std_normal_1d(num_chains=300, dim=7, state_dtype="f32", L=5, step_size=0.4),
        "gauss_diag_1001": W.gauss_diag(dim=1001, num_chains=70, L=10, step_size=0.05),
        "gauss_dense_100": W.gauss_dense(dim=100, num_chains=300, L=20, step_size=0.1),
        "gauss_dense_37": W.gauss_dense(dim=37, num_chains=45, L=7, step_size=0.1, seed=3),
        "logreg_1000x25": W.logreg(1000, 25, 1000, L=10, step_size=0.05),
        "logreg_3000x40_bf16x": W.logreg(3000, 40, 100, L=6, step_size=0.01, bf16=True, init=0.3, seed=2),
        "logreg_77x3": W.logreg(77, 3, 33, L=4, step_size=0.2, seed=5),
    }


CASES = _cases()


def test_paper_example_fp64_full_run_matches_oracle():
    w = W.cfg_std_normal_1d()
    for form in ["plain", "auto"]:
        s = hmc.sampler_for(w, form=FORMS[form])
        out = s.sample_chain(w.num_results, w.num_burnin, adapt=False)
        o = oracle.sample_chain(oracle_target(w), w.num_leapfrog_steps, w.seed, w.x0.astype(np.float64), w.step_size,
                                w.num_burnin, w.num_results)
        smp = to_np(out["samples"])
        assert smp.dtype == np.float64
        assert np.max(np.abs(smp - o["samples"])) <= 1e-12 * max(1.0, np.max(np.abs(o["samples"])))
        assert np.array_equal(to_np(out["is_accepted"]).astype(bool), o["is_accepted"])
        assert np.allclose(to_np(out["log_accept_ratio"]), o["log_accept_ratio"], rtol=1e-10, atol=1e-12)
        assert np.allclose(to_np(out["target_log_prob"]), o["target_log_prob"], rtol=1e-12, atol=1e-14)
        assert np.all(to_np(out["step_size"]) == 1.5)
        # the paper's example: stationary acceptance 0.760 (closed form by quadrature)
        assert abs(to_np(out["is_accepted"]).mean() - 0.760) < 0.03
        s.close()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("form", ["plain", "auto"])
def test_one_step_parity(name, form):
    w = CASES[name]
    s = hmc.sampler_for(w, form=FORMS[form])
    # states: the initial state, then states the oracle reached
    tg = oracle_target(w)
    x = w.x0.astype(np.float64)
    st = oracle.sample_chain(tg, w.num_leapfrog_steps, w.seed, x, w.step_size, 0, 3)["samples"]
    states = [w.x0, st[0].astype(np.float32), st[2].astype(np.float32)]
    ts = [0, 1, 1000]
    errs, agree_all, worst_margin = [], [], []
    for xs, t in zip(states, ts):
        g, o = one_step(w, s, np.ascontiguousarray(xs), t)
        ex = rel_err_rows(g["proposed_state"], o["x_prop"])
        ep = rel_err_rows(g["proposed_momentum"], o["p_prop"])
        errs.append(np.maximum(ex, ep))
        agree, margins, dh_err = decision_report(g, o, w.seed, t)
        agree_all.append(agree)
        if len(margins):
            assert np.all(margins <= 10 * np.max(dh_err) + 1e-12), (margins, np.max(dh_err))
        # post-decision state: the proposal where accepted, the start where rejected
        xg, _, _ = s.get_state()
        xg = to_np(xg)
        acc = g["is_accepted"].astype(bool)
        assert np.array_equal(xg[~acc], xs[~acc])
        assert np.array_equal(xg[acc], g["proposed_state"][acc])
    e = np.concatenate(errs)
    print(f"{name}/{form}: proposal rel err p50={np.median(e):.2e} p99={np.quantile(e, 0.99):.2e} "
          f"max={e.max():.2e}; decisions agree {np.mean(agree_all):.5f}")
    assert e.max() <= 1e-5
    assert np.mean(agree_all) >= 0.999
    s.close()


def test_forms_plain_and_graph_are_bitwise_equal():
    w = W.logreg(500, 9, 200, L=5, step_size=0.05, seed=4)
    outs = []
    for form in ["plain", "graph"]:
        s = hmc.sampler_for(w, form=FORMS[form])
        assert s.form == form
        outs.append(s.sample_chain(20, 10, adapt=True))
        s.close()
    for k in ["samples", "is_accepted", "log_accept_ratio", "step_size", "target_log_prob"]:
        assert torch.equal(outs[0][k], outs[1][k]), k


@pytest.mark.parametrize("form", ["plain", "auto"])
def test_resume_is_bitwise(form):
    w = W.gauss_dense(dim=30, num_chains=64, L=8, step_size=0.15, seed=1)
    s = hmc.sampler_for(w, form=FORMS[form])
    full = s.sample_chain(12, 0)["samples"]
    s.close()
    s1 = hmc.sampler_for(w, form=FORMS[form])
    a = s1.sample_chain(5, 0)["samples"]
    x, e, t = s1.get_state()
    assert t == 5
    s1.close()
    s2 = hmc.sampler_for(w, form=FORMS[form])
    s2.set_state(x, e, t)
    b = s2.sample_chain(7, 0)["samples"]
    assert torch.equal(torch.cat([a, b]), full)
    s2.close()


@pytest.mark.parametrize("form", ["plain", "auto"])
def test_adapted_run_in_chunks_is_bitwise(form):
    # burn-in with dual averaging and 3 kept draws, then two calls without burn-in:
    # the step sizes stay frozen at exp(log eps_bar) and the counter carries on,
    # so the chunks equal one uninterrupted call (also written into slices of one array)
    w = W.logreg(200, 9, 96, L=5, step_size=0.05, seed=4)
    s = hmc.sampler_for(w, form=FORMS[form])
    full = s.sample_chain(10, 6, adapt=True)
    s.close()
    s1 = hmc.sampler_for(w, form=FORMS[form])
    keep = torch.empty(10, w.num_chains, w.dim, dtype=torch.float32, device="cuda")
    parts = [s1.sample_chain(3, 6, adapt=True, out_samples=keep[0:3]),
             s1.sample_chain(4, 0, out_samples=keep[3:7]),
             s1.sample_chain(3, 0, out_samples=keep[7:10])]
    s1.close()
    assert torch.equal(keep, full["samples"])
    for k in ["is_accepted", "log_accept_ratio", "step_size", "target_log_prob"]:
        assert torch.equal(torch.cat([p[k] for p in parts]), full[k]), k


@pytest.mark.parametrize("form", ["plain", "auto"])
def test_batch_semantics_and_determinism(form):
    w = W.logreg(300, 6, 96, L=5, step_size=0.1, seed=7)
    s = hmc.sampler_for(w, form=FORMS[form])
    a = s.sample_chain(10, 5, adapt=True)
    s.close()
    s = hmc.sampler_for(w, form=FORMS[form])
    b = s.sample_chain(10, 5, adapt=True)
    s.close()
    for k in ["samples", "is_accepted", "step_size"]:
        assert torch.equal(a[k], b[k]), k          # repeated runs are bitwise equal
    x0 = w.x0.copy()
    x0[17] += 0.5
    s = hmc.sampler_for(w, form=FORMS[form], x0=x0)
    c = s.sample_chain(10, 5, adapt=True)
    s.close()
    keep = torch.ones(96, dtype=torch.bool)
    keep[17] = False
    assert torch.equal(a["samples"][:, keep], c["samples"][:, keep])
    assert not torch.equal(a["samples"][:, 17], c["samples"][:, 17])


def test_nonfinite_chains_are_rejected_not_fatal():
    w = W.std_normal_1d(num_chains=8, dim=3, state_dtype="f32", L=3, step_size=0.5)
    x0 = w.x0.copy()
    x0[2, 1] = np.nan
    x0[5, 0] = np.inf
    s = hmc.sampler_for(w, x0=x0)
    out = s.sample_chain(4, 0)
    acc = to_np(out["is_accepted"]).astype(bool)
    lar = to_np(out["log_accept_ratio"])
    assert not acc[:, 2].any() and np.all(lar[:, 2] == -np.inf)
    assert not acc[:, 5].any()
    assert acc[:, [0, 1, 3, 4, 6, 7]].any()
    s.close()


# Dual averaging amplifies rounding differences in its early iterations (the
# step size responds to the accept statistic with gain ~ sqrt(m)/(gamma (m+t0))),
# so trajectories under adaptation are not comparable bit for bit even in FP64.
# The recursion itself is pinned where its input is exact on both sides.
@pytest.mark.parametrize("form", ["plain", "auto"])
def test_dual_averaging_recursion_exact(form):
    # NaN states reject every proposal with accept statistic exactly 0: the step
    # size after B burn-in transitions is exp(log eps_bar_B) of the oracle's recursion.
    w = W.std_normal_1d(num_chains=6, dim=2, state_dtype="f64", L=3, step_size=0.3)
    x0 = w.x0.copy()
    x0[:, 0] = np.nan
    eps0 = np.array([0.3, 0.01, 1.0, 0.05, 2.0, 0.7])
    s = hmc.sampler_for(w, form=FORMS[form], x0=x0, step_size=eps0)
    B = 57
    out = s.sample_chain(2, B, adapt=True)
    st = to_np(out["step_size"])
    for c in range(6):
        _, _, leb, _ = oracle.dual_avg_run(eps0[c], [0.0] * B)
        assert st[0, c] == pytest.approx(np.exp(leb[-1]), rel=1e-13)
        assert st[1, c] == st[0, c]
    assert not to_np(out["is_accepted"]).any()
    s.close()


@pytest.mark.parametrize("name", ["logreg_1000x25", "gauss_dense_100", "std_normal_7d"])
@pytest.mark.parametrize("form", ["plain", "auto"])
def test_dual_averaging_first_iteration(name, form):
    # one adapted burn-in transition from a given state: the new step size is
    # 10 eps0 exp(-(delta - alpha) / (gamma (1 + t0))) with the oracle's alpha
    import torch as _t
    w = CASES[name]
    s = hmc.sampler_for(w, form=FORMS[form])
    x = np.ascontiguousarray(w.x0)
    t = 7
    s.set_state(_t.from_numpy(x).to(s.device), None, t)
    out = s.sample_chain(1, 1, adapt=True)
    got = to_np(out["step_size"])[0]
    o = oracle.step(oracle_target(w), w.num_leapfrog_steps, w.seed, t, w.step_size, x.astype(np.float64))
    alpha = np.exp(np.minimum(0.0, o["log_accept_ratio"]))
    want = 10 * w.step_size * np.exp(-(0.8 - alpha) / (0.05 * 11.0))
    rel = np.abs(got - want) / want
    print(f"{name}/{form}: first dual-averaging step rel err max {rel.max():.2e}")
    assert np.quantile(rel, 0.999) < 1e-4
    s.close()


def test_dual_averaging_fp32_reaches_target_like_oracle():
    # FP32 trajectories feed slightly different accept statistics into the
    # (sensitive) early dual-averaging iterations, so per-chain step sizes are
    # compared in distribution: both adapt to the same scale and acceptance.
    w = W.logreg(400, 8, 256, L=6, step_size=0.05, seed=9)
    s = hmc.sampler_for(w)
    out = s.sample_chain(100, 200, adapt=True)
    o = oracle.sample_chain(oracle_target(w), w.num_leapfrog_steps, w.seed, w.x0.astype(np.float64), w.step_size,
                            200, 100, adapt=True)
    st_g, st_o = to_np(out["step_size"])[-1], o["step_size"][-1]
    ratio = np.median(st_g) / np.median(st_o)
    acc_g = np.exp(np.minimum(0, to_np(out["log_accept_ratio"]))).mean()
    acc_o = np.exp(np.minimum(0, o["log_accept_ratio"])).mean()
    print(f"median step ratio {ratio:.4f}; accept gpu {acc_g:.3f} oracle {acc_o:.3f}")
    assert abs(ratio - 1) < 0.05
    assert abs(acc_g - 0.8) < 0.05 and abs(acc_o - 0.8) < 0.05
    assert np.all(to_np(out["step_size"]) == to_np(out["step_size"])[0:1])
    s.close()


FUSED_EXPECTED = {"std_normal_7d": "fused", "gauss_diag_1001": "fused", "gauss_dense_100": "fused",
                  "gauss_dense_37": "fused", "logreg_1000x25": "fused", "logreg_77x3": "fused",
                  "logreg_3000x40_bf16x": "plain"}


@pytest.mark.parametrize("name", list(CASES))
def test_auto_form_selection(name):
    s = hmc.sampler_for(CASES[name])
    assert s.form == FUSED_EXPECTED[name]
    s.close()


def _trajectory_compare(w, chains, form):
    """Full sample_chain on the GPU (all chains, as bench.py launches it) against the
    oracle's run of a sample of chains (same chain ids, so the same Philox streams)."""
    s = hmc.sampler_for(w, form=form)
    out = s.sample_chain(w.num_results, w.num_burnin, adapt=w.adapt)
    g_acc = to_np(out["is_accepted"][:, chains]).astype(bool)
    g_smp = to_np(out["samples"][:, chains])
    g_eps = to_np(out["step_size"][:, chains])
    s.close()
    o = oracle.sample_chain(oracle_target(w), w.num_leapfrog_steps, w.seed, w.x0[:max(chains) + 1].astype(np.float64),
                            w.step_size, w.num_burnin, w.num_results, adapt=w.adapt)
    o_acc = o["is_accepted"][:, chains]
    o_smp = o["samples"][:, chains]
    agree = np.mean(g_acc == o_acc)
    err = np.linalg.norm(g_smp - o_smp, axis=-1) / np.maximum(np.linalg.norm(o_smp, axis=-1), 1e-30)
    return agree, err, g_eps, o["step_size"][:, chains]


def test_full_size_paper_example_fp64():
    w = W.cfg_std_normal_1d()
    agree, err, _, _ = _trajectory_compare(w, list(range(100)), hmc.HMC_FORM_AUTO)
    assert agree == 1.0 and err.max() < 1e-12


@pytest.mark.parametrize("form", ["plain", "auto"])
def test_wide_std_normal_fp64_sampled_chains(form):
    # the paper's target at 2^24 chains (the HBM-roofline shape), every chain on the
    # GPU; the first chains against the oracle
    w = W.cfg_std_normal_1d_wide()
    w.num_burnin, w.num_results = 4, 4
    agree, err, _, _ = _trajectory_compare(w, [0, 1, 2, 17, 63], FORMS[form])
    assert agree == 1.0 and err.max() < 1e-12


@pytest.mark.parametrize("form", ["plain", "auto"])
def test_wide_gauss_diag_1000_sampled_chains(form):
    # diagonal Gaussian D=1000 (variances 1e-2..1e2), 16384 chains, FP32 state
    w = W.cfg_gauss_diag_1000()
    w.num_burnin, w.num_results = 3, 3
    agree, err, _, _ = _trajectory_compare(w, [0, 1, 7, 31], FORMS[form])
    assert agree == 1.0 and err.max() < 1e-5


@pytest.mark.parametrize("form", ["plain", "auto"])
def test_full_size_gauss_dense_100_sampled_chains(form):
    # the dense Gaussian workload at full size (4096 chains, L=20) in bench's launch
    # configuration (fused for auto), fixed step size, sampled chains against the oracle
    w = W.cfg_gauss_dense_100()
    w.num_burnin, w.num_results, w.adapt = 3, 3, False
    agree, err, _, _ = _trajectory_compare(w, [0, 1, 100, 2047, 4095], FORMS[form])
    assert agree == 1.0 and err.max() < 1e-5, err.max()


def test_full_size_logreg_1000x25_fixed_step_sampled_chains():
    # the benchmark workload at full size (1024 chains) in bench's launch
    # configuration, fixed step size: trajectories on sampled chains match the oracle
    w = W.cfg_logreg_1000x25()
    w.adapt = False
    w.num_burnin, w.num_results = 100, 100
    chains = [0, 1, 2, 3, 511, 1020, 1021, 1023]
    agree, err, _, _ = _trajectory_compare(w, chains, hmc.HMC_FORM_AUTO)
    print(f"logreg_1000x25 full size fixed step: decisions agree {agree:.5f}; sample rel err "
          f"p50={np.median(err):.2e} p99={np.quantile(err, 0.99):.2e} max={err.max():.2e}")
    assert agree >= 0.999
    assert np.median(err) < 1e-5


def test_full_size_logreg_1000x25_one_step_all_chains():
    w = W.cfg_logreg_1000x25()
    s = hmc.sampler_for(w)
    assert s.form == "fused"
    st = oracle.sample_chain(oracle_target(w), w.num_leapfrog_steps, w.seed, w.x0.astype(np.float64), w.step_size,
                             0, 2, nthreads=0)["samples"][-1].astype(np.float32)
    g, o = one_step(w, s, np.ascontiguousarray(st), 1500)
    e = np.maximum(rel_err_rows(g["proposed_state"], o["x_prop"]), rel_err_rows(g["proposed_momentum"], o["p_prop"]))
    agree, margins, dh_err = decision_report(g, o, w.seed, 1500)
    print(f"logreg_1000x25 one step, 1024 chains: rel err p50={np.median(e):.2e} max={e.max():.2e}; agree {agree:.5f}")
    assert e.max() <= 1e-5 and agree >= 0.999
    s.close()


def test_full_size_logreg_1000x25_adapted_run_statistics():
    # adapted full run (1000 + 1000): acceptance near the 0.8 target and step sizes
    # of the same scale as the oracle's on sampled chains
    w = W.cfg_logreg_1000x25()
    chains = [0, 5, 100, 1023]
    agree, err, ge, oe = _trajectory_compare(w, chains, hmc.HMC_FORM_AUTO)
    ratio = np.median(ge[-1]) / np.median(oe[-1])
    print(f"logreg_1000x25 adapted: step ratio {ratio:.4f}")
    assert abs(ratio - 1) < 0.1
    assert np.all(ge == ge[0:1])
