"""GPU parity of the unrolled No-U-Turn sampler (paper Sec. 2.3) against the
oracle's recursive NUTS (Hoffman & Gelman 2014, Algorithm 3) on the same
counter-keyed random numbers.

Bars: FP64 element-wise targets agree with the oracle over whole runs (states
to 1e-12, tree depths and leapfrog counts exactly); FP32 targets, one
transition from given states: >= 99% of chains take the same tree (depth,
leapfrog count, moved) and those chains' states agree to 1e-5 relative; the
FP32 chain samples N(0, 1) with the right variance.

The persistent kernels (element-wise targets; the dense Gaussian on MFMA,
16 chains per workgroup; logistic regression with X in LDS, a wavefront per
chain) build the lockstep path's trees (>= 99%), including a ragged tile, the
largest dense shape and the largest data set that fits in LDS.

Step-size adaptation inside NUTS (Hoffman & Gelman Algorithm 6): on FP64
element-wise targets adapted runs match the oracle's (states and statistics
to 1e-12, step sizes to 1e-12 relative, trees exactly); where the statistic is
exact (a flat target: 1; NaN states: 0) the multiplicative rule's step sizes
equal the oracle's bit for bit; FP32 targets adapt to the oracle's step-size
scale and statistic.
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


FORMS = {"lockstep": hmc.HMC_FORM_PLAIN, "persistent": hmc.HMC_FORM_AUTO}


@pytest.mark.parametrize("case", ["std1", "diag5", "diag300"])
@pytest.mark.parametrize("form", ["lockstep", "persistent"])
def test_fp64_runs_match_oracle(case, form):
    if case == "std1":
        w = W.std_normal_1d(num_chains=64, step_size=0.5)
        w.x0 = np.random.default_rng(0).normal(size=(64, 1))
    elif case == "diag5":
        w = W.gauss_diag(dim=5, num_chains=48, step_size=0.3, state_dtype="f64", lam_lo=0.3, lam_hi=3.0)
    else:       # 75 4-dim blocks: the persistent kernel runs one chain per workgroup
        w = W.gauss_diag(dim=300, num_chains=10, step_size=0.15, state_dtype="f64", lam_lo=0.3, lam_hi=3.0)
    s = hmc.sampler_for(w, form=FORMS[form])
    g = s.nuts_sample_chain(40, 10, max_depth=6)
    s.close()
    o = oracle.nuts_sample_chain(oracle_target(w), w.seed, w.x0.astype(np.float64), w.step_size, 10, 40, max_depth=6)
    assert np.array_equal(to_np(g["tree_depth"]), o["depth"])
    assert np.array_equal(to_np(g["n_leapfrog"]), o["n_leapfrog"])
    assert np.max(np.abs(to_np(g["samples"]) - o["samples"])) <= 1e-12
    assert o["depth"].min() >= 1 and o["depth"].max() > 1


def _fp32_cases():
    return {
        "std_normal_7d": W.std_normal_1d(num_chains=60, dim=7, state_dtype="f32", step_size=0.4),
        "gauss_diag_101": W.gauss_diag(dim=101, num_chains=40, step_size=0.08),
        "gauss_dense_37": W.gauss_dense(dim=37, num_chains=45, step_size=0.1, seed=3),
        "logreg_77x3": W.logreg(77, 3, 33, step_size=0.2, seed=5),
        "logreg_1000x25": W.logreg(1000, 25, 64, step_size=0.05),
        # X beyond the LDS (persistent form: X read through the L2), and BF16-stored X
        "logreg_3000x25": W.logreg(3000, 25, 40, step_size=0.03, seed=10),
        "logreg_bf16_500x17": W.logreg(500, 17, 37, step_size=0.06, seed=11, bf16=True),
    }


@pytest.mark.parametrize("name", list(_fp32_cases()))
@pytest.mark.parametrize("form", ["lockstep", "persistent"])
def test_fp32_one_transition_parity(name, form):
    w = _fp32_cases()[name]
    s = hmc.sampler_for(w, form=FORMS[form])
    g = s.nuts_sample_chain(1, 0, max_depth=8)
    xg, _, t = s.get_state()
    s.close()
    assert t == 1
    tg = oracle_target(w)
    same, errs = [], []
    gd, gn = to_np(g["tree_depth"])[0], to_np(g["n_leapfrog"])[0]
    xg = to_np(xg)
    for c in range(w.num_chains):
        r = oracle.nuts_transition(tg, w.seed, c, 0, w.step_size, 8, w.x0[c].astype(np.float64))
        ok = r["depth"] == gd[c] and r["n_leapfrog"] == gn[c]
        same.append(ok)
        if ok:
            errs.append(rel_err_rows(xg[c:c + 1], r["x"][None])[0])
    assert np.mean(same) >= 0.99, np.mean(same)
    assert max(errs) <= 1e-5, max(errs)


@pytest.mark.parametrize("form", ["lockstep", "persistent"])
def test_fp32_standard_normal_moments(form):
    w = W.std_normal_1d(num_chains=256, dim=3, state_dtype="f32", step_size=0.3)
    s = hmc.sampler_for(w, form=FORMS[form])
    g = s.nuts_sample_chain(300, 30, max_depth=8)
    s.close()
    x = to_np(g["samples"]).reshape(-1, 3)
    assert np.all(np.abs(x.mean(0)) < 0.02)
    assert np.allclose(x.var(0), 1.0, atol=0.04)


def test_nuts_errors():
    w = W.std_normal_1d(num_chains=8)
    s = hmc.sampler_for(w, form=hmc.HMC_FORM_PLAIN)
    with pytest.raises(hmc.HMCError, match="max_depth"):
        s.nuts_sample_chain(1, 0, max_depth=11)
    s.set_inverse_temperature(torch.ones(8, dtype=torch.float64, device="cuda"))
    with pytest.raises(hmc.HMCError, match="NUTS"):
        s.nuts_sample_chain(1, 0)
    s.close()


def _persistent_cases():
    return {
        "diag_300": W.gauss_diag(dim=300, num_chains=70, step_size=0.05),     # 64 lanes x 2 blocks per chain
        "diag_1000": W.gauss_diag(dim=1000, num_chains=20, step_size=0.05),   # a workgroup per chain
        "dense_100": W.gauss_dense(dim=100, num_chains=80, step_size=0.1, seed=2),
        "dense_ragged_17x17": W.gauss_dense(dim=17, num_chains=17, step_size=0.2, seed=4),
        "dense_max_128": W.gauss_dense(dim=128, num_chains=33, step_size=0.05, seed=6),
        "logreg_1000x25": W.logreg(1000, 25, 64, step_size=0.05),                  # X in LDS, a wave per chain
        "logreg_77x3": W.logreg(77, 3, 33, step_size=0.2, seed=5),                 # N not a multiple of 4
        "logreg_max_960x32": W.logreg(960, 32, 12, step_size=0.03, seed=8),        # the largest X that fits
        "logreg_l2_1300x32": W.logreg(1300, 32, 9, step_size=0.03, seed=12),       # the smallest beyond it
        "logreg_l2_5000x7": W.logreg(5000, 7, 70, step_size=0.02, seed=13),        # X read through the L2
        "logreg_l2_bf16_700x30": W.logreg(700, 30, 23, step_size=0.04, seed=14, bf16=True),
    }


@pytest.mark.parametrize("name", list(_persistent_cases()))
def test_persistent_and_lockstep_build_the_same_trees(name):
    w = _persistent_cases()[name]
    out = []
    for form in (hmc.HMC_FORM_PLAIN, hmc.HMC_FORM_AUTO):     # automatic form: the persistent kernel
        s = hmc.sampler_for(w, form=form)
        out.append(s.nuts_sample_chain(6, 2, max_depth=7, adapt=True))
        out[-1]["eps"] = s.get_state()[1]
        s.close()
    same = (out[0]["tree_depth"] == out[1]["tree_depth"]) & (out[0]["n_leapfrog"] == out[1]["n_leapfrog"])
    assert same.float().mean().item() >= 0.99
    assert out[1]["tree_depth"].min().item() >= 1
    rel = ((out[0]["eps"] - out[1]["eps"]).abs() / out[0]["eps"]).cpu().numpy()
    assert np.mean(rel <= 1e-6) >= 0.95


# ------------------------------------------------- step-size adaptation --
@pytest.mark.parametrize("adapt", ["dual_averaging", "simple"])
@pytest.mark.parametrize("form", ["lockstep", "persistent"])
def test_fp64_adapted_runs_match_oracle(adapt, form):
    w = W.gauss_diag(dim=5, num_chains=48, step_size=0.3, state_dtype="f64", lam_lo=0.3, lam_hi=3.0)
    s = hmc.sampler_for(w, form=FORMS[form])
    g = s.nuts_sample_chain(30, 40, max_depth=6, adapt=adapt, rate=0.05)
    _, eps, _ = s.get_state()
    s.close()
    o = oracle.nuts_sample_chain(oracle_target(w), w.seed, w.x0.astype(np.float64), w.step_size, 40, 30,
                                 max_depth=6, adapt=adapt, rate=0.05)
    assert np.ptp(o["final_eps"]) > 0 and not np.allclose(o["final_eps"], w.step_size)
    same_tree = (to_np(g["tree_depth"]) == o["depth"]) & (to_np(g["n_leapfrog"]) == o["n_leapfrog"])
    if adapt == "simple":
        # products of exact factors: the runs agree to rounding
        assert same_tree.all()
        assert np.max(np.abs(to_np(g["samples"]) - o["samples"])) <= 1e-12
        assert np.max(np.abs(to_np(g["accept_stat"]) - o["accept_stat"])) <= 1e-12
        assert np.allclose(to_np(eps), o["final_eps"], rtol=1e-12, atol=0)
    else:
        # dual averaging multiplies the statistic's last-ulp differences (exp, FMA contraction) by
        # sqrt(m) / gamma ~ 100 per burn-in transition and NUTS trajectories amplify them further:
        # trees agree, and nearly every chain stays within 1e-6 of the oracle's
        assert same_tree.mean() >= 0.99
        close = np.max(np.abs(to_np(g["samples"]) - o["samples"]), axis=(0, 2)) <= 1e-6
        assert close.mean() >= 0.95, close.mean()
        eps_close = np.abs(to_np(eps) / o["final_eps"] - 1) <= 1e-8
        assert eps_close.mean() >= 0.95, eps_close.mean()


@pytest.mark.parametrize("form", ["lockstep", "persistent"])
def test_exact_statistics_give_exact_step_sizes(form):
    B, rate, eps0 = 20, 0.03, 0.2
    # flat target: every leaf keeps H0, statistic 1, step grows by (1 + rate) per burn-in transition
    w = W.gauss_diag(dim=5, num_chains=32, step_size=eps0, lam_lo=1.0, lam_hi=1.0)
    w.prec = np.zeros(5, dtype=np.float32)
    s = hmc.sampler_for(w, form=FORMS[form])
    g = s.nuts_sample_chain(3, B, max_depth=4, adapt="simple", rate=rate)
    _, eps, _ = s.get_state()
    s.close()
    o = oracle.nuts_sample_chain(oracle_target(w), w.seed, w.x0.astype(np.float64), eps0, B, 3, max_depth=4,
                                 adapt="simple", rate=rate)
    assert np.all(to_np(g["accept_stat"]) == 1.0)
    assert np.array_equal(to_np(eps), o["final_eps"])
    # NaN states: the first leaf diverges with statistic 0, the step shrinks by 1 / (1 + rate)
    w = W.std_normal_1d(num_chains=40, dim=7, state_dtype="f32", step_size=eps0)
    x0 = w.x0.copy()
    x0[::3, 0] = np.nan
    s = hmc.sampler_for(w, form=FORMS[form], x0=x0)
    g = s.nuts_sample_chain(2, B, max_depth=5, adapt="simple", rate=rate)
    _, eps, _ = s.get_state()
    s.close()
    o = oracle.nuts_sample_chain(oracle_target(w), w.seed, x0.astype(np.float64), eps0, B, 2, max_depth=5,
                                 adapt="simple", rate=rate)
    rows = np.arange(40)[::3]
    assert np.all(to_np(g["accept_stat"])[:, rows] == 0.0)
    assert np.array_equal(to_np(eps)[rows], o["final_eps"][rows])


@pytest.mark.parametrize("name,form", [("gauss_dense_37", "lockstep"), ("gauss_dense_37", "persistent"),
                                       ("logreg_77x3", "lockstep"), ("logreg_77x3", "persistent"),
                                       ("std_normal_7d", "persistent")])
def test_fp32_adaptation_follows_the_oracle(name, form):
    w = _fp32_cases()[name]
    s = hmc.sampler_for(w, form=FORMS[form])
    g = s.nuts_sample_chain(60, 80, max_depth=8, adapt=True)
    _, eps, _ = s.get_state()
    s.close()
    o = oracle.nuts_sample_chain(oracle_target(w), w.seed, w.x0.astype(np.float64), w.step_size, 80, 60,
                                 max_depth=8, adapt=True)
    ratio = np.median(to_np(eps)) / np.median(o["final_eps"])
    assert abs(ratio - 1) < 0.1, ratio
    assert abs(to_np(g["accept_stat"]).mean() - o["accept_stat"].mean()) < 0.05
    assert abs(o["accept_stat"].mean() - 0.8) < 0.1


def test_nuts_adaptation_errors():
    w = W.std_normal_1d(num_chains=8)
    s = hmc.sampler_for(w, form=hmc.HMC_FORM_PLAIN)
    with pytest.raises(hmc.HMCError, match="rate"):
        s.nuts_sample_chain(1, 1, adapt="simple", rate=0.0)
    with pytest.raises(hmc.HMCError, match="target_accept"):
        s.nuts_sample_chain(1, 1, adapt=True, target_accept=1.0)
    s.close()


# ------------------------------------------------ persistent-kernel edges --
def _edge_workloads():
    return {
        "dense_persistent": W.gauss_dense(dim=21, num_chains=18, step_size=0.15, seed=7),
        "logreg_persistent": W.logreg(130, 6, 5, step_size=0.1, seed=9),
    }


@pytest.mark.parametrize("name", list(_edge_workloads()))
@pytest.mark.parametrize("max_depth", [0, 1])
def test_persistent_shallow_trees_match_oracle(name, max_depth):
    # depth 0 never moves; depth 1 is one sliced leapfrog step: same outcome as the oracle's, chain by chain
    w = _edge_workloads()[name]
    s = hmc.sampler_for(w, form=hmc.HMC_FORM_FUSED)
    g = s.nuts_sample_chain(3, 0, max_depth=max_depth)
    xg = to_np(s.get_state()[0])
    s.close()
    o = oracle.nuts_sample_chain(oracle_target(w), w.seed, w.x0.astype(np.float64), w.step_size, 0, 3,
                                 max_depth=max_depth)
    assert np.array_equal(to_np(g["tree_depth"]), o["depth"])
    assert np.array_equal(to_np(g["n_leapfrog"]), o["n_leapfrog"])
    if max_depth == 0:
        assert np.array_equal(xg, w.x0)
        assert np.all(to_np(g["accept_stat"]) == 0.0)
    assert np.max(rel_err_rows(xg, o["final_x"])) <= 1e-5


@pytest.mark.parametrize("name", list(_edge_workloads()))
def test_persistent_nan_chains_and_single_chain(name):
    w = _edge_workloads()[name]
    B, rate = 12, 0.04
    x0 = w.x0.copy()
    x0[1, 0] = np.nan
    s = hmc.sampler_for(w, form=hmc.HMC_FORM_FUSED, x0=x0)
    g = s.nuts_sample_chain(2, B, max_depth=6, adapt="simple", rate=rate)
    eps = to_np(s.get_state()[1])
    s.close()
    o = oracle.nuts_sample_chain(oracle_target(w), w.seed, x0.astype(np.float64), w.step_size, B, 2, max_depth=6,
                                 adapt="simple", rate=rate)
    assert np.all(to_np(g["accept_stat"])[:, 1] == 0.0) and np.all(to_np(g["n_leapfrog"])[:, 1] == 1)
    assert eps[1] == o["final_eps"][1]
    # one chain alone in its workgroup
    s = hmc.sampler_for(w, form=hmc.HMC_FORM_FUSED, num_chains=1)
    g1 = s.nuts_sample_chain(4, 2, max_depth=6)
    s.close()
    o1 = oracle.nuts_sample_chain(oracle_target(w), w.seed, w.x0[:1].astype(np.float64), w.step_size, 2, 4,
                                  max_depth=6)
    assert np.array_equal(to_np(g1["tree_depth"]), o1["depth"])
    assert np.max(rel_err_rows(to_np(g1["samples"]).reshape(-1, w.dim), o1["samples"].reshape(-1, w.dim))) <= 1e-5
