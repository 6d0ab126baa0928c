"""Serving form: continuous batching of sampling requests of differing target,
dimension, data size and chain count.  A request's samples are bitwise the
same alone, in a mix of concurrent requests, and as one hmc_sample_chain call
(its random streams are keyed by its own seed and chain ids, its kernels read
and write only its own memory, and the fused kernels resume exactly between
ticks).  Admission follows the HBM budget."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import gpu_available, oracle_target, to_np

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_2002_01184_amd import hmc  # noqa: E402


def _requests():
    a = W.std_normal_1d(num_chains=300, dim=7, state_dtype="f32", L=5, step_size=0.4, burnin=30, results=20, seed=11)
    # two requests of one element-wise shape class, long enough (hundreds of ticks) that they are resident
    # together whatever the delay between their submissions, so they share ragged launches
    b = W.gauss_diag(dim=100, num_chains=200, L=8, step_size=0.05, burnin=1500, results=250, seed=12)
    b2 = W.gauss_diag(dim=90, num_chains=77, L=6, step_size=0.05, burnin=1400, results=170, seed=13, adapt=True)
    c = W.std_normal_1d(num_chains=100, burnin=40, results=20, seed=14)
    d = W.gauss_dense(dim=37, num_chains=45, L=7, step_size=0.1, burnin=10, results=12, seed=15)
    e = W.logreg(1000, 25, 64, L=5, step_size=0.05, burnin=25, results=15, seed=16)
    f = W.logreg(3000, 40, 100, L=4, step_size=0.01, burnin=6, results=9, seed=17, init=0.3)
    g = W.logreg(2000, 300, 48, L=4, step_size=0.005, burnin=5, results=6, seed=18, bf16=True, init=0.1)
    # served with BF16 gradient operands (the server's form for BF16 X up to D = 512)
    h = W.logreg(2500, 400, 70, L=4, step_size=0.004, burnin=6, results=5, seed=19, bf16=True, init=0.1)
    h.extra["grad_bf16"] = True
    return [a, b, b2, c, d, e, f, g, h]


def _bf16(w):
    return w.extra.get("grad_bf16", False)


def _reference(w):
    s = hmc.sampler_for(w, grad_bf16=_bf16(w))
    out = s.sample_chain(w.num_results, w.num_burnin, adapt=w.adapt)
    torch.cuda.synchronize()
    res = {k: v.clone() for k, v in out.items() if v is not None}
    s.close()
    return res


def test_server_results_equal_sample_chain_alone_and_in_mix():
    reqs = _requests()
    refs = [_reference(w) for w in reqs]
    # alone: one request at a time
    srv = hmc.Server(2 << 30, transitions_per_tick=7)
    alone = []
    for w in reqs:
        rid = srv.submit(w, grad_bf16=_bf16(w))
        out, lat = srv.wait(rid)
        assert lat > 0
        alone.append(out)
    st_alone = srv.stats()
    print("server stats after the requests alone:", st_alone)
    # mix: the long diagonal Gaussians first, the rest arriving while they run,
    # some with server-held samples
    order = [1, 2, 0, 3, 4, 7, 8, 5, 6]
    preps = {i: srv.prepare(reqs[i], server_samples=(n % 2 == 1), grad_bf16=_bf16(reqs[i])) for n, i in enumerate(order)}
    mix_ids = {}
    for i in order:
        mix_ids[i] = srv.submit_prepared(preps[i])
    waited = [srv.wait(mix_ids[i]) for i in range(len(reqs))]
    mix = [o for o, _ in waited]
    st = srv.stats()
    srv.close()
    print("server stats:", st)
    print("mix latencies (s):", {reqs[i].name: round(waited[i][1], 3) for i in range(len(reqs))})
    for w, r, al, mx in zip(reqs, refs, alone, mix):
        for k in ["samples", "is_accepted", "step_size", "target_log_prob"]:
            assert torch.equal(al[k], r[k]), (w.name, k, "alone vs sample_chain")
            assert torch.equal(mx[k], r[k]), (w.name, k, "mix vs sample_chain")
    assert st["completed"] == 2 * len(reqs) and st["failed"] == 0
    assert st["max_active"] >= 3
    assert st["batched_launches"] >= 1         # the two diagonal Gaussians share a ragged launch


def test_server_batches_bf16_logistic_requests():
    # three BF16-gradient logistic requests of one shape class (D in (384, 512], L = 4) but
    # different rows, dimension and chain count, with different lengths so that the set of
    # members shrinks inside a tick: each runs one launch per kernel for all of them, and
    # each result is bitwise that of its own hmc_sample_chain call
    reqs = [W.logreg(2500, 400, 70, L=4, step_size=0.004, burnin=30, results=12, seed=31, bf16=True, init=0.1),
            W.logreg(1800, 450, 150, L=4, step_size=0.004, burnin=28, results=10, seed=32, bf16=True, init=0.1),
            W.logreg(700, 500, 33, L=4, step_size=0.004, burnin=33, results=13, seed=33, bf16=True, init=0.1,
                     adapt=False)]
    refs = [hmc.sampler_for(w, grad_bf16=True) for w in reqs]
    ref_out = []
    for s, w in zip(refs, reqs):
        out = s.sample_chain(w.num_results, w.num_burnin, adapt=w.adapt)
        torch.cuda.synchronize()
        ref_out.append({k: v.clone() for k, v in out.items() if v is not None})
        s.close()
    srv = hmc.Server(2 << 30, transitions_per_tick=7)
    preps = [srv.prepare(w, server_samples=(i == 1), grad_bf16=True) for i, w in enumerate(reqs)]
    ids = [srv.submit_prepared(p) for p in preps]
    outs = [srv.wait(i)[0] for i in ids]
    st = srv.stats()
    srv.close()
    print("server stats:", st)
    for w, r, o in zip(reqs, ref_out, outs):
        for k in ["samples", "is_accepted", "step_size", "target_log_prob"]:
            assert torch.equal(o[k], r[k]), (w.name, k)
    assert st["completed"] == 3 and st["failed"] == 0
    assert st["batched_plain_transitions"] >= 1


def test_server_admission_follows_budget():
    w = W.gauss_diag(dim=64, num_chains=512, L=5, step_size=0.05, burnin=10, results=10, seed=3)
    t = hmc.hmc_target(w.kind, 0, w.dim, None, None, hmc.HMC_F32, 0, 0, None, 1.0)
    t.prec = 1      # any non-null pointer for the size query
    cfg = hmc.hmc_config(w.num_chains, w.num_leapfrog_steps, hmc.HMC_F32, hmc.HMC_F32, 0, 0)
    ws = hmc.hmc_workspace_size(t, cfg)
    smp = w.num_results * w.num_chains * w.dim * 4
    one = ((ws + 255) // 256 + (smp + 255) // 256) * 256
    srv = hmc.Server(int(one * 1.5), transitions_per_tick=5)     # room for one request at a time
    ids = [srv.submit(w, seed=s, server_samples=True) for s in range(4)]
    outs = [srv.wait(i)[0] for i in ids]
    st = srv.stats()
    assert st["max_active"] == 1 and st["completed"] == 4
    assert st["peak_bytes_in_use"] <= st["pool_bytes"]
    big = W.gauss_diag(dim=64, num_chains=4096, L=5, step_size=0.05, burnin=10, results=10)
    with pytest.raises(hmc.HMCError) as e:
        srv.submit(big, server_samples=True)
    assert e.value.status == hmc.HMC_E_NOMEM
    srv.close()
    # different seeds give different chains; same seed reproduces
    assert not torch.equal(outs[0]["samples"], outs[1]["samples"])


def test_served_results_match_oracle():
    # a mix served together (fixed step sizes, so trajectories are comparable chain by
    # chain): the paper's FP64 example exactly, FP32 diagonal-Gaussian and logistic
    # requests (one with D > 256 and BF16-stored X) to the FP32 trajectory tolerance
    reqs = [W.std_normal_1d(num_chains=100, burnin=40, results=20, seed=21),
            W.gauss_diag(dim=100, num_chains=200, L=8, step_size=0.05, burnin=30, results=30, seed=22),
            W.logreg(1000, 25, 64, L=5, step_size=0.05, burnin=25, results=15, seed=23),
            W.logreg(2000, 300, 48, L=4, step_size=0.005, burnin=8, results=8, seed=24, bf16=True, init=0.05)]
    for w in reqs:
        w.adapt = False
    srv = hmc.Server(2 << 30, transitions_per_tick=6)
    ids = [srv.submit(w) for w in reqs]
    outs = [srv.wait(i)[0] for i in ids]
    srv.close()
    for w, out in zip(reqs, outs):
        o = oracle.sample_chain(oracle_target(w), w.num_leapfrog_steps, w.seed, w.x0.astype(np.float64),
                                w.step_size, w.num_burnin, w.num_results)
        g_smp = to_np(out["samples"]).astype(np.float64)
        g_acc = to_np(out["is_accepted"]).astype(bool)
        agree = float(np.mean(g_acc == o["is_accepted"]))
        err = np.linalg.norm(g_smp - o["samples"], axis=-1) / np.maximum(np.linalg.norm(o["samples"], axis=-1), 1e-30)
        print(f"served {w.name}: decisions agree {agree:.5f}; sample rel err p50={np.median(err):.2e} "
              f"max={err.max():.2e}")
        if w.state_dtype == "f64":
            assert agree == 1.0 and np.max(np.abs(g_smp - o["samples"])) <= 1e-12
        else:
            assert agree >= 0.999 and np.median(err) < 1e-5
