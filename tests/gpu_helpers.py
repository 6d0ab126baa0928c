"""Helpers of the GPU parity tests: run the HIP path through the C ABI and the
FP64 oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import numpy as np

import oracle
from workloads import Workload


def oracle_target(w: Workload) -> oracle.Target:
    return oracle.Target(w.kind, w.dim, prec=w.prec64(), X=w.X64(), y=w.y64(), prior_scale=w.prior_scale)


def rel_err_rows(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Per-chain ||a - b||_2 / max(||b||_2, 1e-30) (0 where both rows are zero)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    num = np.linalg.norm(a - b, axis=1)
    den = np.maximum(np.linalg.norm(b, axis=1), 1e-30)
    return np.where(num == 0, 0.0, num / den)


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def to_np(t):
    return t.detach().cpu().numpy()


def one_step(w: Workload, sampler, x_state: np.ndarray, t: int, eps: np.ndarray | float | None = None):
    """Both sides take transition t from the same state x_state (state dtype).
    Returns (gpu dict, oracle dict) as numpy arrays."""
    import torch
    dev = sampler.device
    xs = torch.from_numpy(np.ascontiguousarray(x_state)).to(dev)
    eps_t = None
    if eps is not None:
        e = np.broadcast_to(np.asarray(eps, dtype=np.float64), (x_state.shape[0],)).copy()
        eps_t = torch.from_numpy(e).to(dev)
    sampler.set_state(xs, eps_t, t)
    g = sampler.step(want_proposal=True)
    g = {k: to_np(v) for k, v in g.items()}
    _, e_gpu, _ = sampler.get_state()
    e_now = eps if eps is not None else w.step_size
    o = oracle.step(oracle_target(w), w.num_leapfrog_steps, sampler.config.seed, t, e_now,
                    x_state.astype(np.float64))
    return g, o


def decision_report(g, o, seed, t):
    """Agreement of accept decisions; disagreements must sit where |log u + dH|
    is within the dH error."""
    ga = g["is_accepted"].astype(bool)
    oa = o["accepted"]
    agree = float(np.mean(ga == oa))
    C = len(ga)
    u = oracle.accept_uniform(seed, C, t)
    margin = np.abs(np.log(u) + o["delta_h"])
    dh_err = np.abs(g["delta_h"] - o["delta_h"])
    bad = np.nonzero(ga != oa)[0]
    return agree, margin[bad], dh_err
