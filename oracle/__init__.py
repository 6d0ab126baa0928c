"""ctypes wrapper of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py are the only callers.  The product path
(paper_2002_01184_amd) never imports this package, and this package never
imports the product.  Arrays are numpy float64 (targets are upcast exactly by
the caller), states are [C, D] row-major.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB_PATH selects another build of oracle.c (the sanitizer build)
_LIB_OVERRIDE = os.environ.get("ORACLE_LIB_PATH")
_LIB_PATH = _LIB_OVERRIDE or os.path.join(_HERE, "liboracle.so")

STD_NORMAL, GAUSS_DIAG, GAUSS_DENSE, LOGREG = 0, 1, 2, 3
TAG_MOMENTUM, TAG_ACCEPT, TAG_SWAP = 0, 1, 2
TAG_NUTS_MERGE, TAG_NUTS_DIR, TAG_NUTS_TOP, TAG_NUTS_SLICE = 3, 4, 5, 6
ADAPT_NONE, ADAPT_DUAL_AVERAGING, ADAPT_SIMPLE = 0, 1, 2

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i32p = ctypes.POINTER(ctypes.c_int32)


class _Target(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("dim", ctypes.c_int64),
                ("prec", _dp), ("X", _dp), ("y", _dp), ("n_rows", ctypes.c_int64),
                ("prior_scale", ctypes.c_double), ("beta", ctypes.c_double), ("scale", _dp), ("shift", _dp)]


class _DualAvg(ctypes.Structure):
    _fields_ = [("log_eps", ctypes.c_double), ("hbar", ctypes.c_double),
                ("log_eps_bar", ctypes.c_double), ("mu", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        srcs = [os.path.join(_HERE, f) for f in ("oracle.c", "oracle.h")]
        if not _LIB_OVERRIDE and (not os.path.exists(_LIB_PATH)
                                  or max(os.path.getmtime(f) for f in srcs) > os.path.getmtime(_LIB_PATH)):
            from . import build as _b  # noqa: F401  (build script beside the source)
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.orc_philox_many.argtypes = [ctypes.c_int64, _u32p, _u32p, _u32p]
        L.orc_normal4.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_uint32, _dp]
        L.orc_momentum.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64, _dp]
        L.orc_momentum_many.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int64, _dp]
        L.orc_accept_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        L.orc_accept_uniform.restype = ctypes.c_double
        L.orc_accept_uniform_many.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, _dp]
        L.orc_logp_grad.argtypes = [ctypes.POINTER(_Target), _dp, _dp]
        L.orc_logp_grad.restype = ctypes.c_double
        L.orc_leapfrog.argtypes = [ctypes.POINTER(_Target), ctypes.c_double, ctypes.c_int32, _dp, _dp, _dp, _dp]
        L.orc_transition.argtypes = [ctypes.POINTER(_Target), ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_int32, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_transition.restype = ctypes.c_int
        L.orc_dual_avg_init.argtypes = [ctypes.POINTER(_DualAvg), ctypes.c_double]
        L.orc_dual_avg_update.argtypes = [ctypes.POINTER(_DualAvg), ctypes.c_int64, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_bootstrap.argtypes = [ctypes.POINTER(_Target), ctypes.c_int64, _dp, _dp, _dp, ctypes.c_int32]
        L.orc_step.argtypes = [ctypes.POINTER(_Target), ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                               ctypes.c_uint32, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _u8p,
                               ctypes.c_int32]
        L.orc_sample_chain.argtypes = [ctypes.POINTER(_Target), ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                       ctypes.c_uint32, _dp, _dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, _dp, _dp, _u8p, _dp, _dp, ctypes.c_int32]
        L.orc_simple_adapt.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_simple_adapt.restype = ctypes.c_double
        L.orc_sample_chain.restype = ctypes.c_int
        L.orc_nuts_transition.argtypes = [ctypes.POINTER(_Target), ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_double, ctypes.c_int32, _dp, _dp, _dp, _i32p, _i32p, _dp, _dp,
                                          _i32p]
        L.orc_nuts_transition.restype = ctypes.c_int
        L.orc_nuts_sample_chain.argtypes = [ctypes.POINTER(_Target), ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
                                            _dp, _dp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, _dp, _i32p, _i32p, _dp, ctypes.c_int32]
        L.orc_nuts_sample_chain.restype = ctypes.c_int
        L.orc_remc_swap.argtypes = [ctypes.POINTER(_Target), ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                    ctypes.c_uint32, _dp, _dp, _dp, _u8p]
        L.orc_remc_sample_chain.argtypes = [ctypes.POINTER(_Target), ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32, _dp, _dp,
                                            ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            _dp, _u8p, _u8p, ctypes.c_int32]
        L.orc_remc_sample_chain.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, typ=_dp):
    if a is None:
        return None
    return a.ctypes.data_as(typ)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Target:
    """A target in FP64.  kind: STD_NORMAL / GAUSS_DIAG / GAUSS_DENSE / LOGREG."""
    kind: int
    dim: int
    prec: np.ndarray | None = None
    X: np.ndarray | None = None
    y: np.ndarray | None = None
    prior_scale: float = 1.0
    beta: float = 1.0          # inverse temperature (replica exchange): beta * logp
    scale: np.ndarray | None = None   # transformed kernel: x = shift + scale * z
    shift: np.ndarray | None = None

    def __post_init__(self):
        if self.prec is not None:
            self.prec = _f64(self.prec)
        if self.X is not None:
            self.X = _f64(self.X)
        if self.y is not None:
            self.y = _f64(self.y)
        if self.scale is not None:
            self.scale = _f64(self.scale)
        if self.shift is not None:
            self.shift = _f64(self.shift)
        n = 0 if self.X is None else self.X.shape[0]
        self._c = _Target(self.kind, 0, self.dim, _p(self.prec), _p(self.X), _p(self.y), n,
                          float(self.prior_scale), float(self.beta), _p(self.scale), _p(self.shift))

    def tempered(self, beta: float) -> "Target":
        """The same target at inverse temperature beta (shares the arrays)."""
        return Target(self.kind, self.dim, self.prec, self.X, self.y, self.prior_scale, float(beta),
                      self.scale, self.shift)

    def transformed(self, scale, shift=None) -> "Target":
        """The pulled-back target of the diagonal affine bijector x = shift + scale * z."""
        return Target(self.kind, self.dim, self.prec, self.X, self.y, self.prior_scale, self.beta,
                      np.broadcast_to(_f64(scale), (self.dim,)).copy(),
                      None if shift is None else np.broadcast_to(_f64(shift), (self.dim,)).copy())

    @property
    def c(self):
        return ctypes.byref(self._c)


# ---------------------------------------------------------------- RNG --
def philox(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32-10 blocks: ctr [n, 4] uint32 -> [n, 4] uint32 under key (k0, k1)."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.asarray(key, dtype=np.uint32)
    out = np.empty_like(ctr)
    lib().orc_philox_many(ctr.shape[0], _p(ctr, _u32p), _p(k, _u32p), _p(out, _u32p))
    return out


def normal4(seed: int, c0: int, c1: int, c2: int, tag: int) -> np.ndarray:
    z = np.empty(4)
    lib().orc_normal4(seed, c0, c1, c2, tag, _p(z))
    return z


def momentum(seed: int, C: int, t: int, D: int) -> np.ndarray:
    p = np.empty((C, D))
    lib().orc_momentum_many(seed, C, t, D, _p(p))
    return p


def accept_uniform(seed: int, C: int, t: int) -> np.ndarray:
    u = np.empty(C)
    lib().orc_accept_uniform_many(seed, C, t, _p(u))
    return u


# ------------------------------------------------------------- target --
def logp_grad(tg: Target, x: np.ndarray):
    """Batch semantics: x [C, D] -> (logp [C], grad [C, D])."""
    x = _f64(x)
    squeeze = x.ndim == 1
    x2 = x.reshape(-1, tg.dim)
    lp = np.empty(x2.shape[0])
    g = np.empty_like(x2)
    for c in range(x2.shape[0]):
        lp[c] = lib().orc_logp_grad(tg.c, _p(x2[c]), _p(g[c]))
    if squeeze:
        return lp[0], g[0]
    return lp, g


def leapfrog(tg: Target, eps: float, L: int, x: np.ndarray, p: np.ndarray):
    """One chain: L leapfrog steps from (x, p).  Returns (x_L, p_L, logp_L, g_L)."""
    x = _f64(x).copy()
    p = _f64(p).copy()
    _, g = logp_grad(tg, x)
    g = g.copy()
    lp = ctypes.c_double(0.0)
    lib().orc_leapfrog(tg.c, eps, L, _p(x), _p(p), _p(g), ctypes.byref(lp))
    return x, p, lp.value, g


def bootstrap(tg: Target, x: np.ndarray, nthreads: int = 0):
    x = _f64(x)
    C = x.shape[0]
    lp = np.empty(C)
    g = np.empty_like(x)
    lib().orc_bootstrap(tg.c, C, _p(x), _p(lp), _p(g), nthreads)
    return lp, g


def step(tg: Target, L: int, seed: int, t: int, eps, x, logp=None, g=None, nthreads: int = 0):
    """One transition of all chains from state x (logp/g recomputed if None).

    Returns dict with new state x/logp/g, proposal x_prop/p_prop/logp_prop,
    delta_h, log_accept_ratio, accepted."""
    x = _f64(x).copy()
    C, D = x.shape
    if logp is None or g is None:
        logp, g = bootstrap(tg, x, nthreads)
    logp = _f64(logp).copy()
    g = _f64(g).copy()
    eps = np.broadcast_to(_f64(eps), (C,)).copy()
    xp = np.empty_like(x)
    pp = np.empty_like(x)
    lpp = np.empty(C)
    dh = np.empty(C)
    lar = np.empty(C)
    acc = np.empty(C, dtype=np.uint8)
    lib().orc_step(tg.c, C, L, seed, t, _p(eps), _p(x), _p(logp), _p(g), _p(xp), _p(pp), _p(lpp),
                   _p(dh), _p(lar), _p(acc, _u8p), nthreads)
    return dict(x=x, logp=logp, g=g, x_prop=xp, p_prop=pp, logp_prop=lpp, delta_h=dh,
                log_accept_ratio=lar, accepted=acc.astype(bool))


def step_chains(tg: Target, L: int, seed: int, t: int, eps, x_rows, chain_ids, nthreads: int = 0):
    """Transition t of the chains with the given ids only (rows of x_rows are their
    states): the same Philox streams as `step` over all chains, for full-size
    workloads whose every chain the oracle cannot afford.  Chains run on a
    thread pool (the C call releases the GIL).  Returns the same fields as `step`."""
    from concurrent.futures import ThreadPoolExecutor
    x = _f64(x_rows).copy()
    K, D = x.shape
    ids = [int(c) for c in chain_ids]
    assert len(ids) == K
    eps = np.broadcast_to(_f64(eps), (K,)).copy()
    logp, g = np.empty(K), np.empty_like(x)
    xp, pp = np.empty_like(x), np.empty_like(x)
    lpp, dh, lar = np.empty(K), np.empty(K), np.empty(K)
    acc = np.empty(K, dtype=bool)

    def one(i):
        lp = ctypes.c_double(lib().orc_logp_grad(tg.c, _p(x[i]), _p(g[i])))
        d = [ctypes.c_double() for _ in range(3)]
        a = lib().orc_transition(tg.c, seed, ids[i], t, L, float(eps[i]), _p(x[i]), ctypes.byref(lp), _p(g[i]),
                                 _p(xp[i]), _p(pp[i]), ctypes.byref(d[0]), ctypes.byref(d[1]), ctypes.byref(d[2]))
        logp[i], lpp[i], dh[i], lar[i], acc[i] = lp.value, d[0].value, d[1].value, d[2].value, bool(a)

    workers = nthreads if nthreads > 0 else min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(one, range(K)))
    return dict(x=x, logp=logp, g=g, x_prop=xp, p_prop=pp, logp_prop=lpp, delta_h=dh,
                log_accept_ratio=lar, accepted=acc)


def dual_avg_run(eps0: float, alphas, target_accept=0.8, gamma=0.05, t0=10.0, kappa=0.75):
    """Run the dual-averaging recursion over a scripted alpha sequence; returns
    arrays (log_eps, hbar, log_eps_bar) after each iteration m = 1..len(alphas)."""
    s = _DualAvg()
    lib().orc_dual_avg_init(ctypes.byref(s), eps0)
    out = []
    for m, a in enumerate(alphas, start=1):
        lib().orc_dual_avg_update(ctypes.byref(s), m, float(a), target_accept, gamma, t0, kappa)
        out.append((s.log_eps, s.hbar, s.log_eps_bar))
    out = np.array(out)
    return out[:, 0], out[:, 1], out[:, 2], s.mu


def _adapt_code(adapt) -> int:
    """adapt: False / True (dual averaging) / "dual_averaging" / "simple"."""
    if adapt is False or adapt is None:
        return ADAPT_NONE
    if adapt is True or adapt == "dual_averaging":
        return ADAPT_DUAL_AVERAGING
    if adapt == "simple":
        return ADAPT_SIMPLE
    raise ValueError(f"unknown adaptation {adapt!r}")


def simple_adapt(eps: float, alpha: float, target_accept: float = 0.8, rate: float = 0.01) -> float:
    return lib().orc_simple_adapt(eps, alpha, target_accept, rate)


def sample_chain(tg: Target, L: int, seed: int, x0, eps0, num_burnin: int, num_results: int,
                 adapt=False, target_accept=0.8, gamma=0.05, t0=10.0, kappa=0.75, rate=0.01,
                 t_begin: int = 0, store_samples: bool = True, nthreads: int = 0):
    """Oracle sample_chain.  adapt: False, True / "dual_averaging", or "simple"
    (multiplicative rule with the given rate).  Returns dict(samples [R,C,D] or
    None, step_size, is_accepted, log_accept_ratio, target_log_prob [R,C],
    final_x [C,D], final_eps [C])."""
    x = _f64(x0).copy()
    C, D = x.shape
    eps = np.broadcast_to(_f64(eps0), (C,)).copy()
    R = num_results
    samples = np.empty((R, C, D)) if store_samples else None
    st = np.empty((R, C))
    acc = np.empty((R, C), dtype=np.uint8)
    lar = np.empty((R, C))
    lp = np.empty((R, C))
    lib().orc_sample_chain(tg.c, C, L, seed, t_begin, _p(x), _p(eps), num_burnin, num_results,
                           _adapt_code(adapt), target_accept, gamma, t0, kappa, rate,
                           _p(samples), _p(st), _p(acc, _u8p), _p(lar), _p(lp), nthreads)
    return dict(samples=samples, step_size=st, is_accepted=acc.astype(bool), log_accept_ratio=lar,
                target_log_prob=lp, final_x=x, final_eps=eps)


# ------------------------------------------------------ replica exchange --
def _replica_targets(tg: Target, betas):
    tgs = [tg.tempered(b) for b in betas]
    arr = (_Target * len(tgs))(*[t._c for t in tgs])
    return tgs, arr


def remc_swap(tg: Target, betas, seed: int, t: int, x, logp=None, g=None):
    """One exchange step (swap index t) over K = len(betas) replicas of M chains,
    x [K*M, D] replica-major.  logp/g are each chain's tempered values (recomputed
    if None).  Returns dict(x, logp, g, swapped)."""
    betas = list(betas)
    K = len(betas)
    x = _f64(x).copy()
    C, D = x.shape
    M = C // K
    tgs, arr = _replica_targets(tg, betas)
    if logp is None or g is None:
        logp = np.empty(C)
        g = np.empty_like(x)
        for c in range(C):
            logp[c] = lib().orc_logp_grad(tgs[c // M].c, _p(x[c]), _p(g[c]))
    logp = _f64(logp).copy()
    g = _f64(g).copy()
    sw = np.empty(C, dtype=np.uint8)
    lib().orc_remc_swap(arr, K, M, seed, t, _p(x), _p(logp), _p(g), _p(sw, _u8p))
    return dict(x=x, logp=logp, g=g, swapped=sw.astype(bool))


def remc_sample_chain(tg: Target, betas, L: int, seed: int, x0, eps0, num_burnin: int, num_results: int,
                      adapt=False, target_accept=0.8, gamma=0.05, t0=10.0, kappa=0.75, rate=0.01,
                      t_begin: int = 0, store_samples: bool = True, nthreads: int = 0):
    """Oracle replica-exchange sample_chain.  x0 [K*M, D] replica-major.
    Returns dict(samples [R, K*M, D] (post-exchange states), is_accepted, swapped
    [R, K*M], final_x, final_eps)."""
    betas = list(betas)
    K = len(betas)
    x = _f64(x0).copy()
    C, D = x.shape
    assert C % K == 0
    M = C // K
    eps = np.broadcast_to(_f64(eps0), (C,)).copy()
    R = num_results
    tgs, arr = _replica_targets(tg, betas)
    samples = np.empty((R, C, D)) if store_samples else None
    acc = np.empty((R, C), dtype=np.uint8)
    sw = np.empty((R, C), dtype=np.uint8)
    lib().orc_remc_sample_chain(arr, K, M, L, seed, t_begin, _p(x), _p(eps), num_burnin, num_results,
                                _adapt_code(adapt), target_accept, gamma, t0, kappa, rate, _p(samples),
                                _p(acc, _u8p), _p(sw, _u8p), nthreads)
    return dict(samples=samples, is_accepted=acc.astype(bool), swapped=sw.astype(bool), final_x=x,
                final_eps=eps)


# ------------------------------------------------- transformed kernel --
def transformed_sample_chain(tg: Target, scale, shift, L: int, seed: int, x0, eps0, num_burnin: int,
                             num_results: int, **kw):
    """TransformedTransitionKernel (paper Sec. 4.1) with x = shift + scale * z:
    the HMC chain runs on z (initial z0 = (x0 - shift) / scale) against the
    pulled-back target and its samples are pushed forward to x."""
    tz = tg.transformed(scale, shift)
    mu = np.zeros(tg.dim) if shift is None else np.broadcast_to(_f64(shift), (tg.dim,))
    s = tz.scale
    z0 = (_f64(x0) - mu) / s
    r = sample_chain(tz, L, seed, z0, eps0, num_burnin, num_results, **kw)
    if r["samples"] is not None:
        r["samples"] = mu + s * r["samples"]
    r["final_x"] = mu + s * r["final_x"]
    return r


# ------------------------------------------------------------------- NUTS --
def nuts_transition(tg: Target, seed: int, chain: int, t: int, eps: float, max_depth: int, x, logp=None, g=None,
                    record_leaves=False):
    """One NUTS transition of one chain.  Returns dict(x, logp, g, moved, depth,
    n_leapfrog, accept_stat); with record_leaves also leaf_x [n_leapfrog, D] and
    leaf_j [n_leapfrog] (every leaf's position and doubling, in build order)."""
    x = _f64(x).copy()
    if logp is None or g is None:
        logp, g = logp_grad(tg, x)
    g = _f64(g).copy()
    lp = ctypes.c_double(float(logp))
    dep = ctypes.c_int32(0)
    nl = ctypes.c_int32(0)
    stat = ctypes.c_double(0.0)
    nmax = (1 << max_depth) - 1
    leaf_x = np.zeros((max(nmax, 1), x.shape[0])) if record_leaves else None
    leaf_j = np.zeros(max(nmax, 1), dtype=np.int32) if record_leaves else None
    moved = lib().orc_nuts_transition(tg.c, seed, chain, t, eps, max_depth, _p(x), ctypes.byref(lp), _p(g),
                                      ctypes.byref(dep), ctypes.byref(nl), ctypes.byref(stat),
                                      _p(leaf_x) if record_leaves else None,
                                      _p(leaf_j, _i32p) if record_leaves else None)
    out = dict(x=x, logp=lp.value, g=g, moved=bool(moved), depth=dep.value, n_leapfrog=nl.value,
               accept_stat=stat.value)
    if record_leaves:
        out["leaf_x"] = leaf_x[:nl.value]
        out["leaf_j"] = leaf_j[:nl.value]
    return out


def nuts_sample_chain(tg: Target, seed: int, x0, eps0, num_burnin: int, num_results: int, max_depth: int = 10,
                      t_begin: int = 0, nthreads: int = 0, adapt=False, target_accept=0.8, gamma=0.05, t0=10.0,
                      kappa=0.75, rate=0.01):
    """Oracle NUTS sample_chain.  adapt as sample_chain's (the statistic is
    Algorithm 6's accept_stat).  Returns dict(samples [R,C,D], depth [R,C],
    n_leapfrog [R,C], accept_stat [R,C], final_x, final_eps)."""
    x = _f64(x0).copy()
    C, D = x.shape
    eps = np.broadcast_to(_f64(eps0), (C,)).copy()
    R = num_results
    samples = np.empty((R, C, D))
    dep = np.empty((R, C), dtype=np.int32)
    nl = np.empty((R, C), dtype=np.int32)
    stat = np.empty((R, C))
    lib().orc_nuts_sample_chain(tg.c, C, seed, t_begin, _p(x), _p(eps), max_depth, num_burnin, num_results,
                                _adapt_code(adapt), target_accept, gamma, t0, kappa, rate,
                                _p(samples), _p(dep, _i32p), _p(nl, _i32p), _p(stat), nthreads)
    return dict(samples=samples, depth=dep, n_leapfrog=nl, accept_stat=stat, final_x=x, final_eps=eps)
