"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and bench.py.

This module only builds inputs (targets, data sets, initial states) with
numpy's seeded generator.  It holds none of the sampler's arithmetic: no
momentum, no integrator, no accept test.  Random numbers the sampler itself
draws (momenta, accept uniforms) are generated inside the oracle and inside
the HIP kernels from the same Philox4x32-10 streams, each side implementing
the generator on its own.

Workloads follow the paper's HMC example (Sec. 1: 1-D standard normal, 100
chains starting at zero, step size 1.5, 3 leapfrog steps, 300 burn-in + 100
results) and the synthetic shapes of the measured configurations:
  std_normal_1d       1-D N(0,1), 100 chains, FP64
  logreg_1000x25      Bayesian logistic regression, X 1000x25 N(0,1) FP32,
                      1024 chains, L=10, dual averaging to 0.8
  gauss_dense_100     Gaussian D=100, covariance Q diag(lambda) Q^T with
                      lambda log-spaced 1e-2..1e2, Q Haar; 4096 chains, L=20
  logreg_100000x256   logistic regression, X 100000x256 stored BF16,
                      8192 chains, L=10
and two wide shapes of the element-wise targets (1-D N(0,1) at 2^24 chains;
diagonal Gaussian D=1000, 16384 chains) for the HBM-bound plain step.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

STD_NORMAL, GAUSS_DIAG, GAUSS_DENSE, LOGREG = 0, 1, 2, 3
KIND_NAMES = {STD_NORMAL: "std_normal", GAUSS_DIAG: "gauss_diag", GAUSS_DENSE: "gauss_dense",
              LOGREG: "logreg"}


@dataclass
class Workload:
    name: str
    kind: int
    dim: int
    num_chains: int
    num_leapfrog_steps: int
    step_size: float
    num_burnin: int
    num_results: int
    adapt: bool
    seed: int
    state_dtype: str                 # "f64" | "f32"
    x0: np.ndarray                   # [C, D] in state dtype
    prec: np.ndarray | None = None   # diag [D] / dense [D, D], state dtype
    X: np.ndarray | None = None      # [N, D] float32 (values already BF16-exact if x_bf16)
    X_bf16: np.ndarray | None = None  # [N, D] uint16 BF16 bit patterns (None if FP32 data)
    y: np.ndarray | None = None      # [N] uint8
    prior_scale: float = 1.0
    extra: dict = field(default_factory=dict)

    @property
    def n_rows(self) -> int:
        return 0 if self.X is None else self.X.shape[0]

    def chain_steps(self, transitions: int | None = None) -> int:
        T = self.num_burnin + self.num_results if transitions is None else transitions
        return self.num_chains * self.num_leapfrog_steps * T

    # FP64 views of the target data, exactly as the device holds them.
    def prec64(self):
        return None if self.prec is None else self.prec.astype(np.float64)

    def X64(self):
        return None if self.X is None else self.X.astype(np.float64)

    def y64(self):
        return None if self.y is None else self.y.astype(np.float64)


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([seed, stream])


def round_to_bf16(a: np.ndarray):
    """Round float32 to bfloat16 (round to nearest even).  Returns (bits uint16,
    values float32).  Inputs here are finite."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    rounded = (bits + 0x7FFF + ((bits >> 16) & 1)) >> 16
    b16 = rounded.astype(np.uint16)
    vals = (b16.astype(np.uint32) << 16).view(np.float32)
    return b16, vals


def uniform_init(seed: int, C: int, D: int, lo=-2.0, hi=2.0, dtype=np.float32):
    """Over-dispersed starting states x0 ~ U(lo, hi)^D."""
    return _rng(seed, 11).uniform(lo, hi, size=(C, D)).astype(dtype)


def std_normal_1d(num_chains=100, step_size=1.5, L=3, burnin=300, results=100, seed=0,
                  dim=1, state_dtype="f64") -> Workload:
    """The paper's introductory example: N(0,1), chains starting at 0."""
    dt = np.float64 if state_dtype == "f64" else np.float32
    return Workload("std_normal_1d" if dim == 1 else f"std_normal_{dim}d", STD_NORMAL, dim,
                    num_chains, L, step_size, burnin, results, False, seed, state_dtype,
                    np.zeros((num_chains, dim), dtype=dt))


def gauss_diag(dim=1000, num_chains=16384, L=10, step_size=0.1, burnin=500, results=500, seed=0,
               state_dtype="f32", lam_lo=1e-2, lam_hi=1e2, adapt=False) -> Workload:
    """Diagonal Gaussian: variances lambda log-spaced lam_lo..lam_hi, precision 1/lambda."""
    dt = np.float64 if state_dtype == "f64" else np.float32
    lam = np.logspace(np.log10(lam_lo), np.log10(lam_hi), dim) if dim > 1 else np.array([lam_lo])
    prec = (1.0 / lam).astype(dt)
    x0 = uniform_init(seed, num_chains, dim, dtype=dt)
    return Workload(f"gauss_diag_{dim}", GAUSS_DIAG, dim, num_chains, L, step_size, burnin,
                    results, adapt, seed, state_dtype, x0, prec=prec, extra=dict(lam=lam))


def haar_orthogonal(D: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the
    columns' signs fixed by sign(diag R) (Mezzadri 2007)."""
    A = rng.standard_normal((D, D))
    Q, R = np.linalg.qr(A)
    return Q * np.sign(np.diag(R))[None, :]


def gauss_dense(dim=100, num_chains=4096, L=20, step_size=0.1, burnin=1000, results=1000, seed=0,
                lam_lo=1e-2, lam_hi=1e2, adapt=True) -> Workload:
    """Ill-conditioned Gaussian: covariance Q diag(lambda) Q^T, lambda_i =
    10^(log10 lo + i (log10 hi - log10 lo)/(D-1)); precision P = Q diag(1/lambda) Q^T
    built in FP64 and rounded to FP32 (the FP32 matrix is the target)."""
    rng = _rng(seed, 21)
    lam = np.logspace(np.log10(lam_lo), np.log10(lam_hi), dim)
    Q = haar_orthogonal(dim, rng)
    P = (Q * (1.0 / lam)[None, :]) @ Q.T
    P = 0.5 * (P + P.T)
    P32 = P.astype(np.float32)
    P32 = np.ascontiguousarray(np.triu(P32) + np.triu(P32, 1).T)   # exactly symmetric
    x0 = uniform_init(seed, num_chains, dim)
    return Workload(f"gauss_dense_{dim}", GAUSS_DENSE, dim, num_chains, L, step_size, burnin,
                    results, adapt, seed, "f32", x0, prec=P32, extra=dict(lam=lam, Q=Q))


def logreg(n_rows=1000, dim=25, num_chains=1024, L=10, step_size=0.05, burnin=1000, results=1000,
           seed=0, bf16=False, adapt=True, init="uniform") -> Workload:
    """Synthetic Bayesian logistic regression: X iid N(0,1) (rounded to BF16 when
    bf16, and that rounded array is the data set), w_true ~ N(0, I),
    y_n ~ Bernoulli(sigmoid(x_n . w_true)), prior N(0, I)."""
    rng = _rng(seed, 31)
    X = rng.standard_normal((n_rows, dim)).astype(np.float32)
    Xb = None
    if bf16:
        Xb, X = round_to_bf16(X)
    w = rng.standard_normal(dim)
    logits = X.astype(np.float64) @ w
    prob = 0.5 * (1.0 + np.tanh(0.5 * logits))
    y = (rng.uniform(size=n_rows) < prob).astype(np.uint8)
    if init == "uniform":
        x0 = uniform_init(seed, num_chains, dim)
    else:  # near the data-generating weights, for sharply peaked posteriors
        x0 = (w[None, :] + _rng(seed, 12).uniform(-init, init, size=(num_chains, dim))).astype(np.float32)
    name = f"logreg_{n_rows}x{dim}" + ("_bf16" if bf16 else "")
    return Workload(name, LOGREG, dim, num_chains, L, step_size, burnin, results, adapt, seed, "f32",
                    x0, X=X, X_bf16=Xb, y=y, extra=dict(w_true=w))


# The measured configurations -------------------------------------------
def cfg_std_normal_1d():
    return std_normal_1d()


def cfg_logreg_1000x25():
    return logreg(1000, 25, 1024, L=10, step_size=0.05, burnin=1000, results=1000)


def cfg_logreg_10000x25():
    # ten times the rows of the 1000x25 workload: X (1.1 MB padded) is beyond a workgroup's LDS
    return logreg(10000, 25, 1024, L=10, step_size=0.015, burnin=1000, results=1000)


def cfg_gauss_dense_100():
    return gauss_dense(100, 4096, L=20, step_size=0.1, burnin=1000, results=1000)


def cfg_logreg_100000x256():
    return logreg(100000, 256, 8192, L=10, step_size=0.005, burnin=1000, results=1000, bf16=True,
                  init=0.05)


def cfg_logreg_100000x512():
    # the widest logistic request of the served stream (D up to 512), 4096 chains
    return logreg(100000, 512, 4096, L=10, step_size=0.003, burnin=1000, results=1000, bf16=True,
                  init=0.05)


# Wide shapes of the element-wise targets, for the HBM roofline of the plain step:
# the paper's 1-D example at 2^24 chains (FP64) and a diagonal Gaussian D=1000
# (variances 1e-2..1e2) with 16384 chains (FP32).
def cfg_std_normal_1d_wide():
    w = std_normal_1d(num_chains=1 << 24, burnin=50, results=50)
    w.name = "std_normal_1d_2^24"
    return w


def cfg_gauss_diag_1000():
    return gauss_diag(dim=1000, num_chains=16384, L=10, step_size=0.1, burnin=100, results=100)


CONFIGS = {
    "std_normal_1d": cfg_std_normal_1d,
    "std_normal_1d_wide": cfg_std_normal_1d_wide,
    "gauss_diag_1000": cfg_gauss_diag_1000,
    "logreg_1000x25": cfg_logreg_1000x25,
    "logreg_10000x25": cfg_logreg_10000x25,
    "gauss_dense_100": cfg_gauss_dense_100,
    "logreg_100000x256": cfg_logreg_100000x256,
    "logreg_100000x512": cfg_logreg_100000x512,
}


def served_stream(n_requests=64, rate=50.0, seed=0, scale="small", progress=None):
    """Seeded stream of sampling requests with Poisson arrivals.

    Mix: 50% diagonal-Gaussian requests (D ~ U{10..1000}), 50% logistic
    regression (BF16 X, N ~ U{n_lo..n_hi}, D ~ U{25..d_hi}); chains per request
    log-uniform in [64, c_hi]; L = 10; burn-in + kept transitions per request.
    scale="full" is the configuration as stated (N up to 1e5, D up to 512,
    chains up to 16384, 500 + 500 transitions); scale="small" keeps the mix and
    the arrival process but bounds N <= 1e4, D <= 128, chains <= 2048 and uses
    100 + 100 transitions, so that a stream finishes in seconds.
    progress(i, n) is called after each request is generated.
    Returns a list of (arrival_time_s, Workload)."""
    rng = _rng(seed, 41)
    if scale == "full":
        n_lo, n_hi, d_hi, c_hi, B, R = 1000, 100000, 512, 16384, 500, 500
    else:
        n_lo, n_hi, d_hi, c_hi, B, R = 1000, 10000, 128, 2048, 100, 100
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        C = int(round(np.exp(rng.uniform(np.log(64), np.log(c_hi)))))
        rseed = int(rng.integers(0, 2**31))
        if rng.uniform() < 0.5:
            D = int(rng.integers(10, 1001))
            w = gauss_diag(dim=D, num_chains=C, L=10, step_size=0.05, burnin=B, results=R, seed=rseed,
                           adapt=True)
        else:
            N = int(rng.integers(n_lo, n_hi + 1))
            D = int(rng.integers(25, d_hi + 1))
            w = logreg(N, D, C, L=10, step_size=0.01, burnin=B, results=R, seed=rseed, bf16=True, adapt=True,
                       init=0.1)
        w.name = f"req{i}_{w.name}"
        out.append((t, w))
        if progress is not None:
            progress(i + 1, n_requests)
    return out
