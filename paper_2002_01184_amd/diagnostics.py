"""Convergence diagnostics on the host: split R-hat and effective sample size.

The paper (Sec. 5, Discussion) names rank-normalized R-hat (Vehtari et al.
2019) and the effective sample size (Geyer 2011; Gelman et al. 2013) as the
convergence checks for many-chain MCMC; it does not define them.  This module
follows Vehtari et al. (2019): chains are split in half, draws are rank
normalized, R-hat is the larger of the bulk and folded (tail) values, and ESS
uses the multi-chain autocorrelation with Geyer's initial monotone sequence.

These are measurement tools (they read kept samples back from the device);
they are not part of the sampler's hot path.
"""
from __future__ import annotations

import numpy as np
from scipy.special import ndtri


def _split(x: np.ndarray) -> np.ndarray:
    """x [n, M] -> [n//2, 2M] (first and second halves as separate chains)."""
    n = x.shape[0] // 2
    return np.concatenate([x[:n], x[x.shape[0] - n:]], axis=1)


def _rank_normalize(x: np.ndarray) -> np.ndarray:
    """Normal scores of the pooled ranks (average ranks for ties), Blom offset 3/8."""
    from scipy.stats import rankdata
    S = x.size
    r = rankdata(x, method="average").reshape(x.shape)
    return ndtri((r - 0.375) / (S + 0.25))


def _rhat_basic(x: np.ndarray) -> float:
    """Potential scale reduction of chains x [n, M] (Gelman et al. 2013, eq. 11.4)."""
    n, M = x.shape
    means = x.mean(0)
    W = x.var(0, ddof=1).mean()
    B = n * means.var(ddof=1)
    var_plus = (n - 1) / n * W + B / n
    if W == 0:
        return np.nan
    return float(np.sqrt(var_plus / W))


def rhat(x: np.ndarray) -> float:
    """Rank-normalized split R-hat of one scalar quantity; x is [n_draws, n_chains]."""
    xs = _split(np.asarray(x, dtype=np.float64))
    bulk = _rhat_basic(_rank_normalize(xs))
    folded = np.abs(xs - np.median(xs))
    tail = _rhat_basic(_rank_normalize(folded))
    return float(max(bulk, tail))


def _autocov(x: np.ndarray) -> np.ndarray:
    """Per-chain autocovariance (biased, divided by n) for lags 0..n-1; x [n, M]."""
    n = x.shape[0]
    xc = x - x.mean(0)
    nfft = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(xc, n=nfft, axis=0)
    ac = np.fft.irfft(f * np.conj(f), n=nfft, axis=0)[:n]
    return ac / n


def ess(x: np.ndarray) -> float:
    """Effective sample size of chains x [n, M] (no splitting or normalization).

    rho_t = 1 - (W - mean_m(acov_{t,m})) / var_plus, summed over Geyer's initial
    positive sequence of pair sums with the monotone correction."""
    x = np.asarray(x, dtype=np.float64)
    n, M = x.shape
    if n < 4:
        return np.nan
    acov = _autocov(x)                         # [n, M]
    chain_var = acov[0] * n / (n - 1.0)
    W = chain_var.mean()
    var_plus = W * (n - 1.0) / n
    if M > 1:
        var_plus += x.mean(0).var(ddof=1)
    if var_plus <= 0:
        return np.nan
    rho = 1.0 - (W - acov.mean(1)) / var_plus
    rho[0] = 1.0
    # Geyer: pair sums P_k = rho_2k + rho_2k+1, keep the initial positive run,
    # and make it monotone non-increasing.
    npairs = n // 2
    P = rho[0:2 * npairs:2] + rho[1:2 * npairs:2]
    k = 0
    while k < npairs and P[k] > 0:
        k += 1
    P = np.minimum.accumulate(P[:k]) if k > 0 else P[:0]
    tau = -1.0 + 2.0 * P.sum()
    tau = max(tau, 1.0 / np.log10(n * M))
    return float(n * M / tau)


def ess_bulk(x: np.ndarray) -> float:
    """Bulk ESS: ESS of the rank-normalized split chains; x is [n_draws, n_chains]."""
    return ess(_rank_normalize(_split(np.asarray(x, dtype=np.float64))))


def summarize(samples: np.ndarray, max_dims: int | None = None) -> dict:
    """samples [R, C, D] -> min bulk-ESS and max R-hat over coordinates."""
    R, C, D = samples.shape
    dims = range(D) if max_dims is None else range(min(D, max_dims))
    e = [ess_bulk(samples[:, :, d]) for d in dims]
    r = [rhat(samples[:, :, d]) for d in dims]
    return dict(min_ess_bulk=float(np.min(e)), max_rhat=float(np.max(r)),
                ess_bulk=np.array(e), rhat=np.array(r))


# ---------------------------------------------------------------------------
# The same estimators over torch tensors (any device), for long runs whose
# samples stay on the GPU.  Identical arithmetic to the numpy versions above.
# ---------------------------------------------------------------------------
def _t_rank_normalize(x):
    import torch
    flat = x.reshape(-1)
    S = flat.numel()
    order = torch.argsort(flat, stable=True)
    sorted_vals = flat[order]
    ranks = torch.empty(S, dtype=torch.float64, device=x.device)
    ranks[order] = torch.arange(1, S + 1, dtype=torch.float64, device=x.device)
    # average ranks of ties
    uniq, inv, counts = torch.unique_consecutive(sorted_vals, return_inverse=True, return_counts=True)
    if uniq.numel() < S:
        first = torch.cumsum(counts, 0) - counts + 1
        avg = first.double() + (counts.double() - 1) / 2
        ranks[order] = avg[inv]
    z = torch.special.ndtri((ranks - 0.375) / (S + 0.25))
    return z.reshape(x.shape)


def _t_split(x):
    import torch
    n = x.shape[0] // 2
    return torch.cat([x[:n], x[x.shape[0] - n:]], dim=1)


def _t_rhat_basic(x):
    n = x.shape[0]
    W = x.var(0, unbiased=True).mean()
    B = n * x.mean(0).var(unbiased=True)
    return float(((n - 1) / n * W + B / n).div(W).sqrt())


def t_rhat(x):
    import torch
    xs = _t_split(x.double())
    bulk = _t_rhat_basic(_t_rank_normalize(xs))
    folded = (xs - xs.median()).abs()
    return max(bulk, _t_rhat_basic(_t_rank_normalize(folded)))


def t_ess(x):
    import torch
    x = x.double()
    n, M = x.shape
    xc = x - x.mean(0)
    nfft = 1 << int(np.ceil(np.log2(2 * n)))
    f = torch.fft.rfft(xc, n=nfft, dim=0)
    acov = torch.fft.irfft(f * f.conj(), n=nfft, dim=0)[:n] / n
    chain_var = acov[0] * n / (n - 1.0)
    W = chain_var.mean()
    var_plus = W * (n - 1.0) / n + (x.mean(0).var(unbiased=True) if M > 1 else 0.0)
    rho = 1.0 - (W - acov.mean(1)) / var_plus
    rho = rho.cpu().numpy()
    rho[0] = 1.0
    npairs = n // 2
    P = rho[0:2 * npairs:2] + rho[1:2 * npairs:2]
    k = 0
    while k < npairs and P[k] > 0:
        k += 1
    P = np.minimum.accumulate(P[:k]) if k > 0 else P[:0]
    tau = max(-1.0 + 2.0 * P.sum(), 1.0 / np.log10(n * M))
    return float(n * M / tau)


def t_summarize(samples, progress=None) -> dict:
    """samples: torch tensor [R, C, D] (any device) -> min bulk-ESS, max R-hat.
    progress: optional callable(d, D) invoked after each coordinate."""
    e, r = [], []
    for d in range(samples.shape[2]):
        x = samples[:, :, d]
        e.append(t_ess(_t_rank_normalize(_t_split(x.double()))))
        r.append(t_rhat(x))
        if progress is not None:
            progress(d + 1, samples.shape[2])
    return dict(min_ess_bulk=float(np.min(e)), max_rhat=float(np.max(r)), ess_bulk=np.array(e), rhat=np.array(r))


# ---------------------------------------------------------------------------
# Diagnostics from streamed moments (no stored samples): per chain and
# coordinate the mean and sum of squared deviations of each half of the kept
# draws, and optionally the sums of equal batches.
# ---------------------------------------------------------------------------
def moments_rhat(mean, m2, R: int) -> np.ndarray:
    """Split R-hat per coordinate (Gelman et al. 2013, eq. 11.4, on the 2C half
    chains; not rank-normalized) from mean/m2 [2, C, D] of halves of n = R // 2
    draws (R even).  Equals the split R-hat of the samples themselves."""
    mean = np.asarray(mean, dtype=np.float64)
    m2 = np.asarray(m2, dtype=np.float64)
    if R % 2:
        raise ValueError("split R-hat from moments needs an even number of draws")
    n = R // 2
    mh = mean.reshape(-1, mean.shape[-1])          # [2C, D] half-chain means
    s2 = m2.reshape(-1, m2.shape[-1]) / (n - 1)    # half-chain variances
    W = s2.mean(0)
    B = n * mh.var(0, ddof=1)
    return np.sqrt(((n - 1) / n * W + B / n) / W)


def moments_ess_batch(mean, m2, batch_sum, R: int, batch_len: int) -> np.ndarray:
    """Batch-means ESS per coordinate, pooled over chains: M R s^2 / sigma2_BM with
    s^2 the average within-chain variance and sigma2_BM = batch_len times the
    variance of the batch means about their chain's mean (Flegal & Jones 2010)."""
    mean = np.asarray(mean, dtype=np.float64)
    m2 = np.asarray(m2, dtype=np.float64)
    bs = np.asarray(batch_sum, dtype=np.float64)   # [a, C, D]
    a = bs.shape[0]
    h0 = R // 2
    chain_mean = (h0 * mean[0] + (R - h0) * mean[1]) / R                      # [C, D]
    # within-chain variance from the two halves (parallel-variance combination)
    d = mean[1] - mean[0]
    m2c = m2[0] + m2[1] + d * d * h0 * (R - h0) / R
    s2 = (m2c / (R - 1)).mean(0)
    bm = bs / batch_len
    sig2 = batch_len * ((bm - chain_mean[None]) ** 2).sum(0).sum(0) / (bs.shape[1] * (a - 1))
    return bs.shape[1] * R * s2 / sig2


def moments_summary(mean, m2, R: int, batch_sum=None, batch_len=None) -> dict:
    out = dict(max_rhat=float(np.max(moments_rhat(mean, m2, R))))
    if batch_sum is not None:
        out["min_ess_batch"] = float(np.min(moments_ess_batch(mean, m2, batch_sum, R, batch_len)))
    return out
