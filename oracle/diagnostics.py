"""Oracle chain diagnostics (float64).

Test infrastructure only (see ``oracle/__init__``).

* Effective sample size of M chains of n draws (Section 4.1 uses ESS as its
  efficiency measure): multi-chain autocorrelation estimate with Geyer's
  initial monotone sequence (Gelman et al., Bayesian Data Analysis 3rd ed.,
  Section 11.5), without rank normalisation.
* R-hat: the classic (non-split) potential scale reduction of Gelman & Rubin
  (1992), as used for the convergence test of Section 4.1, and the split
  form (Gelman et al., BDA3 Section 11.4): every chain cut into its first and
  last floor(n/2) draws (the middle draw of an odd n dropped), then the
  classic statistic over the 2M half-chains, which also flags a chain whose
  level drifts during the run.
* Time per galaxy to a target number of effective samples: the extrapolation
  formula of Section 4.1, T_warmup / G + T_sampling / (G * n_eff) * target.
"""
from __future__ import annotations

import numpy as np


def _autocov(x):
    """Biased autocovariance of one series at every lag (direct sums)."""
    n = x.shape[0]
    y = x - x.mean()
    return np.array([np.dot(y[: n - t], y[t:]) / n for t in range(n)])


def ess(chains) -> float:
    """ESS of one scalar quantity; chains has shape (M, n)."""
    x = np.asarray(chains, dtype=np.float64)
    M, n = x.shape
    acov = np.stack([_autocov(c) for c in x])          # (M, n)
    chain_mean = x.mean(axis=1)
    W = np.mean(acov[:, 0] * n / (n - 1.0))            # mean within-chain variance
    var_plus = W * (n - 1.0) / n
    if M > 1:
        var_plus += np.var(chain_mean, ddof=1)
    if not var_plus > 0:
        return float(M * n)
    rho = 1.0 - (W - acov.mean(axis=0)) / var_plus
    rho[0] = 1.0
    # Geyer: sums of adjacent pairs, truncated at the first non-positive pair,
    # then forced to be non-increasing.
    pairs = []
    k = 0
    while 2 * k + 1 < n:
        P = rho[2 * k] + rho[2 * k + 1]
        if P <= 0.0:
            break
        if pairs and P > pairs[-1]:
            P = pairs[-1]
        pairs.append(P)
        k += 1
    tau = -1.0 + 2.0 * float(np.sum(pairs)) if pairs else 1.0
    tau = max(tau, 1.0 / np.log10(M * n))
    return float(M * n / tau)


def ess_params(samples) -> np.ndarray:
    """ESS per parameter; samples has shape (M, n, P)."""
    s = np.asarray(samples, dtype=np.float64)
    return np.array([ess(s[:, :, j]) for j in range(s.shape[2])])


def rhat(chains) -> float:
    x = np.asarray(chains, dtype=np.float64)
    M, n = x.shape
    W = np.mean(np.var(x, axis=1, ddof=1))
    B_over_n = np.var(x.mean(axis=1), ddof=1)
    var_plus = (n - 1.0) / n * W + B_over_n
    return float(np.sqrt(var_plus / W))


def split_rhat(chains) -> float:
    x = np.asarray(chains, dtype=np.float64)
    M, n = x.shape
    h = n // 2
    halves = np.concatenate([x[:, :h], x[:, n - h:]], axis=0)      # (2M, h)
    return rhat(halves)


def time_per_galaxy(t_warmup, t_sampling, n_gal, n_eff_mean, target=300.0):
    return t_warmup / n_gal + t_sampling / (n_gal * n_eff_mean) * target
