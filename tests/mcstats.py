"""Monte-Carlo standard errors for pooled MCMC moments (test helper).

Batch means: each chain's K retained samples are cut into B = floor(sqrt(K))
consecutive batches of equal size; the variance of the batch means (pooled
over chains, around the pooled mean) times the batch size estimates the
asymptotic variance.  The standard deviation's error uses batch means of the
squared deviations and the delta method d(sd) = d(var) / (2 sd).
"""
from __future__ import annotations

import numpy as np


def _batch(samples: np.ndarray):
    """samples [C, K, ...] -> batch means [C*B, ...] and batch size."""
    C, K = samples.shape[:2]
    B = max(int(np.floor(np.sqrt(K))), 2)
    s = K // B
    x = samples[:, : B * s].reshape((C, B, s) + samples.shape[2:]).mean(axis=2)
    return x.reshape((C * B,) + samples.shape[2:]), s, C * B * s


def mcse_mean(samples: np.ndarray) -> np.ndarray:
    bm, s, n = _batch(samples)
    var = s * bm.var(axis=0, ddof=1)
    return np.sqrt(var / n)


def mcse_std(samples: np.ndarray) -> np.ndarray:
    C, K = samples.shape[:2]
    flat = samples.reshape((C * K,) + samples.shape[2:])
    mu = flat.mean(axis=0)
    sd = flat.std(axis=0, ddof=1)
    sq = (samples - mu) ** 2
    return mcse_mean(sq) / (2.0 * np.maximum(sd, 1e-300))


def zscores(a_mean, b_mean, a_se, b_se):
    return (np.asarray(a_mean) - np.asarray(b_mean)) / np.sqrt(np.asarray(a_se) ** 2 +
                                                              np.asarray(b_se) ** 2)


def mcse_mean_ensemble(samples: np.ndarray) -> np.ndarray:
    """samples [W, K, ...] of W coupled walkers: the pooled mean is the mean
    of the walker-averaged series, whose batch means give its error."""
    return mcse_mean(samples.mean(axis=0, keepdims=True))


def mcse_std_ensemble(samples: np.ndarray) -> np.ndarray:
    W, K = samples.shape[:2]
    flat = samples.reshape((W * K,) + samples.shape[2:])
    mu = flat.mean(axis=0)
    sd = flat.std(axis=0, ddof=1)
    sq = ((samples - mu) ** 2).mean(axis=0, keepdims=True)
    return mcse_mean(sq) / (2.0 * np.maximum(sd, 1e-300))
