"""Oracle multiplicative and additive shear bias by shape-noise cancellation,
with bootstrap errors (Section 3.5 "Multiplicative bias and shape noise
cancellation"; Table 2 reports the results).

Test infrastructure only (see ``oracle/__init__``).

Bias model: an estimator g_hat of an applied shear g obeys g_hat = (1 + m) g + c.
Shape-noise cancellation (Pujol et al. 2019): two datasets share every galaxy
and every noise realisation; one is sheared by +g, the other by -g, with only
g1 non-zero.  With the shear estimator taken as the posterior mean of g,

    m = (g_hat+,1 - g_hat-,1) / (2 |g|) - 1,      c = (g_hat+,2 + g_hat-,2) / 2.

Errors come from a bootstrap over galaxies: a resample draws galaxy indices
with replacement, the same draw is used for both datasets (the pair stays a
pair), and the shear phase is re-run on the original interim samples.  The
error is the standard deviation of the resamples' m (and c); the quoted
estimate uses every galaxy once, not the resamples.

Shear phase for the settings whose population parameters are fixed
(``*-fixed``): the posterior of g alone,
    ln P(g | d) = sum_n ell_n(g) + const,
ell_n the galaxy's Monte-Carlo log-marginal (``shear.galaxy_loglike``).  A
resample that draws galaxy n c_n times has ln P_b(g) = sum_n c_n ell_n(g), so
one table ell_n(g_p) over evaluation points serves every resample.  The
posterior mean is taken on a (g1, g2) grid: the grid points' normalised
posterior weights times their g.
"""
from __future__ import annotations

import math

import numpy as np

from . import shear


def galaxy_loglikes(S, pts, tp: shear.TruePrior, ip: shear.Interim):
    """ell[p, n] = ell_n at point p.  S = (e1p, e2p, l10s, l10f), each (G, K);
    pts (P, 5) = (g1, g2, mu_ln_s, sigma_ln_s, sigma_e)."""
    e1p, e2p, l10s, l10f = S
    G = e1p.shape[0]
    out = np.empty((len(pts), G))
    for p, q in enumerate(pts):
        g = complex(q[0], q[1])
        alpha = (q[2], q[3], q[4])
        for n in range(G):
            out[p, n] = shear.galaxy_loglike(e1p[n], e2p[n], l10s[n],
                                             None if l10f is None else l10f[n], g, alpha, tp, ip)
    return out


def resample_counts(indices, G):
    """c[b, n] = number of times galaxy n appears in resample b (indices (B, G))."""
    idx = np.asarray(indices)
    c = np.zeros((idx.shape[0], G))
    for b in range(idx.shape[0]):
        for n in idx[b]:
            c[b, n] += 1.0
    return c


def resampled_logpost(ell, counts):
    """ln P_b(g_p) = sum over the galaxies drawn (c[b, n] > 0) of c[b, n] ell[p, n]:
    (B, P).  A galaxy not drawn contributes nothing, also where its ell is -inf."""
    c = np.asarray(counts, dtype=np.float64)
    e = np.asarray(ell, dtype=np.float64)
    out = np.empty((c.shape[0], e.shape[0]))
    for b in range(c.shape[0]):
        drawn = c[b] > 0
        out[b] = e[:, drawn] @ c[b, drawn]
    return out


def grid_mean(logpost, gpts):
    """Posterior mean of g for each row of ln P over the grid points gpts (P, 2)."""
    lp = np.atleast_2d(logpost)
    out = np.empty((lp.shape[0], 2))
    for b in range(lp.shape[0]):
        w = np.exp(lp[b] - np.max(lp[b]))
        out[b] = (w @ gpts) / np.sum(w)
    return out


def mc_from_means(gplus, gminus, g_abs):
    """m and c from the posterior means of the +g and -g datasets."""
    gp = np.asarray(gplus, dtype=np.float64)
    gm = np.asarray(gminus, dtype=np.float64)
    m = (gp[..., 0] - gm[..., 0]) / (2.0 * g_abs) - 1.0
    c = 0.5 * (gp[..., 1] + gm[..., 1])
    return m, c


def mc_bootstrap(ell_plus, ell_minus, gpts_plus, gpts_minus, counts, g_abs):
    """m, c from all galaxies and their bootstrap standard deviations; each
    dataset's table and posterior mean are on its own grid."""
    G = ell_plus.shape[1]
    ones = np.ones((1, G))
    m0, c0 = mc_from_means(grid_mean(resampled_logpost(ell_plus, ones), gpts_plus)[0],
                           grid_mean(resampled_logpost(ell_minus, ones), gpts_minus)[0], g_abs)
    mb, cb = mc_from_means(grid_mean(resampled_logpost(ell_plus, counts), gpts_plus),
                           grid_mean(resampled_logpost(ell_minus, counts), gpts_minus), g_abs)
    return {"m": float(m0), "c": float(c0), "m_err": float(np.std(mb)), "c_err": float(np.std(cb)),
            "m_boot": mb, "c_boot": cb}
