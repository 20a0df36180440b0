"""Oracle interim prior P0 in sampling coordinates (float64).

Test infrastructure only (see ``oracle/__init__``).

Sampling coordinates theta = (log10 F, log10 s, e1, e2, Dx, Dy), where
(Dx, Dy) are pixel offsets from a per-galaxy reference centroid.  The
interim prior of eq. interim-prior factorises as

    log10 F ~ U(lo_F, hi_F)          (paper: U(-1, 9))
    log10 s ~ U(lo_s, hi_s)          (paper: U(-2, 1), s in arcsec)
    Dx, Dy  ~ N(0, sigma_d)          (paper: sigma_d = 0.5)
    (e1, e2) ~ (1 - E)^2 exp(-E / (2 sigma_e^2)),  E = e1^2 + e2^2 < 1
                                     (paper: sigma_e = 0.3; the density in
                                      (e1, e2) follows from the magnitude
                                      prior eq. ellip-mag-prior and the
                                      polar Jacobian, Section 3.3)

``log_prior`` drops additive constants (they cancel in every HMC energy
difference).  Outside the support it returns -inf.
"""
from __future__ import annotations

import numpy as np

PAPER_INTERIM = dict(log10f_lo=-1.0, log10f_hi=9.0, log10s_lo=-2.0, log10s_hi=1.0,
                     sigma_d=0.5, sigma_e=0.3)


def in_support(theta, ip=PAPER_INTERIM) -> bool:
    lf, ls, e1, e2 = theta[0], theta[1], theta[2], theta[3]
    E = e1 * e1 + e2 * e2
    return bool(ip["log10f_lo"] < lf < ip["log10f_hi"] and
                ip["log10s_lo"] < ls < ip["log10s_hi"] and E < 1.0)


def log_prior(theta, ip=PAPER_INTERIM) -> float:
    if not in_support(theta, ip):
        return -np.inf
    e1, e2, dx, dy = theta[2], theta[3], theta[4], theta[5]
    E = e1 * e1 + e2 * e2
    sd, se = ip["sigma_d"], ip["sigma_e"]
    return float(-(dx * dx + dy * dy) / (2.0 * sd * sd)
                 + 2.0 * np.log(1.0 - E) - E / (2.0 * se * se))


def grad_log_prior(theta, ip=PAPER_INTERIM) -> np.ndarray:
    """Gradient of log_prior inside the support (zero for the uniform axes)."""
    e1, e2, dx, dy = theta[2], theta[3], theta[4], theta[5]
    E = e1 * e1 + e2 * e2
    sd, se = ip["sigma_d"], ip["sigma_e"]
    g = np.zeros(6)
    c = -4.0 / (1.0 - E) - 1.0 / (se * se)
    g[2] = c * e1
    g[3] = c * e2
    g[4] = -dx / (sd * sd)
    g[5] = -dy / (sd * sd)
    return g
