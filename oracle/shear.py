"""Oracle shear-phase posterior (float64).

Test infrastructure only (see ``oracle/__init__``).

Given interim samples omega'_nk = (e1', e2', log10 s, log10 F) of each galaxy
n (k = 1..K) drawn under the interim prior P0, the Monte-Carlo shear
likelihood eq. likelihood-shear is

    P(d | g, alpha) ~ prod_n (Z_n / K) sum_k p(omega'_nk | alpha, g) / P0(omega'_nk)

and eq. true-prior-jacobian-shear writes the numerator as the true prior of
the intrinsic properties times |d eps / d eps'|, with the intrinsic
ellipticity eps = h_g^-1(eps') obtained by inverting eq. shear-transform:

    eps = (eps' - g) / (1 - conj(g) eps'),
    |d eps / d eps'| = (1 - |g|^2)^2 / |1 - conj(g) eps'|^4

(the map is holomorphic, so the real 2x2 Jacobian determinant is the squared
modulus of its complex derivative).  Centroid terms cancel (Section 3.3) and
are omitted; Z_n does not depend on (g, alpha) and is dropped.

All densities are taken in the sampling coordinates (e1, e2, log10 s,
log10 F).  Hyper-parameters alpha = (mu_ln_s, sigma_ln_s, sigma_e):
ln s ~ N(mu_ln_s, sigma_ln_s) (so log10 s ~ N(mu/ln10, sigma/ln10)); flux
lognormal with fixed (mu_ln_F, sigma_ln_F) or omitted; intrinsic ellipticity
either the prior of eq. ellip-mag-prior in (e1, e2) form (kind 0, support
|e| < 1) or a circular 2-D Gaussian truncated at |e| < e_max (kind 1).
The shear prior is uniform on the unit disk and the hyper-priors are uniform
boxes, so both add 0 inside their support.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

LN10 = math.log(10.0)
E_KIND_BA14 = 0
E_KIND_TRUNC_GAUSS = 1


@dataclass
class TruePrior:
    e_kind: int = E_KIND_TRUNC_GAUSS
    e_max: float = 0.7
    mu_lnf: float = math.nan        # NaN: flux term omitted
    sig_lnf: float = math.nan
    size_term: bool = True          # False: size term omitted (true = interim in size)


@dataclass
class Interim:
    log10f_lo: float = -1.0
    log10f_hi: float = 9.0
    log10s_lo: float = -2.0
    log10s_hi: float = 1.0
    sigma_e: float = 0.3


# ---- shear response (eq. shear-transform) -------------------------------------

def shear_forward(e, g):
    """h_g(e) = (e + g) / (1 + conj(g) e) for complex arrays."""
    return (e + g) / (1.0 + np.conj(g) * e)


def shear_inverse(ep, g):
    return (ep - g) / (1.0 - np.conj(g) * ep)


def log_jacobian(ep, g):
    """ln |d eps / d eps'| of the inverse map."""
    return 2.0 * np.log(1.0 - abs(g) ** 2) - 4.0 * np.log(np.abs(1.0 - np.conj(g) * ep))


# ---- ellipticity densities ---------------------------------------------------

def z_ba14(sig):
    """Normaliser of (1-E)^2 exp(-E/2sig^2) over the unit disk (closed form)."""
    c = 1.0 / (2.0 * sig * sig)
    return math.pi * (2 * sig**2 - 8 * sig**4 + 16 * sig**6 * (1.0 - math.exp(-c)))


def z_trunc_gauss(sig, e_max):
    return 2.0 * math.pi * sig * sig * (1.0 - math.exp(-e_max * e_max / (2.0 * sig * sig)))


def log_pe(E, sig, kind, e_max):
    """ln density of (e1, e2) as a function of E = |e|^2 (normalised)."""
    E = np.asarray(E, dtype=np.float64)
    if kind == E_KIND_BA14:
        out = np.full(E.shape, -np.inf)
        m = E < 1.0
        out[m] = 2.0 * np.log(1.0 - E[m]) - E[m] / (2 * sig * sig) - math.log(z_ba14(sig))
        return out
    out = np.full(E.shape, -np.inf)
    m = E < e_max * e_max
    out[m] = -E[m] / (2 * sig * sig) - math.log(z_trunc_gauss(sig, e_max))
    return out


def dlogZ_dsig(sig, kind, e_max):
    if kind == E_KIND_BA14:
        c = 1.0 / (2.0 * sig * sig)
        ex = math.exp(-c)
        f = 2 * sig**2 - 8 * sig**4 + 16 * sig**6 * (1.0 - ex)
        fp = 4 * sig - 32 * sig**3 + 96 * sig**5 * (1.0 - ex) - 16 * sig**3 * ex
        return fp / f
    c = e_max * e_max / (2.0 * sig * sig)
    ex = math.exp(-c)
    return 2.0 / sig - 2.0 * c * ex / (sig * (1.0 - ex))


def log_normal_log10(y, mu_ln, sig_ln):
    """ln density of log10 x when ln x ~ N(mu_ln, sig_ln)."""
    z = (y * LN10 - mu_ln) / sig_ln
    return math.log(LN10) - math.log(sig_ln) - 0.5 * math.log(2 * math.pi) - 0.5 * z * z


# ---- importance weights and the shear likelihood -------------------------------

def log_weights(e1p, e2p, l10s, l10f, g, alpha, tp: TruePrior, ip: Interim):
    """ln w_k for one galaxy's samples; g complex, alpha = (mu_ln_s, sig_ln_s, sigma_e)."""
    mu_s, sig_s, sig_e = alpha
    ep = np.asarray(e1p, np.float64) + 1j * np.asarray(e2p, np.float64)
    l10s = np.asarray(l10s, np.float64)
    l10f = np.asarray(l10f, np.float64)
    eps = shear_inverse(ep, g)
    E = np.abs(eps) ** 2
    Ep = np.abs(ep) ** 2
    lw = log_pe(E, sig_e, tp.e_kind, tp.e_max) + log_jacobian(ep, g)
    lw = lw - log_pe(Ep, ip.sigma_e, E_KIND_BA14, 1.0)
    if tp.size_term:
        lw = lw + log_normal_log10(l10s, mu_s, sig_s) + math.log(ip.log10s_hi - ip.log10s_lo)
    if not math.isnan(tp.mu_lnf):
        lw = lw + log_normal_log10(l10f, tp.mu_lnf, tp.sig_lnf) + math.log(ip.log10f_hi - ip.log10f_lo)
    return lw


def galaxy_loglike(e1p, e2p, l10s, l10f, g, alpha, tp, ip):
    """ell_n = ln sum_k w_k - ln K, max-subtracted."""
    lw = log_weights(e1p, e2p, l10s, l10f, g, alpha, tp, ip)
    mx = np.max(lw)
    if not np.isfinite(mx):
        return -math.inf
    return float(mx + math.log(np.sum(np.exp(lw - mx))) - math.log(lw.shape[0]))


def in_hyper_support(g, alpha):
    mu_s, sig_s, sig_e = alpha
    return (abs(g) < 1.0 and 1e-4 < sig_e < 1.0 and -2 * LN10 < mu_s < 2 * LN10
            and 0.0 < sig_s < 0.5 * LN10)


def log_posterior(S, g, alpha, tp, ip):
    """S = (e1p, e2p, l10s, l10f), each (G, K).  Returns ln P(g, alpha | d) + const."""
    if not in_hyper_support(g, alpha):
        return -math.inf
    e1p, e2p, l10s, l10f = S
    lw = log_weights(e1p, e2p, l10s, l10f, g, alpha, tp, ip)      # (G, K)
    mx = np.max(lw, axis=1)
    if not np.all(np.isfinite(mx)):
        return -math.inf
    ell = mx + np.log(np.sum(np.exp(lw - mx[:, None]), axis=1)) - math.log(lw.shape[1])
    return float(np.sum(ell))


def dlogw(e1p, e2p, l10s, g, alpha, tp: TruePrior):
    """d ln w_k / d(g1, g2, mu_ln_s, sig_ln_s, sigma_e), shape (5, K), closed form."""
    mu_s, sig_s, sig_e = alpha
    g1, g2 = g.real, g.imag
    e1p = np.asarray(e1p, np.float64)
    e2p = np.asarray(e2p, np.float64)
    ar, ai = e1p - g1, e2p - g2
    br = 1.0 - g1 * e1p - g2 * e2p
    bi = g2 * e1p - g1 * e2p
    A = ar * ar + ai * ai
    B = br * br + bi * bi
    E = A / B
    dA = np.stack([-2.0 * ar, -2.0 * ai])
    dB = np.stack([2.0 * (-br * e1p - bi * e2p), 2.0 * (-br * e2p + bi * e1p)])
    dE = (dA - E * dB) / B
    if tp.e_kind == E_KIND_BA14:
        dlp_dE = -2.0 / (1.0 - E) - 1.0 / (2 * sig_e * sig_e)
    else:
        dlp_dE = -1.0 / (2 * sig_e * sig_e) * np.ones_like(E)
    gg = g1 * g1 + g2 * g2
    dJ = np.stack([-4.0 * g1 / (1.0 - gg) - 2.0 * dB[0] / B,
                   -4.0 * g2 / (1.0 - gg) - 2.0 * dB[1] / B])
    out = np.empty((5,) + E.shape)
    out[0:2] = dlp_dE * dE + dJ
    if tp.size_term:
        z = (np.asarray(l10s, np.float64) * LN10 - mu_s) / sig_s
        out[2] = z / sig_s
        out[3] = -1.0 / sig_s + z * z / sig_s
    else:
        out[2:4] = 0.0
    out[4] = E / sig_e**3 - dlogZ_dsig(sig_e, tp.e_kind, tp.e_max)
    return out


def log_posterior_grad(S, g, alpha, tp, ip):
    """(ln P, d ln P / d(g1, g2, mu_ln_s, sig_ln_s, sigma_e)): softmax-weighted sums."""
    e1p, e2p, l10s, l10f = S
    tot = 0.0
    grad = np.zeros(5)
    for n in range(e1p.shape[0]):
        lw = log_weights(e1p[n], e2p[n], l10s[n], l10f[n], g, alpha, tp, ip)
        mx = np.max(lw)
        if not np.isfinite(mx):
            return -math.inf, np.full(5, np.nan)
        wk = np.exp(lw - mx)
        sw = np.sum(wk)
        tot += float(mx + math.log(sw) - math.log(lw.shape[0]))
        fin = np.isfinite(lw)
        d = dlogw(e1p[n][fin], e2p[n][fin], l10s[n][fin], g, alpha, tp)
        grad += d @ wk[fin] / sw
    if not in_hyper_support(g, alpha):
        return -math.inf, grad
    return tot, grad


def grid_posterior(S, g1s, g2s, alpha, tp, ip):
    """ln P on a (g1, g2) grid and the posterior mean of g."""
    lp = np.array([[log_posterior(S, complex(a, b), alpha, tp, ip) for a in g1s] for b in g2s])
    mx = np.max(lp)
    w = np.exp(lp - mx)
    G1, G2 = np.meshgrid(g1s, g2s)
    return lp, float(np.sum(w * G1) / np.sum(w)), float(np.sum(w * G2) / np.sum(w))


def hyper_potential(S, tp, ip):
    """Potential of the shear-level sampler (Section 3.4 samples P(g, alpha | d)):
    x = (g1, g2, mu_ln_s, sigma_ln_s, sigma_e) -> (U, grad U) with
    U = -ln P(g, alpha | d); outside the hyper-prior support U = +inf and the
    gradient is undefined (NaN): a trajectory that gets there is rejected.  Combined
    with ``hmc.run_chain`` (n_dim = 5) this is the oracle shear-level HMC."""
    def fn(x):
        g, alpha = complex(x[0], x[1]), (x[2], x[3], x[4])
        if not in_hyper_support(g, alpha):
            return math.inf, np.full(5, np.nan)
        lp, gr = log_posterior_grad(S, g, alpha, tp, ip)
        return -lp, -np.asarray(gr, dtype=np.float64)
    return fn
