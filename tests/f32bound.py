"""Float32 error bounds for the shear-phase parity tests.

The library evaluates each importance weight w_nk (eq.
true-prior-jacobian-shear over the interim prior) in float32, as
x = 2^(lw2 - U) with lw2 = ln w / ln 2 and U a wave-uniform bound >= lw2
(the Jacobian's 1/B^2 applied as a product rather than through a
logarithm), and everything after it (the log-sum-exp over k, the sum over
galaxies, the gradient assembly) in float64, except the per-lane partial
sums of at most 16 terms x in float32 (reading R17).  These bounds are
derived from that split with the float32 unit roundoff u = 2^-24, using the
oracle's float64 functions only; nothing here depends on the library.

Per sample, a float32 evaluation of ln w = sum_i t_i (the ellipticity
density, the shear Jacobian, minus the interim density, the size and flux
terms) carries an absolute error at most c u M with

    M = sum_i |t_i| + sum_x |x d ln w / dx|,

the first sum covering the rounding of each term and of their sum, the
second the rounding of every intermediate computed from an input x (the
sample's e1', e2', log10 s, log10 F and the point's g1, g2, mu, sigma,
sigma_e), which is equivalent to a relative perturbation of x of a few u.
c = 16 covers the longest chain of float32 operations (the inverse shear map,
|.|^2, a reciprocal, a hardware logarithm, the quadratic size term), each
hardware transcendental counted at 2 u.

Per galaxy, with s_k the softmax weights, ln sum_k w_k - ln K moves by
sum_k s_k d ln w_k to first order, plus the float32 partial sums (relative
error <= 16 u, so <= 16 u absolute after the logarithm, twice for the
rescaling):

    |d ell_n| <= c u sum_k s_k M_nk + 32 u,

and the log-posterior bound is the sum over galaxies.  For a gradient
component with d_k = d ln w_k / d theta and mean dbar = sum_k s_k d_k, the
weights move it by sum_k s_k d ln w_k (d_k - dbar) to first order, and the
float32 derivative terms by at most c u sum_k s_k D_k,

    |d grad_n| <= c u sum_k s_k M_nk |d_k - dbar| + c u sum_k s_k D_k + 32 u C,
    D_k = |d_k| + sum_x |x d d_k / dx| + C,

C the magnitude of the point's constant part subtracted in float64 (the
Jacobian's |g| derivative, 1/sigma, d ln Z / d sigma_e).  Derivatives with
respect to the inputs are central differences of the oracle's own functions
(relative step 1e-6; they set a tolerance, not a value under test).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import shear

U32 = 2.0 ** -24
C_OPS = 16.0


def _terms(e1p, e2p, l10s, l10f, g, alpha, tp, ip):
    """The summands of ln w (oracle functions), each an array over the samples."""
    mu_s, sig_s, sig_e = alpha
    ep = np.asarray(e1p, np.float64) + 1j * np.asarray(e2p, np.float64)
    E = np.abs(shear.shear_inverse(ep, g)) ** 2
    Ep = np.abs(ep) ** 2
    out = [shear.log_pe(E, sig_e, tp.e_kind, tp.e_max),
           shear.log_jacobian(ep, g) + 0.0 * E,
           -shear.log_pe(Ep, ip.sigma_e, shear.E_KIND_BA14, 1.0)]
    if tp.size_term:
        out.append(shear.log_normal_log10(np.asarray(l10s, np.float64), mu_s, sig_s))
        out.append(np.full(E.shape, math.log(ip.log10s_hi - ip.log10s_lo)))
    if not math.isnan(tp.mu_lnf):
        out.append(shear.log_normal_log10(np.asarray(l10f, np.float64), tp.mu_lnf, tp.sig_lnf))
        out.append(np.full(E.shape, math.log(ip.log10f_hi - ip.log10f_lo)))
    return out


def _inputs(e1p, e2p, l10s, l10f, g, alpha):
    return [np.asarray(e1p, np.float64), np.asarray(e2p, np.float64), np.asarray(l10s, np.float64),
            np.asarray(l10f, np.float64), g.real, g.imag, alpha[0], alpha[1], alpha[2]]


def _call(f, xs):
    e1p, e2p, l10s, l10f, g1, g2, mu, sg, se = xs
    return f(e1p, e2p, l10s, l10f, complex(g1, g2), (mu, sg, se))


def _sensitivity(f, xs, h=1e-6):
    """sum_x |x df/dx| by central differences in each input (arrays broadcast)."""
    tot = 0.0
    for j, x in enumerate(xs):
        step = h * np.maximum(np.abs(x), 1e-12)
        lo, hi = list(xs), list(xs)
        lo[j], hi[j] = x - step, x + step
        fl, fh = _call(f, lo), _call(f, hi)
        with np.errstate(invalid="ignore"):
            d = np.where(np.isfinite(fl) & np.isfinite(fh), (fh - fl) / (2.0 * step), 0.0)
        tot = tot + np.nan_to_num(np.abs(x * d))
    return tot


def _point_constants(g, alpha, tp):
    """Magnitudes of the sample-independent parts of d ln w / d theta."""
    mu_s, sig_s, sig_e = alpha
    h = 1e-7
    cg = [abs((shear.log_jacobian(0.0, g + h) - shear.log_jacobian(0.0, g - h)) / (2 * h)),
          abs((shear.log_jacobian(0.0, g + 1j * h) - shear.log_jacobian(0.0, g - 1j * h)) / (2 * h))]
    return np.array([cg[0], cg[1], 0.0, 1.0 / sig_s if tp.size_term else 0.0,
                     abs(shear.dlogZ_dsig(sig_e, tp.e_kind, tp.e_max))])


def galaxy_bounds(e1p, e2p, l10s, l10f, g, alpha, tp, ip, want_grad=True):
    """Per-galaxy bounds for samples shaped (G, K) (or (K,)): (bound on
    |d ell_n| (G,), bound on |d grad ell_n| (G, 5)).  A galaxy with no finite
    weight has ell_n = -inf on both sides and bound 0."""
    xs = _inputs(*(np.atleast_2d(np.asarray(a, np.float64)) for a in (e1p, e2p, l10s, l10f)), g, alpha)
    lwf = lambda a, b, c, d, gg, al: shear.log_weights(a, b, c, d, gg, al, tp, ip)
    lw = lwf(*xs[:4], g, alpha)
    fin = np.isfinite(lw)
    M = sum(np.abs(np.where(fin, t, 0.0)) for t in _terms(*xs[:4], g, alpha, tp, ip))
    M = np.where(fin, M + _sensitivity(lwf, xs), 0.0)
    mx = np.max(np.where(fin, lw, -np.inf), axis=-1, keepdims=True)
    mx = np.where(np.isfinite(mx), mx, 0.0)
    s = np.where(fin, np.exp(np.where(fin, lw, 0.0) - mx), 0.0)
    sn = s.sum(axis=-1, keepdims=True)
    any_fin = sn[:, 0] > 0
    s = s / np.where(sn > 0, sn, 1.0)
    tol_ell = np.where(any_fin, C_OPS * U32 * np.sum(s * M, axis=-1) + 32.0 * U32, 0.0)
    tol_g = np.zeros((lw.shape[0], 5))
    if not want_grad:
        return tol_ell, tol_g
    with np.errstate(invalid="ignore", divide="ignore"):
        d = np.where(fin, shear.dlogw(xs[0], xs[1], xs[2], g, alpha, tp), 0.0)   # (5, G, K)
    Cp = _point_constants(g, alpha, tp)
    for j in range(5):
        dj = lambda a, b, c, dd, gg, al, j=j: shear.dlogw(a, b, c, gg, al, tp)[j]
        with np.errstate(invalid="ignore", divide="ignore"):
            D = np.where(fin, np.abs(d[j]) + _sensitivity(dj, xs) + Cp[j], 0.0)
        dbar = np.sum(s * d[j], axis=-1, keepdims=True)
        tol_g[:, j] = np.where(any_fin, C_OPS * U32 * (np.sum(s * M * np.abs(d[j] - dbar), axis=-1)
                                                        + np.sum(s * D, axis=-1)) + 32.0 * U32 * Cp[j], 0.0)
    return tol_ell, tol_g


def posterior_bounds(S, g, alpha, tp, ip, want_grad=True):
    """Bounds on the float32-induced error of ln P(g, alpha | d) and its gradient:
    sums of the per-galaxy bounds (the galaxy sum itself is float64)."""
    tl, tg = galaxy_bounds(*S, g, alpha, tp, ip, want_grad)
    return float(np.sum(tl)), np.sum(tg, axis=0)
