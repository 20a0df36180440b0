"""Oracle Hamiltonian Monte Carlo for the per-galaxy interim posterior (float64).

Test infrastructure only (see ``oracle/__init__``).

Target (eq. interim-post): P0(theta) * P(d | theta) with the pixel likelihood
eq. likelihood-pixels and the interim prior eq. interim-prior, in sampling
coordinates theta = (log10 F, log10 s, e1, e2, Dx, Dy).  Potential energy
U = -log L - log P0; kinetic energy p^T M^-1 p / 2 with a diagonal inverse
mass ``inv_mass`` (identity by default).  The paper uses NUTS with a
dual-averaging step-size warmup (Section 3.3); this is the fixed-length
Hamiltonian sampler (Neal 2011) with the same warmup (Hoffman & Gelman 2014,
Algorithm 5, Stan constants).

One iteration at global index t:
  1. p = z / sqrt(inv_mass), z from the Philox momentum stream of (chain, t);
  2. L leapfrog steps of size eps (half kick, L drifts with full kicks in
     between, final half kick), reusing the gradient at the start point;
  3. dH = H(end) - H(start) in float64; accept iff log(u) < -dH with u the
     Philox accept uniform of (chain, t); a trajectory that leaves the
     support or has a non-finite dH is rejected;
  4. during warmup, dual averaging on alpha = min(1, exp(-dH)) (0 when
     rejected for support or non-finiteness).
Optionally the step of iteration t is jittered, eps_t = eps (1 + j (2u - 1))
with u from the Philox jitter stream of (chain, t): Neal (2011, Section
5.4.2.2) randomises the step size so that a fixed trajectory length cannot
resonate with a period of the target.  The number of steps L stays fixed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import render, prior, philox

LN10 = math.log(10.0)
E_CLAMP = 1.0 - 1e-6
DIVERGENCE_DH = 1000.0


@dataclass
class Galaxy:
    data: np.ndarray          # (N, N) stamp
    N: int
    pixel_scale: float
    psf_fwhm: float
    sigma: float
    ref_xy: tuple = (0.0, 0.0)
    profile: object = render.PROFILE_EXP   # PROFILE_EXP, PROFILE_GAUSS or a render.Spergel


@dataclass
class Exposures:
    """One galaxy seen in several exposures (Appendix C): stamps of one side N,
    each with its PSF, noise sigma and (optionally) stationary noise power."""
    datas: list               # (N, N) stamps
    N: int
    pixel_scale: float
    psf_fwhm: list
    sigma: list
    noise_ps: list | None = None      # (N, N) DFT-mode noise powers in FFT order, or None (white)
    ref_xy: tuple = (0.0, 0.0)
    profile: object = render.PROFILE_EXP


def _loglik_grad(gal, prm):
    if isinstance(gal, Exposures):
        return render.loglik_grad_exposures(gal.datas, prm, gal.N, gal.pixel_scale, gal.psf_fwhm,
                                            gal.sigma, gal.noise_ps, gal.profile)
    return render.loglik_grad(gal.data, prm, gal.N, gal.pixel_scale, gal.psf_fwhm, gal.sigma,
                              gal.profile)


def clamp_theta(theta, ip=prior.PAPER_INTERIM):
    """Position used to evaluate the likelihood when theta is outside the support."""
    t = np.array(theta, dtype=np.float64)
    t[0] = min(max(t[0], ip["log10f_lo"]), ip["log10f_hi"])
    t[1] = min(max(t[1], ip["log10s_lo"]), ip["log10s_hi"])
    E = t[2] * t[2] + t[3] * t[3]
    if E > E_CLAMP:
        f = math.sqrt(E_CLAMP / E)
        t[2] *= f
        t[3] *= f
    return t


def theta_to_params(theta, ref_xy):
    return np.array([10.0 ** theta[0], 10.0 ** theta[1], theta[2], theta[3],
                     ref_xy[0] + theta[4], ref_xy[1] + theta[5]])


def potential(gal: Galaxy, theta, ip=prior.PAPER_INTERIM):
    """U(theta) (+inf outside the support) and grad U (finite everywhere)."""
    inside = prior.in_support(theta, ip)
    tc = clamp_theta(theta, ip)
    prm = theta_to_params(tc, gal.ref_xy)
    ll, g_p = _loglik_grad(gal, prm)
    g_theta = g_p.copy()
    g_theta[0] *= prm[0] * LN10
    g_theta[1] *= prm[1] * LN10
    gU = -(g_theta + prior.grad_log_prior(tc, ip))
    U = -(ll + prior.log_prior(tc, ip)) if inside else math.inf
    return U, gU


def kinetic(p, inv_mass):
    return 0.5 * float(np.sum(inv_mass * p * p))


def galaxy_potential(gal: Galaxy, ip=prior.PAPER_INTERIM):
    """Potential-energy function of one galaxy's interim posterior."""
    return lambda theta: potential(gal, theta, ip)


def leapfrog(potential_fn, theta, p, gU, eps, L, inv_mass, support_fn=None, trace=None):
    """L leapfrog steps; returns (theta, p, U, gradU, stayed_in_support)."""
    theta = np.array(theta, dtype=np.float64)
    p = np.array(p, dtype=np.float64) - 0.5 * eps * gU
    ok = True
    U = math.nan
    for step in range(1, L + 1):
        theta = theta + eps * inv_mass * p
        U, gU = potential_fn(theta)
        if support_fn is not None:
            ok = ok and support_fn(theta)
        else:
            ok = ok and math.isfinite(U)
        p = p - (eps if step < L else 0.5 * eps) * gU
        if trace is not None:
            trace.append(theta.copy())
    return theta, p, U, gU, ok


@dataclass
class DualAveraging:
    """Step-size adaptation (Hoffman & Gelman 2014, Algorithm 5; Stan constants)."""
    eps0: float
    delta: float = 0.8
    gamma: float = 0.05
    t0: float = 10.0
    kappa: float = 0.75
    m: int = 0
    hbar: float = 0.0
    log_eps_bar: float = 0.0
    log_eps: float = field(default=0.0)

    def __post_init__(self):
        self.mu = math.log(10.0 * self.eps0)
        self.log_eps = math.log(self.eps0)

    def update(self, alpha: float) -> float:
        self.m += 1
        eta = 1.0 / (self.m + self.t0)
        self.hbar = (1.0 - eta) * self.hbar + eta * (self.delta - alpha)
        self.log_eps = self.mu - math.sqrt(self.m) / self.gamma * self.hbar
        x = self.m ** (-self.kappa)
        self.log_eps_bar = x * self.log_eps + (1.0 - x) * self.log_eps_bar
        return math.exp(self.log_eps)

    def final(self) -> float:
        return math.exp(self.log_eps_bar)


def f32(x: float) -> float:
    """The step size is carried in float32 by the sampler; use the same value."""
    return float(np.float32(x))


def jittered_step(eps, jitter, seed, uid, t):
    """Step of iteration t: float32 eps and jitter, product formed in float64."""
    eps = f32(eps)
    if jitter <= 0.0:
        return eps
    u = philox.jitter_uniform(seed, uid, t)
    return f32(eps * (1.0 + f32(jitter) * (2.0 * u - 1.0)))


def hmc_iteration(potential_fn, theta, U, gU, eps, L, seed, uid, t, inv_mass, n_dim=6,
                  jitter=0.0):
    """One HMC transition.  Returns (theta, U, gU, info dict)."""
    eps = jittered_step(eps, jitter, seed, uid, t)
    z = philox.momentum_normals(seed, uid, t)[:n_dim]
    p0 = z / np.sqrt(inv_mass)
    H0 = U + kinetic(p0, inv_mass)
    th1, p1, U1, g1, ok = leapfrog(potential_fn, theta, p0, gU, eps, L, inv_mass)
    H1 = U1 + kinetic(p1, inv_mass)
    dH = H1 - H0
    u = philox.accept_uniform(seed, uid, t)
    finite = math.isfinite(dH)
    accept = ok and finite and math.log(u) < -dH
    alpha = min(1.0, math.exp(-dH)) if (ok and finite) else 0.0
    info = dict(dH=dH, accept=accept, alpha=alpha, in_support=ok,
                divergent=(not finite) or abs(dH) > DIVERGENCE_DH, theta_prop=th1, p_end=p1)
    if accept:
        return th1, U1, g1, info
    return np.array(theta, dtype=np.float64), U, gU, info


def run_chain(potential_fn, theta0, seed, uid, L, n_warmup, n_samples, eps0, adapt=True,
              inv_mass=None, jitter=0.0):
    """Warmup (dual averaging if adapt) then sampling; returns dict of arrays."""
    theta = np.array(theta0, dtype=np.float64)
    n_dim = theta.shape[0]
    inv_mass = np.ones(n_dim) if inv_mass is None else np.asarray(inv_mass, dtype=np.float64)
    U, gU = potential_fn(theta)
    da = DualAveraging(eps0)
    eps = eps0
    samples = np.empty((n_samples, n_dim))
    n_acc = 0
    n_div = 0
    alpha_sum = 0.0
    alpha_warm = []
    eps_hist = []
    trace = []
    for t in range(n_warmup + n_samples):
        eps_hist.append(f32(eps))
        theta, U, gU, info = hmc_iteration(potential_fn, theta, U, gU, eps, L, seed, uid, t,
                                           inv_mass, n_dim, jitter)
        n_div += int(info["divergent"])
        trace.append((f32(eps), info["dH"], info["alpha"], float(info["accept"])))
        if t < n_warmup:
            alpha_warm.append(info["alpha"])
            if adapt:
                eps = da.update(info["alpha"])
                if t == n_warmup - 1:
                    eps = da.final()
        else:
            samples[t - n_warmup] = theta
            n_acc += int(info["accept"])
            alpha_sum += info["alpha"]
    return dict(samples=samples, eps=f32(eps), accept_rate=n_acc / max(n_samples, 1),
                alpha_mean=alpha_sum / max(n_samples, 1), alpha_warmup=np.array(alpha_warm),
                trace=np.array(trace).reshape(-1, 4),
                n_div=n_div, U=U, eps_hist=np.array(eps_hist))


def init_chain(data, sigma, log10s_center, e_center, seed, uid, half_s=0.015, half_e=0.1,
               e_max=0.95, max_tries=64):
    """Chain start of eq. initialize.

    F = sum of the stamp (floored at sigma * N, since the sum can be <= 0 for
    faint galaxies); log10 s and (e1, e2) uniform in boxes around the given
    centres, redrawn until |e| < e_max; centroid offsets zero.  Jitter words
    come from the Philox init stream, counter (uid, attempt, tag 2, 0).
    """
    N = data.shape[0]
    F = max(float(np.sum(data, dtype=np.float64)), sigma * N)
    key = philox.seed_key(seed)
    for attempt in range(max_tries):
        w = philox.philox4x32_10((uid, attempt, philox.TAG_INIT, 0), key)
        u = [philox.uniform_from_word(x) for x in w[:3]]
        ls = log10s_center + (2.0 * u[0] - 1.0) * half_s
        e1 = e_center[0] + (2.0 * u[1] - 1.0) * half_e
        e2 = e_center[1] + (2.0 * u[2] - 1.0) * half_e
        if e1 * e1 + e2 * e2 < e_max * e_max:
            break
    else:
        e1, e2 = 0.0, 0.0
    return np.array([math.log10(F), ls, e1, e2, 0.0, 0.0])


def fisher_inv_mass(gal: Galaxy, theta, ip=prior.PAPER_INTERIM):
    """Inverse of the diagonal Fisher information of the likelihood plus the
    interim-prior curvature, in sampling coordinates (a diagonal metric).

    F_jj = sigma^-2 sum_pixels (dm/dtheta_j)^2, with each stamp derivative
    synthesised from the spectrum derivative (forward mode)."""
    tc = clamp_theta(theta, ip)
    prm = theta_to_params(tc, gal.ref_xy)
    jac = np.array([prm[0] * LN10, prm[1] * LN10, 1.0, 1.0, 1.0, 1.0])
    if isinstance(gal, Exposures):
        fi = render.fisher_diag_exposures(prm, gal.N, gal.pixel_scale, gal.psf_fwhm, gal.sigma,
                                          gal.noise_ps, gal.profile) * jac * jac
    else:
        _, dT = render.spectrum(prm, gal.N, gal.pixel_scale, gal.psf_fwhm, gal.profile, derivs=True)
        fi = np.array([np.sum(render.synthesize(dT[j], gal.N) ** 2) for j in range(6)])
        fi = fi * jac * jac / (gal.sigma * gal.sigma)
    e1, e2 = tc[2], tc[3]
    E = e1 * e1 + e2 * e2
    se, sd = ip["sigma_e"], ip["sigma_d"]
    fi[2] += 4.0 / (1 - E) + 8.0 * e1 * e1 / (1 - E) ** 2 + 1.0 / (se * se)
    fi[3] += 4.0 / (1 - E) + 8.0 * e2 * e2 / (1 - E) ** 2 + 1.0 / (se * se)
    fi[4] += 1.0 / (sd * sd)
    fi[5] += 1.0 / (sd * sd)
    return 1.0 / fi
