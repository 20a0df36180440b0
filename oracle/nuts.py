"""Oracle No-U-Turn sampler (the paper's sampler, Section 3.3: NUTS with
dual-averaging warmup and a maximum tree depth, 5 in the paper).

Test infrastructure only (see ``oracle/__init__``).

The transition (Hoffman and Gelman 2014, with the multinomial trajectory
sampling and the momentum-sum termination criterion of Betancourt 2017):

  draw p0 ~ N(0, M); H0 = U(theta) + p0' M^-1 p0 / 2; the trajectory is the
  single point theta.  For doubling d = 0, 1, ..., max_depth - 1: pick a
  direction v = +-1 uniformly; extend the trajectory by 2^d leapfrog steps of
  size v eps from its end in that direction (a new subtree); each new point
  x gets the weight w = exp(H0 - H(x)).
    * Within the subtree a candidate is kept by uniform progressive sampling:
      the n-th new point replaces it with probability w_n / (w_1 + ... + w_n).
    * The subtree is abandoned, and the transition ends with the proposal it
      had, as soon as a point has H - H0 > 1000 (divergence, also for a
      non-finite H) or any complete aligned block of 2^k points of the
      subtree (k >= 1, every node of its binary tree, the whole subtree
      included) makes a U-turn.
    * Otherwise the subtree's candidate replaces the proposal with probability
      min(1, W_sub / W_old) (biased progressive sampling), the weights add up,
      and the transition ends if the whole trajectory makes a U-turn.
  A span of points makes a U-turn when rho = sum of its momenta satisfies
  (M^-1 p_first) . rho <= 0 or (M^-1 p_last) . rho <= 0, p_first and p_last the
  momenta at its two ends.
  The warmup statistic is the mean of min(1, exp(H0 - H)) over every point
  computed in the transition (0 for divergent or non-finite ones).

Random numbers come from the Philox NUTS stream (``philox.nuts_*``): the
direction and merge uniform of doubling d, and the uniform of the n-th point
of the transition, so that any implementation drawing the same counters takes
the same decisions.
"""
from __future__ import annotations

import math

import numpy as np

from . import philox
from .hmc import DualAveraging, f32, kinetic

DIVERGENCE = 1000.0


def _turning(p_first, p_last, rho, inv_mass):
    return float(np.dot(inv_mass * p_first, rho)) <= 0.0 or float(np.dot(inv_mass * p_last, rho)) <= 0.0


def _logaddexp(a, b):
    if a == -math.inf:
        return b
    if b == -math.inf:
        return a
    m = max(a, b)
    return m + math.log(math.exp(a - m) + math.exp(b - m))


class Stream:
    """The transition's random numbers (the Philox NUTS stream)."""

    def __init__(self, seed, uid, t):
        self.seed, self.uid, self.t = seed, uid, t

    def direction(self, d):
        return philox.nuts_direction(self.seed, self.uid, self.t, d)

    def merge_uniform(self, d):
        return philox.nuts_merge_uniform(self.seed, self.uid, self.t, d)

    def leaf_uniform(self, n):
        return philox.nuts_leaf_uniform(self.seed, self.uid, self.t, n)


def nuts_iteration(potential_fn, theta, U, gU, eps, p0, inv_mass, max_depth, rand):
    """One NUTS transition from (theta, U, gU) with momentum p0.  Returns
    (theta, U, gU, info) with info: alpha (warmup statistic), n_leapfrog,
    depth (doublings completed), divergent, turning, leaves (every point, in
    trajectory order, for tests)."""
    theta = np.array(theta, dtype=np.float64)
    H0 = U + kinetic(p0, inv_mass)
    # ends of the trajectory: (theta, p, U, gU)
    left = right = (theta, np.array(p0, dtype=np.float64), U, np.array(gU, dtype=np.float64))
    prop = (theta, U, np.array(gU, dtype=np.float64))
    log_w = 0.0
    rho = np.array(p0, dtype=np.float64)
    sum_alpha, n_lf, n_leaf = 0.0, 0, 0
    divergent = turning = False
    depth = 0
    for d in range(max_depth):
        v = rand.direction(d)
        th, p, Ue, ge = right if v > 0 else left
        sub_logw = -math.inf
        sub_prop = None
        sub_p = []                      # the subtree's momenta in build order
        sub_turn = False
        for j in range(2 ** d):
            # one leapfrog step of size v eps
            ph = p - 0.5 * v * eps * ge
            th = th + v * eps * inv_mass * ph
            Ue, ge = potential_fn(th)
            p = ph - 0.5 * v * eps * ge
            H = Ue + kinetic(p, inv_mass)
            dH = H - H0
            n_lf += 1
            finite = math.isfinite(dH)
            sum_alpha += min(1.0, math.exp(-dH)) if finite else 0.0
            if not (finite and dH <= DIVERGENCE):
                divergent = True
                break
            lw = -dH
            new_logw = _logaddexp(sub_logw, lw)
            if math.log(rand.leaf_uniform(n_leaf)) < lw - new_logw:
                sub_prop = (th.copy(), Ue, ge.copy())
            sub_logw = new_logw
            n_leaf += 1
            sub_p.append(p.copy())
            # every complete aligned block ending at this point
            k = 1
            while (2 ** k) <= len(sub_p) and len(sub_p) % (2 ** k) == 0:
                blk = sub_p[len(sub_p) - 2 ** k:]
                if _turning(blk[0], blk[-1], np.sum(blk, axis=0), inv_mass):
                    sub_turn = True
                    break
                k += 1
            if sub_turn:
                break
        if divergent or sub_turn:
            turning = sub_turn
            break
        if math.log(rand.merge_uniform(d)) < sub_logw - log_w:
            prop = sub_prop
        log_w = _logaddexp(log_w, sub_logw)
        rho = rho + np.sum(sub_p, axis=0)
        end = (th, p, Ue, ge)
        if v > 0:
            right = end
        else:
            left = end
        depth = d + 1
        if _turning(left[1], right[1], rho, inv_mass):
            turning = True
            break
    info = dict(alpha=sum_alpha / max(n_lf, 1), n_leapfrog=n_lf, depth=depth, divergent=divergent,
                turning=turning)
    return prop[0], prop[1], prop[2], info


def run_chain_nuts(potential_fn, theta0, seed, uid, n_warmup, n_samples, eps0, max_depth=5,
                   adapt=True, inv_mass=None):
    """Warmup (dual averaging on the mean acceptance statistic) then sampling."""
    theta = np.array(theta0, dtype=np.float64)
    n_dim = theta.shape[0]
    inv_mass = np.ones(n_dim) if inv_mass is None else np.asarray(inv_mass, dtype=np.float64)
    U, gU = potential_fn(theta)
    da = DualAveraging(eps0)
    eps = eps0
    samples = np.empty((n_samples, n_dim))
    n_lf = np.empty(n_warmup + n_samples, dtype=np.int64)
    alphas = np.empty(n_warmup + n_samples)
    n_div = 0
    for t in range(n_warmup + n_samples):
        z = philox.momentum_normals(seed, uid, t)[:n_dim]
        p0 = z / np.sqrt(inv_mass)
        theta, U, gU, info = nuts_iteration(potential_fn, theta, U, gU, f32(eps), p0, inv_mass,
                                            max_depth, Stream(seed, uid, t))
        n_lf[t] = info["n_leapfrog"]
        alphas[t] = info["alpha"]
        n_div += int(info["divergent"])
        if t < n_warmup:
            if adapt:
                eps = da.update(info["alpha"])
                if t == n_warmup - 1:
                    eps = da.final()
        else:
            samples[t - n_warmup] = theta
    return dict(samples=samples, eps=f32(eps), n_leapfrog=n_lf, alpha=alphas, n_div=n_div, U=U)
