"""Pins of the oracle NUTS transition (Section 3.3's sampler): stationary
moments of a Gaussian target, termination depth against a brute-force scan of
every binary-tree node of the trajectory, and the multinomial proposal
distribution against its closed form."""
import math

import numpy as np
import pytest

from oracle import nuts
from oracle.hmc import kinetic


class FixedStream:
    """Directions from a list; uniforms from a numpy generator (or constant)."""

    def __init__(self, dirs, rng=None, u=0.5):
        self.dirs, self.rng, self.u = dirs, rng, u

    def direction(self, d):
        return self.dirs[d]

    def merge_uniform(self, d):
        return self.rng.uniform() if self.rng is not None else self.u

    def leaf_uniform(self, n):
        return self.rng.uniform() if self.rng is not None else self.u


def _quadratic(A):
    return lambda x: (0.5 * float(x @ A @ x), A @ x)


def test_gaussian_target_moments():
    cov = np.array([[1.0, 0.8], [0.8, 1.0]]) * np.array([[1.0, 0.5], [0.5, 0.25]]) * 4
    A = np.linalg.inv(cov)
    res = nuts.run_chain_nuts(_quadratic(A), np.array([1.0, -1.0]), 11, 3, 300, 4000, 0.5,
                              max_depth=6)
    s = res["samples"]
    assert np.all(np.abs(s.mean(axis=0)) < 0.12 * np.sqrt(np.diag(cov)))
    c = np.cov(s.T)
    assert np.all(np.abs(np.diag(c) / np.diag(cov) - 1) < 0.12)
    r = c[0, 1] / math.sqrt(c[0, 0] * c[1, 1])
    assert abs(r - 0.8) < 0.05
    assert res["n_div"] <= 5              # early warmup steps may diverge


def _trajectory(x0, p0, eps, n, sign, grad):
    """n leapfrog steps of size sign * eps: positions and momenta."""
    xs, ps = [], []
    x, p = x0.copy(), p0.copy()
    for _ in range(n):
        p = p - 0.5 * sign * eps * grad(x)
        x = x + sign * eps * p
        p = p - 0.5 * sign * eps * grad(x)
        xs.append(x.copy())
        ps.append(p.copy())
    return xs, ps


def _brute_depth(p0, fwd_p, bwd_p, dirs, max_depth):
    """Doublings completed and the stop reason, by checking every node of the
    binary tree: each subtree's aligned blocks (in its build order) and the
    whole trajectory after each merge (criterion on explicit sums)."""
    def turn(block):
        rho = np.sum(block, axis=0)
        return np.dot(block[0], rho) <= 0 or np.dot(block[-1], rho) <= 0
    nf = nb = 0
    traj = [p0]                          # momenta in time order
    for d in range(max_depth):
        size = 2 ** d
        if dirs[d] > 0:
            sub = fwd_p[nf:nf + size]
            nf += size
        else:
            sub = bwd_p[nb:nb + size]
            nb += size
        for k in range(1, d + 1):
            for start in range(0, size, 2 ** k):
                if turn(sub[start:start + 2 ** k]):
                    return d, True
        traj = traj + sub if dirs[d] > 0 else sub[::-1] + traj
        if turn(traj):
            return d + 1, True
    return max_depth, False


@pytest.mark.parametrize("dirs", [[1, 1, 1, 1, 1, 1], [1, -1, 1, -1, -1, 1], [-1, -1, 1, 1, -1, 1]])
@pytest.mark.parametrize("eps", [0.07, 0.21, 0.4])
def test_termination_depth_brute_force(dirs, eps):
    A = np.array([[1.0, 0.3], [0.3, 2.0]])
    pot = _quadratic(A)
    grad = lambda x: A @ x
    x0 = np.array([0.8, -0.4])
    p0 = np.array([0.3, 0.9])
    U, g = pot(x0)
    D = 6
    _, _, _, info = nuts.nuts_iteration(pot, x0, U, g, eps, p0, np.ones(2), D, FixedStream(dirs))
    _, fwd = _trajectory(x0, p0, eps, 2 ** D, 1, grad)
    _, bwd = _trajectory(x0, p0, eps, 2 ** D, -1, grad)
    depth, turned = _brute_depth(p0, fwd, bwd, dirs, D)
    assert (info["depth"], info["turning"]) == (depth, turned)


def test_multinomial_proposal_distribution():
    # forced forward doublings without a U-turn: the final proposal is leaf i of
    # subtree d with probability a_d w_i / W_d prod_{d' > d} (1 - a_d'), where
    # a_d = min(1, W_d / W_before) and the start point has weight 1
    A = np.array([[1.0]])
    pot = _quadratic(A)
    x0, p0 = np.array([0.1]), np.array([1.0])
    eps, D = 0.45, 2
    U, g = pot(x0)
    H0 = U + kinetic(p0, np.ones(1))
    xs, ps = _trajectory(x0, p0, eps, 2 ** D - 1, 1, lambda x: A @ x)
    w = np.array([math.exp(H0 - (pot(x)[0] + kinetic(p, np.ones(1)))) for x, p in zip(xs, ps)])
    probs = [1.0]
    W = 1.0
    n = 0
    for d in range(D):
        ws = w[n:n + 2 ** d]
        a = min(1.0, ws.sum() / W)
        probs = [q * (1 - a) for q in probs] + list(a * ws / ws.sum())
        W += ws.sum()
        n += 2 ** d
    rng = np.random.default_rng(7)
    counts = np.zeros(len(probs))
    n_run = 20000
    for _ in range(n_run):
        th, _, _, info = nuts.nuts_iteration(pot, x0, U, g, eps, p0, np.ones(1), D,
                                             FixedStream([1] * D, rng))
        assert not info["turning"] and info["depth"] == D
        idx = 0 if th[0] == x0[0] else 1 + int(np.argmin([abs(th[0] - x[0]) for x in xs]))
        counts[idx] += 1
    freq = counts / n_run
    sd = np.sqrt(np.array(probs) * (1 - np.array(probs)) / n_run)
    assert np.all(np.abs(freq - probs) < 4.5 * sd + 1e-12), (freq, probs)
