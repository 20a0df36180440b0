"""Pins of the m/c bias oracle (Section 3.5: shape-noise cancellation and
bootstrap errors) against closed forms and brute force."""
import math

import numpy as np

from oracle import bias, shear


def test_mc_recovers_planted_bias():
    # g_hat(+-g) = +-(1 + m) g + c exactly: the estimator returns m and c
    rng = np.random.default_rng(1)
    for _ in range(20):
        g1 = rng.uniform(0.005, 0.05)
        m, c1, c2 = rng.normal(0, 0.01, 3)
        gp = np.array([(1 + m) * g1 + c1, c2])
        gm = np.array([-(1 + m) * g1 + c1, c2])
        mh, ch = bias.mc_from_means(gp, gm, g1)
        assert abs(mh - m) < 1e-12 and abs(ch - c2) < 1e-15


def test_grid_mean_of_gaussian_loglikes_is_weighted_mean():
    # ell_n(g) = -|g - a_n|^2 / (2 s^2): the resample's posterior is Gaussian with
    # mean sum_n c_n a_n / sum_n c_n, which a fine grid reproduces to rounding
    rng = np.random.default_rng(2)
    G, B, s = 40, 7, 0.05
    a = rng.normal(0.01, 0.05, G) + 1j * rng.normal(-0.005, 0.05, G)
    g1 = np.linspace(-0.07, 0.09, 81)
    g2 = np.linspace(-0.085, 0.075, 81)
    G1, G2 = np.meshgrid(g1, g2)
    gpts = np.stack([G1.ravel(), G2.ravel()], axis=1)
    ell = -((gpts[:, :1] - a.real[None, :]) ** 2 + (gpts[:, 1:] - a.imag[None, :]) ** 2) / (2 * s * s)
    idx = rng.integers(0, G, (B, G))
    counts = bias.resample_counts(idx, G)
    assert np.all(counts.sum(axis=1) == G)
    got = bias.grid_mean(bias.resampled_logpost(ell, counts), gpts)
    want = np.stack([counts @ a.real, counts @ a.imag], axis=1) / G
    assert np.max(np.abs(got - want)) < 1e-12


def _exact_pairs(n, sig, emax, g1, seed):
    rng = np.random.default_rng(seed)
    e = rng.normal(0, sig, 3 * n) + 1j * rng.normal(0, sig, 3 * n)
    e = e[np.abs(e) < emax][:n]
    ls = np.full((n, 1), math.log10(0.6))
    out = []
    for g in (complex(g1, 0.0), complex(-g1, 0.0)):
        ep = shear.shear_forward(e, g)
        out.append((ep.real[:, None], ep.imag[:, None], ls, ls))
    return out


def test_bootstrap_equals_resampled_datasets_brute_force():
    # each resample's m and c from the resampled galaxy lists themselves, run
    # through the shear posterior on the grid, equal the count-weighted form
    n, sig, emax, g1 = 30, 0.2, 0.7, 0.02
    Sp, Sm = _exact_pairs(n, sig, emax, g1, 3)
    tp = shear.TruePrior(e_kind=1, e_max=emax, size_term=False)
    ip = shear.Interim()
    alpha = (math.log(0.6), 0.3, sig)
    g1s = np.linspace(-0.16, 0.16, 17)
    g2s = np.linspace(-0.15, 0.15, 15)
    G1, G2 = np.meshgrid(g1s, g2s)
    gpts = np.stack([G1.ravel(), G2.ravel()], axis=1)
    pts = np.array([[p[0], p[1], *alpha] for p in gpts])
    ell_p = bias.galaxy_loglikes(Sp, pts, tp, ip)
    ell_m = bias.galaxy_loglikes(Sm, pts, tp, ip)
    rng = np.random.default_rng(4)
    idx = rng.integers(0, n, (5, n))
    res = bias.mc_bootstrap(ell_p, ell_m, gpts, gpts, bias.resample_counts(idx, n), g1)
    for b in range(idx.shape[0]):
        means = []
        for S in (Sp, Sm):
            Sb = tuple(x[idx[b]] for x in S)
            _, m1, m2 = shear.grid_posterior(Sb, g1s, g2s, alpha, tp, ip)
            means.append((m1, m2))
        m, c = bias.mc_from_means(np.array(means[0]), np.array(means[1]), g1)
        assert abs(m - res["m_boot"][b]) < 1e-9 and abs(c - res["c_boot"][b]) < 1e-11
    # the quoted estimate uses every galaxy once
    _, p1, p2 = shear.grid_posterior(Sp, g1s, g2s, alpha, tp, ip)
    _, q1, q2 = shear.grid_posterior(Sm, g1s, g2s, alpha, tp, ip)
    m0, c0 = bias.mc_from_means(np.array([p1, p2]), np.array([q1, q2]), g1)
    assert abs(m0 - res["m"]) < 1e-9 and abs(c0 - res["c"]) < 1e-11
    assert abs(res["m_err"] - np.std(res["m_boot"])) == 0.0


def test_pairing_cancels_shape_noise():
    # exact ellipticities of 1500 galaxies: the +g dataset alone misses g by the
    # shape-noise mean (about sigma_e / sqrt(n) ~ 5e-3, a quarter of g); the
    # +-g combination cancels it in g1 to second order.  In g2 both datasets
    # carry the same shape-noise mean, so c is of order sigma_e / sqrt(n)
    n, sig, emax, g1 = 1500, 0.2, 0.7, 0.02
    Sp, Sm = _exact_pairs(n, sig, emax, g1, 5)
    tp = shear.TruePrior(e_kind=1, e_max=emax, size_term=False)
    ip = shear.Interim()
    alpha = (math.log(0.6), 0.3, sig)
    g1s = np.linspace(-0.04, 0.04, 41)
    g2s = np.linspace(-0.04, 0.04, 41)
    _, p1, p2 = shear.grid_posterior(Sp, g1s, g2s, alpha, tp, ip)
    g1s_m = -g1s[::-1]
    _, q1, q2 = shear.grid_posterior(Sm, g1s_m, g2s, alpha, tp, ip)
    m_single = p1 / g1 - 1.0
    m, c = bias.mc_from_means(np.array([p1, p2]), np.array([q1, q2]), g1)
    assert abs(m_single) > 0.05
    assert abs(m) < 0.2 * abs(m_single) and abs(m) < 0.02
    assert abs(c) < 3 * sig / math.sqrt(n)
    assert abs(c - 0.5 * (p2 + q2)) == 0.0
