"""Pins of the oracle sampler pieces: Philox known answers, the leapfrog as an
exact linear map on quadratic potentials, reversibility, energy-error order,
Gaussian-target moments, dual-averaging acceptance, ESS and R-hat (no GPU)."""
import math

import numpy as np
import pytest

from oracle import philox, hmc, diagnostics, prior, render


# Published known-answer vectors of Philox4x32-10 (Salmon et al., SC'11; the
# Random123 distribution's test vectors).
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(ctr, key, out):
    assert philox.philox4x32_10(ctr, key) == out


def test_uniform_mapping_exact_in_float32():
    for w in (0, 1, 255, 256, 0xFFFFFFFF, 0x80000000, 0x12345678):
        u = philox.uniform_from_word(w)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u


def test_momentum_normals_moments():
    z = np.array([philox.momentum_normals(123, uid, t) for uid in range(40) for t in range(100)])
    assert z.shape == (4000, 6)
    assert np.all(np.abs(z.mean(axis=0)) < 4 / math.sqrt(4000))
    assert np.all(np.abs(z.var(axis=0) - 1) < 0.1)
    c = np.corrcoef(z.T)
    assert np.max(np.abs(c - np.eye(6))) < 0.08


def _quadratic(A):
    return lambda th: (0.5 * float(th @ A @ th), A @ th)


def test_leapfrog_is_the_exact_linear_map_on_quadratics():
    w2 = np.array([0.5, 1.0, 2.0, 4.0, 9.0, 0.1])
    A = np.diag(w2)
    eps, L = 0.13, 7
    th0 = np.array([0.3, -1.0, 0.2, 0.5, -0.1, 2.0])
    p0 = np.array([1.0, 0.2, -0.4, 0.1, 0.3, -0.2])
    U0, g0 = _quadratic(A)(th0)
    th, p, *_ = hmc.leapfrog(_quadratic(A), th0, p0, g0, eps, L, np.ones(6))
    # per coordinate: one step is [[1 - e^2 w^2/2, e], [-e w^2 (1 - e^2 w^2/4), 1 - e^2 w^2/2]]
    for j in range(6):
        a = 1 - eps**2 * w2[j] / 2
        M = np.array([[a, eps], [-eps * w2[j] * (1 - eps**2 * w2[j] / 4), a]])
        v = np.linalg.matrix_power(M, L) @ np.array([th0[j], p0[j]])
        assert abs(v[0] - th[j]) < 1e-13 and abs(v[1] - p[j]) < 1e-13


def test_leapfrog_reversibility_and_energy_order():
    A = np.array([[2.0, 0.3], [0.3, 1.0]])
    f = _quadratic(A)
    th0, p0 = np.array([0.7, -0.4]), np.array([0.2, 0.9])
    U0, g0 = f(th0)
    th, p, U, g, _ = hmc.leapfrog(f, th0, p0, g0, 0.1, 25, np.ones(2))
    thb, pb, *_ = hmc.leapfrog(f, th, -p, g, 0.1, 25, np.ones(2))
    assert np.max(np.abs(thb - th0)) < 1e-12 and np.max(np.abs(-pb - p0)) < 1e-12
    errs = []
    for eps in (0.1, 0.05):
        L = int(round(2.0 / eps))
        th, p, U, g, _ = hmc.leapfrog(f, th0, p0, g0, eps, L, np.ones(2))
        errs.append(abs(U + 0.5 * p @ p - U0 - 0.5 * p0 @ p0))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_hmc_gaussian_target_moments_and_dual_averaging():
    rng = np.random.default_rng(0)
    B = rng.normal(size=(6, 6))
    cov = B @ B.T / 6 + 0.2 * np.eye(6)
    A = np.linalg.inv(cov)
    f = _quadratic(A)
    chains = []
    accs = []
    for c in range(4):
        r = hmc.run_chain(f, np.zeros(6), seed=99, uid=c, L=10, n_warmup=300, n_samples=1500,
                          eps0=0.05, adapt=True, jitter=0.3)
        chains.append(r["samples"])
        accs.append(r["alpha_warmup"][150:].mean())
        # the averaged step used after warmup accepts somewhat more often
        assert 0.75 < r["accept_rate"] < 0.95
    S = np.stack(chains)                    # (4, n, 6)
    # dual averaging drives the mean acceptance statistic during warmup to delta
    assert abs(np.mean(accs) - 0.8) < 0.05
    ess = diagnostics.ess_params(S)
    mean = S.reshape(-1, 6).mean(axis=0)
    for j in range(6):
        se = math.sqrt(cov[j, j] / ess[j])
        assert abs(mean[j]) < 4.5 * se
    emp = np.cov(S.reshape(-1, 6).T)
    assert np.max(np.abs(emp - cov) / np.sqrt(np.outer(np.diag(cov), np.diag(cov)))) < 0.15
    assert max(diagnostics.rhat(S[:, :, j]) for j in range(6)) < 1.02


def test_dual_averaging_recursion_values():
    # hand-evaluated first two updates of Hoffman & Gelman Alg. 5 with eps0 = 0.1
    da = hmc.DualAveraging(0.1)
    e1 = da.update(0.5)
    mu = math.log(1.0)
    hbar1 = (1 / 11) * (0.8 - 0.5)
    assert abs(math.log(e1) - (mu - 1 / 0.05 * hbar1)) < 1e-14
    e2 = da.update(1.0)
    hbar2 = (1 - 1 / 12) * hbar1 + (1 / 12) * (0.8 - 1.0)
    le2 = mu - math.sqrt(2) / 0.05 * hbar2
    assert abs(math.log(e2) - le2) < 1e-14
    x1, x2 = 1.0, 2 ** -0.75
    lbar = x2 * le2 + (1 - x2) * (x1 * math.log(e1))
    assert abs(math.log(da.final()) - lbar) < 1e-14


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9])
def test_ess_on_ar1(rho):
    rng = np.random.default_rng(int(rho * 10) + 1)
    M, n = 4, 20000
    x = np.empty((M, n))
    for m in range(M):
        e = rng.normal(size=n)
        x[m, 0] = e[0] / math.sqrt(1 - rho * rho)
        for t in range(1, n):
            x[m, t] = rho * x[m, t - 1] + e[t]
    want = M * n * (1 - rho) / (1 + rho)
    got = diagnostics.ess(x)
    assert abs(got / want - 1) < 0.12


def test_rhat_detects_unmixed_chains():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(4, 2000))
    assert diagnostics.rhat(x) < 1.01
    x[1] += 1.0
    assert diagnostics.rhat(x) > 1.1


def test_time_per_galaxy_formula():
    # Section 4.1 example magnitudes: 4000 chains, 1784 s total at 300 ESS
    t = diagnostics.time_per_galaxy(1040.0, 744.0, 4000, 300.0)
    assert abs(t - 1784.0 / 4000) < 1e-12


def test_galaxy_potential_gradient_matches_differences():
    N = 25
    p = np.array([300.0, 0.5, 0.2, -0.1, 0.1, -0.2])
    d = render.render_one(p, N, 0.2, 0.7) + np.random.default_rng(0).normal(0, 1, (N, N))
    gal = hmc.Galaxy(data=d, N=N, pixel_scale=0.2, psf_fwhm=0.7, sigma=1.0, ref_xy=(0.1, -0.2))
    th = np.array([math.log10(310.0), math.log10(0.52), 0.15, -0.05, 0.05, 0.02])
    U, gU = hmc.potential(gal, th)
    for j in range(6):
        e = np.zeros(6)
        e[j] = 1e-5
        fd = (hmc.potential(gal, th + e)[0] - hmc.potential(gal, th - e)[0]) / 2e-5
        assert abs(fd - gU[j]) < 1e-4 * (abs(gU[j]) + 10.0)
    assert math.isinf(hmc.potential(gal, np.array([2.0, 0.0, 0.8, 0.7, 0, 0]))[0])


def test_init_chain_rule():
    d = np.full((25, 25), 0.4)
    th = hmc.init_chain(d, 1.0, -0.2, (0.3, 0.1), seed=5, uid=3)
    assert abs(th[0] - math.log10(0.4 * 625)) < 1e-12
    assert abs(th[1] + 0.2) <= 0.015 and abs(th[2] - 0.3) <= 0.1 and abs(th[3] - 0.1) <= 0.1
    assert th[4] == 0 and th[5] == 0
    th = hmc.init_chain(-d, 1.0, -0.2, (0.9, 0.0), seed=5, uid=4)
    assert abs(th[0] - math.log10(25.0)) < 1e-12     # floor sigma * N
    assert th[2] ** 2 + th[3] ** 2 < 0.95 ** 2


def test_fisher_metric_matches_finite_difference_curvature():
    # at the true parameters of a noiseless stamp the likelihood Hessian equals
    # minus the Fisher information; check the diagonal by differences of U
    N = 25
    th = np.array([math.log10(400.0), math.log10(0.5), 0.2, -0.1, 0.1, -0.05])
    ref = (0.1, -0.2)
    prm = hmc.theta_to_params(th, ref)
    d = render.render_one(prm, N, 0.2, 0.7)
    gal = hmc.Galaxy(data=d, N=N, pixel_scale=0.2, psf_fwhm=0.7, sigma=1.0, ref_xy=ref)
    im = hmc.fisher_inv_mass(gal, th)
    for j in range(6):
        h = 1e-4
        e = np.zeros(6)
        e[j] = h
        curv = (hmc.potential(gal, th + e)[0] - 2 * hmc.potential(gal, th)[0] +
                hmc.potential(gal, th - e)[0]) / (h * h)
        assert abs(curv * im[j] - 1.0) < 2e-3, (j, curv, 1 / im[j])


def test_jittered_step_is_uniform_on_the_stated_interval():
    """Reading R8: the step of iteration t is eps (1 + j (2u - 1)) with u the
    Philox jitter uniform, i.e. uniform on [eps (1 - j), eps (1 + j)] (Neal
    2011, section 5.4.2.2: a step drawn at random from a small interval around
    the nominal one).  Pinned by its law, not by its formula: over 10^4
    (uid, t) pairs every value lies in the interval, a Kolmogorov-Smirnov test
    accepts the uniform law on it, and the mean and spread match the uniform
    ones.  A one-sided or mis-scaled jitter fails the KS test or the range."""
    from scipy import stats
    eps, j = 0.0137, 0.3
    e32 = hmc.f32(eps)
    lo, hi = e32 * (1.0 - hmc.f32(j)), e32 * (1.0 + hmc.f32(j))
    v = np.array([hmc.jittered_step(eps, j, 2024, uid, t) for uid in range(100) for t in range(100)])
    # float32 rounding of the product: half an ulp at each end
    assert np.all(v >= lo * (1 - 2 ** -24)) and np.all(v <= hi * (1 + 2 ** -24))
    ks = stats.kstest(v, stats.uniform(loc=lo, scale=hi - lo).cdf)
    assert ks.pvalue > 1e-3, ks
    n = v.size
    sd = (hi - lo) / math.sqrt(12.0)
    assert abs(v.mean() - e32) < 4.0 * sd / math.sqrt(n)
    assert abs(v.std() / sd - 1.0) < 0.05
    # both halves of the interval are used (a one-sided jitter puts nothing below eps)
    assert 0.45 < np.mean(v < e32) < 0.55
    # the values are distinct per (uid, t): the jitter stream is not shared across iterations
    assert np.unique(v).size > 0.99 * n


def test_jittered_step_without_jitter_is_the_float32_step():
    for eps in (0.01, 0.0137, 0.5, 1e-3):
        for t in range(5):
            assert hmc.jittered_step(eps, 0.0, 7, 3, t) == hmc.f32(eps)


@pytest.mark.parametrize("n", [40, 41])
def test_split_rhat_closed_form(n):
    """Split R-hat on draws built from an alternating pattern: each half-chain
    of length m = floor(n/2) is a level a_h plus (+1, -1, +1, ...), so every
    half-chain has the same sample variance v (m / (m - 1) for even m) and
    mean a_h + pattern mean; the statistic is then sqrt(((m - 1)/m v +
    var(means)) / v) exactly.  The levels rise within each chain (first half
    a, second half a + d), which the classic statistic over whole chains
    cannot see when every chain drifts alike."""
    M, d = 3, 1.0
    m = n // 2
    pat = np.array([(-1.0) ** k for k in range(m)])
    v = np.var(pat, ddof=1)                     # exact for the pattern
    if m % 2 == 0:
        assert abs(v - m / (m - 1.0)) < 1e-15
    base = np.array([0.1, -0.2, 0.3])
    x = np.empty((M, n))
    for c in range(M):
        x[c, :m] = base[c] + pat
        x[c, n - m:] = base[c] + d + pat
        if n % 2:
            x[c, m] = 1e6                       # the middle draw of an odd n is dropped
    levels = np.concatenate([base, base + d])
    pat_mean = pat.mean()
    want = math.sqrt(((m - 1.0) / m * v + np.var(levels + pat_mean, ddof=1)) / v)
    assert abs(diagnostics.split_rhat(x) - want) < 1e-12
    assert want > 1.05
    # the same drift in every chain leaves the classic statistic near 1 (n even)
    if n % 2 == 0:
        assert diagnostics.rhat(x) < diagnostics.split_rhat(x)


def test_split_rhat_on_iid_draws():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(4, 4000))
    assert abs(diagnostics.split_rhat(x) - 1.0) < 0.01
    x[:, 2000:] += 1.0                           # every chain shifts half way through
    assert diagnostics.rhat(x) < 1.05 and diagnostics.split_rhat(x) > 1.1
