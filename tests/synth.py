"""Test-side synthetic data: workload draws rendered by the oracle plus noise."""
from __future__ import annotations

import math

import numpy as np

from oracle import render, shear, hmc
from workloads import gen


def make_population(cfg_name="tiny", n_gal=None, seed=None, sizes=None, profile=render.PROFILE_EXP,
                    g=None):
    """Truth, lensed physical params [G,6], packed float32 data, offsets."""
    cfg = gen.CONFIGS[cfg_name]
    t = gen.draw_truth(cfg, n_gal=n_gal, seed=seed, size_override=sizes)
    gg = complex(*(cfg.g_true if g is None else g))
    ep = shear.shear_forward(t.e1 + 1j * t.e2, gg)
    params = np.stack([t.flux, t.hlr, ep.real, ep.imag, t.dx, t.dy], axis=1)
    noise, off = gen.draw_noise(t, (seed if seed is not None else gen.data_seed(cfg.index)) + 7)
    data = np.empty_like(noise)
    for i in range(len(t)):
        N = int(t.n_pix[i])
        m = render.render_one(params[i], N, gen.PIXEL_SCALE, t.psf_fwhm[i], profile)
        data[off[i]:off[i] + N * N] = (m.ravel() + noise[off[i]:off[i] + N * N]).astype(np.float32)
    return t, params, data, off


def stamp(data, off, n, i):
    N = int(n[i])
    return data[off[i]:off[i] + N * N].reshape(N, N).astype(np.float64)


def oracle_galaxy(t, data, off, i, profile=render.PROFILE_EXP):
    """oracle.hmc.Galaxy for galaxy i with its true centroid as reference."""
    return hmc.Galaxy(data=stamp(data, off, t.n_pix, i), N=int(t.n_pix[i]),
                      pixel_scale=gen.PIXEL_SCALE, psf_fwhm=float(t.psf_fwhm[i]),
                      sigma=float(t.sigma[i]), ref_xy=(float(t.dx[i]), float(t.dy[i])),
                      profile=profile)


def init_positions(t, params, data, off, C, seed):
    """Chain starts of eq. initialize for every galaxy and chain: [G, C, 6]."""
    G = len(t)
    out = np.empty((G, C, 6))
    for i in range(G):
        d = stamp(data, off, t.n_pix, i)
        es = (params[i, 2], params[i, 3])
        for c in range(C):
            out[i, c] = hmc.init_chain(d, float(t.sigma[i]), math.log10(params[i, 1]), es, seed,
                                       i * C + c)
    return out


def interim_population(G, K, seed, g=(0.02, 0.0), sig_e=0.2, e_max=0.7, mu_ln_s=math.log(0.6),
                       sig_ln_s=0.3, noise_e=0.05, noise_ln_s=0.05):
    """Stand-in interim samples with a population behind them: galaxy n has an
    intrinsic ellipticity from a circular Gaussian truncated at e_max, lensed
    by g with the oracle's shear map, and a lognormal size; its K samples
    scatter around those with measurement-like noise (ellipticities kept
    inside |e| < 0.95).  Returns float32 (e1', e2', log10 s, log10 F), each
    [G, K]."""
    rng = np.random.default_rng(seed)
    e = np.empty(0, complex)
    while e.size < G:
        z = rng.normal(0, sig_e, 2 * G) + 1j * rng.normal(0, sig_e, 2 * G)
        e = np.concatenate([e, z[np.abs(z) < e_max]])
    ep = shear.shear_forward(e[:G], complex(*g))
    ln_s = rng.normal(mu_ln_s, sig_ln_s, G)
    smp = ep[:, None] + rng.normal(0, noise_e, (G, K)) + 1j * rng.normal(0, noise_e, (G, K))
    r = np.abs(smp)
    smp = np.where(r < 0.95, smp, smp * 0.9 / np.maximum(r, 1e-12))
    l10s = (ln_s[:, None] + rng.normal(0, noise_ln_s, (G, K))) / math.log(10.0)
    l10f = rng.normal(3.0, 0.1, (G, K))
    return [a.astype(np.float32) for a in (smp.real, smp.imag, l10s, l10f)]


noise_kernel_ps = gen.noise_kernel_ps
correlated_noise = gen.correlated_noise


def exposure_population(rng, sizes, E, correlated=True):
    """Galaxies (params [G, 6]) seen in E exposures each: per stamp (galaxy-major)
    side, PSF FWHM, sigma, noise powers (or None) and the data stamps."""
    G = len(sizes)
    p = np.empty((G, 6))
    p[:, 0] = rng.uniform(200, 2000, G)
    p[:, 1] = rng.uniform(0.3, 0.9, G)
    e = rng.uniform(0, 0.6, G)
    a = rng.uniform(0, np.pi, G)
    p[:, 2] = e * np.cos(2 * a)
    p[:, 3] = e * np.sin(2 * a)
    p[:, 4] = rng.uniform(-1.0, 1.0, G)
    p[:, 5] = rng.uniform(-1.0, 1.0, G)
    n = np.repeat(np.asarray(sizes), E)
    psf = rng.uniform(0.6, 0.9, G * E)
    sig = rng.uniform(0.7, 1.5, G * E)
    ps, stamps = [], []
    for s in range(G * E):
        N = int(n[s])
        m = render.render_one(p[s // E], N, gen.PIXEL_SCALE, float(np.float32(psf[s])))
        if correlated:
            q, kap = noise_kernel_ps(rng, N)
            ps.append(q)
            stamps.append(m + correlated_noise(rng, kap, sig[s]))
        else:
            ps.append(None)
            stamps.append(m + rng.normal(0, sig[s], (N, N)))
    return p, n, psf, sig, ps, stamps
