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
