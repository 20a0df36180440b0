"""Synthetic workload generator: determinism, distributions, stored constants."""
import json
import math
import os

import numpy as np

from oracle import render, diagnostics
from workloads import gen

HERE = os.path.dirname(os.path.abspath(__file__))


def test_unit_flux_norm_matches_oracle_and_golden():
    g = json.load(open(os.path.join(HERE, "golden", "unit_flux_norm.json")))
    assert g["unit_flux_norm_median"] == gen.UNIT_FLUX_NORM_MEDIAN
    m = render.render_one([1.0, 0.6, 0, 0, 0, 0], 53, 0.2, 0.7)
    assert abs(math.sqrt(np.sum(m * m)) - gen.UNIT_FLUX_NORM_MEDIAN) < 1e-15
    assert abs(g["exponential_hlr_over_r0"] - gen.HLR_OVER_R0) < 1e-15


def test_paper_timing_consistent_with_extrapolation_formula():
    # Section 4.1 / 5.1: 0.26 s burn-in per galaxy + 0.6 ms per effective sample
    g = json.load(open(os.path.join(HERE, "golden", "paper_timing.json")))
    c = g["n_chains"]
    t = diagnostics.time_per_galaxy(g["burn_in_seconds_per_galaxy"] * c,
                                    g["ms_per_effective_sample"] * 1e-3 * c * 500, c, 500.0,
                                    g["target_ess"])
    assert abs(t - g["seconds_per_galaxy"]) < 0.015
    assert abs(g["total_seconds_4000_chains"] / c - g["seconds_per_galaxy"]) < 0.005


def test_draws_are_seeded_and_distributed():
    cfg = gen.CONFIGS["uniform"]
    a = gen.draw_truth(cfg, n_gal=20000)
    b = gen.draw_truth(cfg, n_gal=20000)
    assert np.array_equal(a.flux, b.flux) and np.array_equal(a.e1, b.e1)
    assert abs(np.median(a.hlr) - 0.6) < 0.01
    assert abs(np.std(np.log(a.hlr)) - 0.3) < 0.01
    assert np.all(a.e1 ** 2 + a.e2 ** 2 < 0.49)
    assert np.all(np.abs(a.dx) <= 0.5) and np.all(np.abs(a.dy) <= 0.5)
    lo, hi = 15 / gen.UNIT_FLUX_NORM_MEDIAN, 100 / gen.UNIT_FLUX_NORM_MEDIAN
    q = np.quantile(a.flux, [0.025, 0.975])
    assert abs(q[0] / lo - 1) < 0.05 and abs(q[1] / hi - 1) < 0.05
    assert np.all(a.n_pix == 53) and np.all(a.psf_fwhm == 0.7)


def test_uneven_size_mix_and_psf_range():
    cfg = gen.CONFIGS["uneven"]
    t = gen.draw_truth(cfg, n_gal=20000)
    assert set(np.unique(t.n_pix)) <= set(gen.SIZE_CLASSES)
    frac = {s: float(np.mean(t.n_pix == s)) for s in gen.SIZE_CLASSES}
    assert frac[25] + frac[41] > 0.6          # most galaxies need small stamps
    assert frac[101] < 0.05
    assert 0.6 <= t.psf_fwhm.min() and t.psf_fwhm.max() <= 0.9


def test_noise_layout():
    cfg = gen.CONFIGS["tiny"]
    t = gen.draw_truth(cfg)
    noise, off = gen.draw_noise(t, 5)
    assert noise.dtype == np.float32 and noise.shape == (16 * 32 * 32,)
    assert np.array_equal(off, np.arange(16) * 1024)
    assert abs(noise.std() - 1) < 0.05


def test_requests_poisson():
    t = gen.draw_requests(20000, 2000.0, 1)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 20000 - 1 / 2000.0) < 2e-5
