"""GPU parity of the Appendix C likelihood extensions (stationary correlated
noise, several exposures per galaxy) against the FP64 oracle, which forms
each exposure's covariance explicitly.

Tolerances (the likelihood bar): log L relative error <= 1e-6; gradient
|g - g_oracle| <= 1e-4 (|g_oracle| + sqrt(F_jj)), F the oracle's summed
Fisher information; leapfrog positions within 1e-4 under identical momenta.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import hmc, render             # noqa: E402
from workloads import gen                  # noqa: E402
from tests import synth                    # noqa: E402

PS = gen.PIXEL_SCALE


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bsi(device):
    from paper_2604_22048_amd import api
    return api


def _upload(bsi, torch, n, psf, sig, ps, stamps, E):
    sizes = n.astype(np.int64) ** 2
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    data = np.concatenate([m.ravel() for m in stamps]).astype(np.float32)
    nps = None
    if ps[0] is not None:
        nps = torch.tensor(np.concatenate([q.ravel() for q in ps]).astype(np.float32)).cuda()
    b = bsi.Batch(n=n, psf_fwhm=torch.tensor(psf.astype(np.float32)).cuda(),
                  sigma=torch.tensor(sig.astype(np.float32)).cuda(), pixel_scale=PS, off=off,
                  n_exp=E, noise_ps=nps)
    return b, torch.tensor(data).cuda()


@pytest.mark.parametrize("E,corr", [(3, True), (1, True), (2, False)])
def test_loglik_exposures_parity(bsi, E, corr):
    import torch
    _log(f"exposures loglik parity E={E} correlated={corr}")
    rng = np.random.default_rng(80 + E)
    sizes = [25, 32, 41, 25]
    p, n, psf, sig, ps, stamps = synth.exposure_population(rng, sizes, E, corr)
    G = len(sizes)
    q = p.copy()
    q[:, 0] *= rng.uniform(0.9, 1.1, G)
    q[:, 1] *= rng.uniform(0.9, 1.1, G)
    q[:, 2:4] += rng.uniform(-0.05, 0.05, (G, 2))
    q[:, 4:6] += rng.uniform(-0.2, 0.2, (G, 2))
    q32 = q.astype(np.float32).astype(np.float64)
    b, data = _upload(bsi, torch, n, psf, sig, ps, stamps, E)
    ll, gr, st = bsi.loglik_grad(b, data, torch.tensor(q32, dtype=torch.float32).cuda(), 0)
    ll, gr, st = ll.cpu().numpy(), gr.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0)
    for i in range(G):
        sl = slice(i * E, (i + 1) * E)
        ds = [m.astype(np.float32).astype(np.float64) for m in stamps[sl]]
        f32 = [float(np.float32(x)) for x in psf[sl]]
        s32 = [float(np.float32(x)) for x in sig[sl]]
        pss = None if not corr else [x.astype(np.float32).astype(np.float64) for x in ps[sl]]
        N = int(n[i * E])
        rll, rg = render.loglik_grad_exposures(ds, q32[i], N, PS, f32, s32, pss)
        assert abs(ll[i] - rll) <= 1e-6 * abs(rll), (i, N, ll[i], rll)
        sc = np.sqrt(render.fisher_diag_exposures(q32[i], N, PS, f32, s32, pss))
        assert np.all(np.abs(gr[i] - rg) <= 1e-4 * (np.abs(rg) + sc)), (i, gr[i], rg, sc)
    with pytest.raises(bsi.BsiError):      # the pixel method has no weighted form
        bsi.loglik_grad(b, data, torch.tensor(q32, dtype=torch.float32).cuda(), 1)


def _compare_chain(gpu, ora, tol=1e-4):
    n_ok = 0
    for k in range(gpu.shape[0]):
        d = np.max(np.abs(gpu[k] - ora[k]))
        if d > tol:
            moved_g = k == 0 or np.any(gpu[k] != gpu[k - 1])
            moved_o = k == 0 or np.any(ora[k] != ora[k - 1])
            assert moved_g != moved_o, (k, d, gpu[k], ora[k])
            break
        n_ok += 1
    return n_ok


# (sizes, chains, exposures): the size-specialised kernels with two chains per
# wave (one exposure with correlated noise, 25 and 41 with C = 2) and one chain
# per wave (several exposures: 25 with C = 2; odd C: 32 and 41 with C = 3),
# and the general kernels (30 has no specialised kernel)
KERNEL_FORMS = [([25, 41], 2, 1), ([25, 25], 2, 2), ([32, 41], 3, 2), ([30, 30], 2, 2)]


@pytest.mark.parametrize("sizes,C,E", KERNEL_FORMS)
@pytest.mark.parametrize("metric", [0, 1])
def test_hmc_exposures_parity(bsi, metric, sizes, C, E):
    """Exposures with correlated noise per galaxy: chains follow the oracle's
    under the same Philox momenta (given metric and Fisher metric)."""
    import torch
    _log(f"exposures hmc parity metric={metric} sizes={sizes} C={C} E={E}")
    rng = np.random.default_rng(90 + metric + sizes[-1] + 7 * E)
    S = 4
    p, n, psf, sig, ps, stamps = synth.exposure_population(rng, sizes, E, True)
    G = len(sizes)
    b, data = _upload(bsi, torch, n, psf, sig, ps, stamps, E)
    ref = p[:, 4:6].copy()
    init = np.empty((G, C, 6))
    for i in range(G):
        for c in range(C):
            init[i, c] = [math.log10(p[i, 0]) + 0.01 * (c + 1), math.log10(p[i, 1]) - 0.01 * c,
                          p[i, 2] + 0.02 * c, p[i, 3] - 0.01, 0.05 * c, -0.05]
    step = 0.004 if metric == 0 else 0.3
    cfg = bsi.HmcConfig(n_chains=C, n_leapfrog=10, n_warmup=0, n_samples=S, adapt=False,
                        step_size=step, jitter=0.1, seed=123, metric=metric)
    s, stats, st = bsi.hmc_sample(b, data, torch.tensor(ref, dtype=torch.float32).cuda(),
                                  torch.tensor(init, dtype=torch.float32).cuda(), cfg)
    s = s.cpu().numpy()
    stats = stats.cpu().numpy()
    agree = 0
    for i in range(G):
        sl = slice(i * E, (i + 1) * E)
        gal = hmc.Exposures(datas=[m.astype(np.float32).astype(np.float64) for m in stamps[sl]],
                            N=int(n[i * E]), pixel_scale=PS,
                            psf_fwhm=[float(np.float32(x)) for x in psf[sl]],
                            sigma=[float(np.float32(x)) for x in sig[sl]],
                            noise_ps=[x.astype(np.float32).astype(np.float64) for x in ps[sl]],
                            ref_xy=(float(np.float32(ref[i, 0])), float(np.float32(ref[i, 1]))))
        for c in range(C):
            th0 = init[i, c].astype(np.float32).astype(np.float64)
            im = hmc.fisher_inv_mass(gal, th0) if metric == 1 else None
            r = hmc.run_chain(hmc.galaxy_potential(gal), th0, 123, i * C + c, 10, 0, S, step,
                              adapt=False, jitter=0.1, inv_mass=im)
            agree += _compare_chain(s[i, c], r["samples"], tol=1e-4 if metric == 0 else 2e-4)
            U, _ = hmc.potential(gal, s[i, c, -1].astype(np.float64))
            assert abs(stats[i, c, 3] - U) <= 1e-6 * abs(U), (stats[i, c, 3], U)
    assert agree >= G * C * S - 2


@pytest.mark.parametrize("sizes,C", [([25, 25], 2), ([30, 30], 2), ([53, 53], 4)])
def test_nuts_exposures_parity(bsi, sizes, C):
    """NUTS on galaxies seen in two exposures with correlated noise (the
    weighted form of the 25- and 53-pixel specialised kernels, the latter
    with four chains as in the exposures benchmark, and of the general
    kernels): chains follow the oracle's NUTS."""
    import torch
    from oracle import nuts
    _log(f"exposures nuts parity sizes={sizes} C={C}")
    rng = np.random.default_rng(95 + sizes[0])
    E, S = 2, 4
    p, n, psf, sig, ps, stamps = synth.exposure_population(rng, sizes, E, True)
    G = len(sizes)
    b, data = _upload(bsi, torch, n, psf, sig, ps, stamps, E)
    ref = p[:, 4:6].copy()
    init = np.empty((G, C, 6))
    for i in range(G):
        for c in range(C):
            init[i, c] = [math.log10(p[i, 0]) + 0.01 * (c + 1), math.log10(p[i, 1]) - 0.01 * c,
                          p[i, 2] + 0.02 * c, p[i, 3] - 0.01, 0.05 * c, -0.05]
    cfg = bsi.HmcConfig(n_chains=C, n_warmup=0, n_samples=S, adapt=False, step_size=0.3, seed=17,
                        metric=1, iters_per_launch=S, sampler=bsi.N.SAMPLER_NUTS, max_tree_depth=4)
    s, stats, st = bsi.hmc_sample(b, data, torch.tensor(ref, dtype=torch.float32).cuda(),
                                  torch.tensor(init, dtype=torch.float32).cuda(), cfg)
    s = s.cpu().numpy()
    agree = total = 0
    for i in range(G):
        sl = slice(i * E, (i + 1) * E)
        gal = hmc.Exposures(datas=[m.astype(np.float32).astype(np.float64) for m in stamps[sl]],
                            N=int(n[i * E]), pixel_scale=PS,
                            psf_fwhm=[float(np.float32(x)) for x in psf[sl]],
                            sigma=[float(np.float32(x)) for x in sig[sl]],
                            noise_ps=[x.astype(np.float32).astype(np.float64) for x in ps[sl]],
                            ref_xy=(float(np.float32(ref[i, 0])), float(np.float32(ref[i, 1]))))
        for c in range(C):
            th0 = init[i, c].astype(np.float32).astype(np.float64)
            r = nuts.run_chain_nuts(hmc.galaxy_potential(gal), th0, 17, i * C + c, 0, S, 0.3,
                                    max_depth=4, adapt=False, inv_mass=hmc.fisher_inv_mass(gal, th0))
            for k in range(S):
                total += 1
                if np.max(np.abs(s[i, c, k] - r["samples"][k])) > 2e-4:
                    break
                agree += 1
    assert agree >= total - 2, (agree, total)
