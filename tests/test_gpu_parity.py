"""GPU parity: every C-ABI call against the FP64 oracle on seeded inputs.

Tolerances (fixed by the method's specification):
  stamps        max |m_gpu - m_oracle| <= 1e-5 of the stamp's peak
  log L         relative error <= 1e-6; for stamps below the 25-pixel minimum
                of the paper's workloads, where |log L| ~ N^2 / 2 is small,
                plus the float32 floor 4 eps32 |d| |d - m| / sigma^2 of spectra
                held in float32 (|.| the pixel 2-norms)
  gradient      |g_gpu - g_oracle| <= 1e-4 (|g_oracle| + sqrt(F_jj)), with
                F_jj = sigma^-2 sum_p (dm_p/dp_j)^2 the gradient's natural scale
  leapfrog      positions within 1e-4 under identical Philox momenta
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import render, hmc, diagnostics, shear          # noqa: E402
from workloads import gen                                    # noqa: E402
from tests import synth                                      # noqa: E402

PS = gen.PIXEL_SCALE


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bsi(device):
    from paper_2604_22048_amd import api
    return api


def _batch(api, torch, sizes, psf, sigma=None, profile=0, nu=0.5):
    G = len(sizes)
    sigma = np.ones(G) if sigma is None else sigma
    return api.Batch(n=np.asarray(sizes), psf_fwhm=torch.tensor(np.asarray(psf, np.float32)).cuda(),
                     sigma=torch.tensor(np.asarray(sigma, np.float32)).cuda(), pixel_scale=PS,
                     profile=profile, spergel_nu=nu)


# profile cases: (library kind, Spergel index, oracle profile).  Spergel at
# nu = -0.6 (near de Vaucouleurs) and 3 (near Gaussian), the ends of the
# model-bias scan of Appendix B.
PROFILES = {
    "exp": (0, 0.5, render.PROFILE_EXP),
    "gauss": (1, 0.5, render.PROFILE_GAUSS),
    "spergel-0.6": (2, -0.6, render.Spergel(-0.6)),
    "spergel3": (2, 3.0, render.Spergel(3.0)),
}


def _random_params(rng, G, sizes):
    p = np.empty((G, 6))
    p[:, 0] = rng.uniform(50, 2000, G)
    p[:, 1] = rng.uniform(0.25, 1.0, G)
    e = rng.uniform(0, 0.7, G)
    a = rng.uniform(0, np.pi, G)
    p[:, 2] = e * np.cos(2 * a)
    p[:, 3] = e * np.sin(2 * a)
    p[:, 4] = rng.uniform(-1.5, 1.5, G)
    p[:, 5] = rng.uniform(-1.5, 1.5, G)
    return p


@pytest.mark.parametrize("pname", list(PROFILES))
@pytest.mark.parametrize("transform", [1, 2])
def test_render_parity_ragged(bsi, pname, transform):
    """Both render transforms (float64 direct sums, FP32 MFMA products)."""
    import torch
    _log(f"render parity profile={pname} transform={transform}")
    kind, nu, profile = PROFILES[pname]
    rng = np.random.default_rng(10 + list(PROFILES).index(pname))
    sizes = [8, 9, 25, 32, 41, 53, 64, 73, 101, 128, 25, 53]
    G = len(sizes)
    params = _random_params(rng, G, sizes)
    psf = rng.uniform(0.6, 0.9, G)
    b = _batch(bsi, torch, sizes, psf, profile=kind, nu=nu)
    for N in set(sizes):
        bsi.set_transform(N, transform)
        assert bsi.get_transform(N) == transform
    out = bsi.render_stamps(b, torch.tensor(params, dtype=torch.float32).cuda()).cpu().numpy()
    for N in set(sizes):
        bsi.set_transform(N, 0)
    for i, N in enumerate(sizes):
        p32 = params[i].astype(np.float32).astype(np.float64)
        ref = render.render_one(p32, N, PS, float(np.float32(psf[i])), profile)
        got = out[b.off[i]:b.off[i] + N * N].reshape(N, N)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err <= 1e-5, (N, err)


def _grad_scale(p, N, psf, sigma, profile):
    _, dT = render.spectrum(p, N, PS, psf, profile, derivs=True)
    return np.array([math.sqrt(np.sum(render.synthesize(dT[j], N) ** 2)) / sigma for j in range(6)])


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("pname", list(PROFILES))
@pytest.mark.parametrize("transform", [1, 2])
def test_loglik_grad_parity(bsi, method, pname, transform):
    """Both likelihood methods, with the data (or residual) spectrum from
    either transform (direct sums, MFMA products)."""
    import torch
    _log(f"loglik parity method={method} profile={pname} transform={transform}")
    kind, nu, profile = PROFILES[pname]
    rng = np.random.default_rng(20 + method + 2 * list(PROFILES).index(pname))
    sizes = [8, 25, 32, 32, 41, 53, 73, 101, 128]
    G = len(sizes)
    truth = _random_params(rng, G, sizes)
    psf = rng.uniform(0.6, 0.9, G)
    sig = rng.uniform(0.5, 2.0, G)
    b = _batch(bsi, torch, sizes, psf, sig, kind, nu)
    data = np.zeros(b.n_pixels, np.float32)
    for i, N in enumerate(sizes):
        m = render.render_one(truth[i], N, PS, psf[i], profile) + rng.normal(0, sig[i], (N, N))
        data[b.off[i]:b.off[i] + N * N] = m.ravel()
    params = truth.copy()
    params[:, 0] *= rng.uniform(0.9, 1.1, G)
    params[:, 1] *= rng.uniform(0.9, 1.1, G)
    params[:, 2:4] += rng.uniform(-0.05, 0.05, (G, 2))
    params[:, 4:6] += rng.uniform(-0.2, 0.2, (G, 2))
    p32 = params.astype(np.float32).astype(np.float64)
    for N in set(sizes):
        bsi.set_transform(N, transform)
    ll, gr, st = bsi.loglik_grad(b, torch.tensor(data).cuda(),
                                 torch.tensor(p32, dtype=torch.float32).cuda(), method)
    for N in set(sizes):
        bsi.set_transform(N, 0)
    ll, gr, st = ll.cpu().numpy(), gr.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0)
    for i, N in enumerate(sizes):
        d = data[b.off[i]:b.off[i] + N * N].reshape(N, N).astype(np.float64)
        psf32 = float(np.float32(psf[i]))
        sig32 = float(np.float32(sig[i]))
        rll, rg = render.loglik_grad(d, p32[i], N, PS, psf32, sig32, profile)
        tol = 1e-6 * abs(rll)
        if N < 25:
            r = d - render.render_one(p32[i], N, PS, psf32, profile)
            tol += 4 * 2.0 ** -24 * np.linalg.norm(d) * np.linalg.norm(r) / sig32 ** 2
        assert abs(ll[i] - rll) <= tol, (N, ll[i], rll, tol)
        sc = _grad_scale(p32[i], N, psf32, sig32, profile)
        assert np.all(np.abs(gr[i] - rg) <= 1e-4 * (np.abs(rg) + sc)), (N, gr[i], rg, sc)


def test_loglik_edge_cases(bsi):
    import torch
    _log("loglik edge cases")
    b = _batch(bsi, torch, [], [])
    ll, gr, st = bsi.loglik_grad(b, torch.zeros(1).cuda(), torch.zeros(0, 6).cuda())
    assert ll.numel() == 0
    b = _batch(bsi, torch, [25, 25, 25], [0.7, 0.7, 0.7])
    p = torch.tensor([[100, 0.5, 0.8, 0.7, 0, 0], [100, -0.5, 0, 0, 0, 0], [100, 0.5, 0.1, 0, 0, 0]],
                     dtype=torch.float32).cuda()
    ll, gr, st = bsi.loglik_grad(b, torch.zeros(3 * 625).cuda(), p)
    st = st.cpu().numpy()
    assert st[0] & 1 and st[1] & 1 and st[2] == 0
    with pytest.raises(bsi.BsiError):
        bad = _batch(bsi, torch, [7], [0.7])
        bsi.loglik_grad(bad, torch.zeros(49).cuda(), torch.zeros(1, 6).cuda())
    with pytest.raises(bsi.BsiError):
        bad = _batch(bsi, torch, [129], [0.7])
        bsi.loglik_grad(bad, torch.zeros(129 * 129).cuda(), torch.zeros(1, 6).cuda())
    for nu in (-0.9, 4.5, float("nan")):       # Spergel index outside the accepted range
        with pytest.raises(bsi.BsiError):
            bad = _batch(bsi, torch, [25], [0.7], profile=2, nu=nu)
            bsi.loglik_grad(bad, torch.zeros(625).cuda(), torch.ones(1, 6).cuda())


def _hmc_setup(bsi, torch, cfg_name, n_gal, C, seed=3, sizes=None):
    t, params, data, off = synth.make_population(cfg_name, n_gal=n_gal, seed=seed, sizes=sizes)
    init = synth.init_positions(t, params, data, off, C, seed=seed + 1)
    b = _batch(bsi, torch, t.n_pix, t.psf_fwhm, t.sigma)
    ref = np.stack([t.dx, t.dy], axis=1)
    return t, params, data, off, init, b, ref


def _run_gpu(bsi, torch, b, data, ref, init, cfg, inv_mass=None):
    s, stats, st = bsi.hmc_sample(b, torch.tensor(data).cuda(),
                                  torch.tensor(ref, dtype=torch.float32).cuda(),
                                  torch.tensor(init, dtype=torch.float32).cuda(), cfg,
                                  inv_mass=inv_mass)
    torch.cuda.synchronize()
    return s.cpu().numpy(), stats.cpu().numpy(), st.cpu().numpy()


def _compare_chain(gpu, ora, tol=1e-4):
    """Samples agree to tol until the first accept/reject disagreement."""
    n_ok = 0
    for k in range(gpu.shape[0]):
        d = np.max(np.abs(gpu[k] - ora[k]))
        if d > tol:
            # a differing accept decision is only legitimate if the step moved
            moved_g = k == 0 or np.any(gpu[k] != gpu[k - 1])
            moved_o = k == 0 or np.any(ora[k] != ora[k - 1])
            assert moved_g != moved_o, (k, d, gpu[k], ora[k])
            break
        n_ok += 1
    return n_ok


@pytest.mark.parametrize("cfg_name,C,jitter", [("tiny", 1, 0.0), ("tiny", 2, 0.2), ("uniform", 2, 0.0)])
def test_hmc_fixed_step_parity(bsi, cfg_name, C, jitter):
    import torch
    _log(f"hmc fixed-step parity {cfg_name} C={C} jitter={jitter}")
    G = 3
    t, params, data, off, init, b, ref = _hmc_setup(bsi, torch, cfg_name, G, C)
    seed = 1234
    cfg = bsi.HmcConfig(n_chains=C, n_leapfrog=10, n_warmup=0, n_samples=6, adapt=False,
                        step_size=0.004, jitter=jitter, seed=seed, iters_per_launch=2)
    s, stats, st = _run_gpu(bsi, torch, b, data, ref, init, cfg)
    agree = 0
    for i in range(G):
        gal = synth.oracle_galaxy(t, data, off, i)
        for c in range(C):
            r = hmc.run_chain(hmc.galaxy_potential(gal), init[i, c].astype(np.float32), seed, i * C + c,
                              10, 0, 6, 0.004, adapt=False, jitter=jitter)
            agree += _compare_chain(s[i, c], r["samples"])
            # potential energy at the chain's final position (float32 sums vs float64)
            U, _ = hmc.potential(gal, s[i, c, -1].astype(np.float64))
            assert abs(stats[i, c, 3] - U) <= 1e-6 * abs(U), (stats[i, c, 3], U)
    assert agree >= G * C * 6 - 2


@pytest.mark.parametrize("nu", [-0.6, 3.0])
def test_hmc_spergel_fit_parity(bsi, nu):
    """The model-bias setting of Appendix B: exponential galaxies fitted with a
    Spergel profile of fixed index; chains follow the oracle's under the same
    Philox momenta (the general kernel, 25- and 53-pixel stamps)."""
    import torch
    _log(f"hmc Spergel fit parity nu={nu}")
    sizes = [25, 53, 25]
    G, C, S = len(sizes), 2, 5
    t, params, data, off = synth.make_population("uneven", n_gal=G, seed=41, sizes=sizes)
    init = synth.init_positions(t, params, data, off, C, seed=42)
    b = _batch(bsi, torch, t.n_pix, t.psf_fwhm, t.sigma, profile=2, nu=nu)
    ref = np.stack([t.dx, t.dy], axis=1)
    seed = 99
    cfg = bsi.HmcConfig(n_chains=C, n_leapfrog=10, n_warmup=0, n_samples=S, adapt=False,
                        step_size=0.004, jitter=0.1, seed=seed)
    s, stats, st = _run_gpu(bsi, torch, b, data, ref, init, cfg)
    prof = render.Spergel(nu)
    agree = 0
    for i in range(G):
        gal = synth.oracle_galaxy(t, data, off, i, prof)
        for c in range(C):
            r = hmc.run_chain(hmc.galaxy_potential(gal), init[i, c].astype(np.float32), seed, i * C + c,
                              10, 0, S, 0.004, adapt=False, jitter=0.1)
            agree += _compare_chain(s[i, c], r["samples"])
            U, _ = hmc.potential(gal, s[i, c, -1].astype(np.float64))
            assert abs(stats[i, c, 3] - U) <= 1e-6 * abs(U), (stats[i, c, 3], U)
    assert agree >= G * C * S - 2


@pytest.mark.parametrize("C,sizes", [(2, [25, 41, 53, 73, 101]), (4, [25, 41, 53, 73, 101, 41])])
def test_hmc_mixed_sizes_parity_and_invariance(bsi, C, sizes):
    """One batch of several stamp sizes: each chain follows the oracle under
    the same Philox momenta; graph replay (sizes in sequence) and direct
    launches (sizes on forked streams) agree bitwise; each galaxy's chains are bitwise
    those of the galaxy alone.  With two chains the 25-, 41- and 53-pixel
    galaxies run two chains per wave; with four, the 25-, 41- and 53-pixel
    ones run four per wave (16 lanes each, one wave per galaxy), and the
    others one wave per chain."""
    import torch
    _log(f"hmc mixed sizes {sizes} C={C}")
    G, S = len(sizes), 3
    t, params, data, off = synth.make_population("uneven", n_gal=G, seed=17, sizes=sizes)
    init = synth.init_positions(t, params, data, off, C, seed=18)
    b = _batch(bsi, torch, t.n_pix, t.psf_fwhm, t.sigma)
    ref = np.stack([t.dx, t.dy], axis=1)
    seed = 77
    base = dict(n_chains=C, n_leapfrog=8, n_warmup=0, n_samples=S, adapt=False, step_size=0.003,
                jitter=0.1, seed=seed)
    s, stats, st = _run_gpu(bsi, torch, b, data, ref, init, bsi.HmcConfig(**base))
    # graph replay and direct launches agree bitwise
    s_direct = _run_gpu(bsi, torch, b, data, ref, init, bsi.HmcConfig(use_graph=False, **base))[0]
    assert np.array_equal(s, s_direct)
    agree = 0
    for i in range(G):
        gal = synth.oracle_galaxy(t, data, off, i)
        for c in range(C):
            r = hmc.run_chain(hmc.galaxy_potential(gal), init[i, c].astype(np.float32), seed, i * C + c,
                              8, 0, S, 0.003, adapt=False, jitter=0.1)
            agree += _compare_chain(s[i, c], r["samples"])
        N = int(t.n_pix[i])
        b1 = _batch(bsi, torch, [N], t.psf_fwhm[i:i + 1], t.sigma[i:i + 1])
        alone = _run_gpu(bsi, torch, b1, data[off[i]:off[i] + N * N], ref[i:i + 1], init[i:i + 1],
                         bsi.HmcConfig(uid_base=i * C, **base))[0]
        assert np.array_equal(alone[0], s[i]), N
    assert agree >= G * C * S - 1


@pytest.mark.parametrize("workload,C,sizes", [("tiny", 2, None), ("uniform", 2, None),
                                               ("uneven", 4, [41, 25, 53])])
def test_hmc_dual_averaging_parity(bsi, workload, C, sizes):
    """Trajectories agree until the first accept/reject decision that float32
    and float64 potentials take differently; the step-size recursion is then
    checked exactly by replaying the GPU's own acceptance statistics.  The
    53-pixel case with two chains runs the two-chains-per-wave kernel, the
    25-, 41- and 53-pixel case with four chains the four-chains-per-wave
    kernel (trace included)."""
    import torch
    _log(f"hmc dual averaging parity {workload} C={C} sizes={sizes}")
    G, W, S = 3, 30, 4
    t, params, data, off, init, b, ref = _hmc_setup(bsi, torch, workload, G, C, seed=11, sizes=sizes)
    seed = 77
    # Fisher-diagonal metric: a well-conditioned trajectory (with the identity
    # metric the log-flux direction puts eps * omega near the leapfrog
    # stability limit, where float32 and float64 trajectories separate fast)
    cfg = bsi.HmcConfig(n_chains=C, n_leapfrog=10, n_warmup=W, n_samples=S, adapt=True,
                        step_size=0.3, jitter=0.1, seed=seed, iters_per_launch=4,
                        metric=bsi.N.METRIC_FISHER)
    tr = torch.zeros(G, C, W + S, 4, device="cuda")
    s, stats, st = bsi.hmc_sample(b, torch.tensor(data).cuda(),
                                  torch.tensor(ref, dtype=torch.float32).cuda(),
                                  torch.tensor(init, dtype=torch.float32).cuda(), cfg, trace=tr)
    tr = tr.cpu().numpy()
    stats = stats.cpu().numpy()
    agreed = 0
    for i in range(G):
        gal = synth.oracle_galaxy(t, data, off, i)
        for c in range(C):
            th0 = init[i, c].astype(np.float32).astype(np.float64)
            r = hmc.run_chain(hmc.galaxy_potential(gal), th0, seed, i * C + c, 10, W, S, 0.3,
                              adapt=True, jitter=0.1, inv_mass=hmc.fisher_inv_mass(gal, th0))
            ot = r["trace"]
            # strict agreement over the first iterations: afterwards dual averaging
            # feeds the float32-rounded dH back into the step, and the two runs
            # drift apart by design (checked below through the replay instead)
            for k in range(6):
                if tr[i, c, k, 3] != ot[k, 3]:
                    u = __import__("oracle").philox.accept_uniform(seed, i * C + c, k)
                    assert abs(-math.log(u) - tr[i, c, k, 1]) < 5e-3, (i, c, k, tr[i, c, k], ot[k])
                    break
                # the recursion's gain sqrt(m) / (gamma (m + t0)) ~ 3 times the
                # float32 rounding of dH (a few 1e-4) accumulates from step to step
                if k <= 2:
                    assert abs(tr[i, c, k, 0] / ot[k, 0] - 1) < 1e-3, (i, c, k, tr[i, c, k, 0], ot[k, 0])
                else:
                    assert abs(tr[i, c, k, 0] / ot[k, 0] - 1) < 2e-2, (i, c, k, tr[i, c, k, 0], ot[k, 0])
                # dH at an identical step (the first iteration) to float32 rounding;
                # later steps differ slightly, and dH with them
                if k == 0 and (np.isfinite(ot[k, 1]) or np.isfinite(tr[i, c, k, 1])):
                    assert abs(tr[i, c, k, 1] - ot[k, 1]) < 2e-3 * max(1.0, abs(ot[k, 1])), (i, c, k)
                agreed += 1
            assert 0.5 < stats[i, c, 1] / r["eps"] < 2.0
            # the step-size recursion on the GPU's own acceptance statistics
            da = hmc.DualAveraging(0.3)
            eps = 0.3
            # (the trace holds alpha rounded to float32, hence 1e-5 rather than bitwise)
            for k in range(W):
                assert abs(tr[i, c, k, 0] / eps - 1) < 1e-5, (i, c, k, tr[i, c, k, 0], eps)
                eps = da.update(float(tr[i, c, k, 2]))
                if k == W - 1:
                    eps = da.final()
            assert abs(stats[i, c, 1] / eps - 1) < 1e-5
    assert agreed >= G * C * 4


def test_hmc_fisher_metric_parity(bsi):
    import torch
    _log("hmc fisher metric parity")
    G, C = 2, 1
    t, params, data, off, init, b, ref = _hmc_setup(bsi, torch, "uniform", G, C, seed=5)
    seed = 99
    cfg = bsi.HmcConfig(n_chains=C, n_leapfrog=10, n_warmup=0, n_samples=4, adapt=False,
                        step_size=0.3, metric=bsi.N.METRIC_FISHER,
                        seed=seed, iters_per_launch=1)
    s, stats, st = _run_gpu(bsi, torch, b, data, ref, init, cfg)
    agree = 0
    for i in range(G):
        gal = synth.oracle_galaxy(t, data, off, i)
        th0 = init[i, 0].astype(np.float32).astype(np.float64)
        im = hmc.fisher_inv_mass(gal, th0)
        r = hmc.run_chain(hmc.galaxy_potential(gal), th0, seed, i, 10, 0, 4, 0.3, adapt=False,
                          inv_mass=im)
        agree += _compare_chain(s[i, 0], r["samples"], tol=2e-4)
    assert agree >= G * 4 - 1


@pytest.mark.parametrize("workload,C,sizes", [("tiny", 2, None), ("uneven", 4, [41, 53, 41, 25])])
def test_hmc_forms_and_batch_invariance_bitwise(bsi, workload, C, sizes):
    """Plain form (one galaxy and one leapfrog step per launch), one and three
    iterations per launch, graph and direct launches give the same chains
    bitwise, and a galaxy alone equals its slice of the batch (with four
    chains at 25, 41 and 53 pixels: the four-chains-per-wave kernel)."""
    import torch
    _log(f"hmc plain/batched/graph/batch-invariance {workload} C={C}")
    G = 4
    t, params, data, off, init, b, ref = _hmc_setup(bsi, torch, workload, G, C, seed=21, sizes=sizes)
    base = dict(n_chains=C, n_leapfrog=5, n_warmup=4, n_samples=5, adapt=True, step_size=0.005,
                jitter=0.1, seed=5)
    outs = []
    for form, ipl, graph in [(0, 1, True), (0, 1, False), (0, 3, True), (1, 1, False)]:
        cfg = bsi.HmcConfig(form=form, iters_per_launch=ipl, use_graph=graph, **base)
        outs.append(_run_gpu(bsi, torch, b, data, ref, init, cfg)[0])
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    # galaxy 2 alone, with its chain uids, equals its slice of the batch
    import torch as T
    b1 = _batch(bsi, T, t.n_pix[2:3], t.psf_fwhm[2:3], t.sigma[2:3])
    d1 = data[off[2]:off[2] + int(t.n_pix[2]) ** 2]
    cfg = bsi.HmcConfig(uid_base=2 * C, **base)
    alone = _run_gpu(bsi, T, b1, d1, ref[2:3], init[2:3], cfg)[0]
    assert np.array_equal(alone[0], outs[0][2])


def test_ess_rhat_parity(bsi):
    import torch
    _log("ess parity")
    rng = np.random.default_rng(8)
    G, C, S, P = 3, 4, 400, 6
    x = np.empty((G, C, S, P), np.float32)
    for g in range(G):
        for p in range(P):
            rho = [0.0, 0.3, 0.6, 0.9, -0.3, 0.95][p]
            for c in range(C):
                e = rng.normal(size=S)
                v = np.empty(S)
                v[0] = e[0]
                for k in range(1, S):
                    v[k] = rho * v[k - 1] + e[k]
                x[g, c, :, p] = v + 0.1 * c * (g == 2) + 0.8 * np.arange(S) / S * (g == 1)
    # galaxy 2's chains sit at different levels, galaxy 1's all drift alike (seen by the
    # split form only); S odd drops a middle draw in the split form
    for S_ in (S, S - 1):
        xs = np.ascontiguousarray(x[:, :, :S_])
        e, r, rs = bsi.ess(torch.tensor(xs).cuda(), split=True)
        e, r, rs = e.cpu().numpy(), r.cpu().numpy(), rs.cpu().numpy()
        for g in range(G):
            for p in range(P):
                xe = xs[g, :, :, p].astype(np.float64)
                assert abs(e[g, p] / diagnostics.ess(xe) - 1) < 1e-5, (g, p, e[g, p], diagnostics.ess(xe))
                assert abs(r[g, p] / diagnostics.rhat(xe) - 1) < 1e-6
                assert abs(rs[g, p] / diagnostics.split_rhat(xe) - 1) < 1e-6, (g, p, rs[g, p])


def _shear_samples(rng, G, K):
    e1 = rng.normal(0.02, 0.25, (G, K))
    e2 = rng.normal(0.0, 0.25, (G, K))
    r = np.hypot(e1, e2)
    e1 = np.where(r < 0.9, e1, e1 * 0.5)
    e2 = np.where(r < 0.9, e2, e2 * 0.5)
    ls = rng.normal(math.log10(0.6), 0.13, (G, K))
    lf = rng.normal(3.0, 0.2, (G, K))
    return [a.astype(np.float32) for a in (e1, e2, ls, lf)]


# Points at the edges of the hyper-prior boxes (reading R14: the paper's log10
# boxes mu_s in (-2, 2), sigma_s in (0, 0.5) converted to ln units;
# sigma_e in (1e-4, 1); |g| < 1): (g1, g2, mu, sigma, sigma_e, inside?).  Just
# inside the disk is |g| = 1 - 1e-3: closer to the circle the float32 inverse
# shear cannot resolve 1 - |eps|^2.
def _edge_points():
    L = math.log(10.0)
    b = (0.01, -0.02, math.log(0.6), 0.3, 0.25)
    pts = []
    for mu10 in (-2.0, 2.0):
        pts.append(((b[0], b[1], mu10 * (1 - 1e-9) * L, b[3], b[4]), True))
        pts.append(((b[0], b[1], mu10 * (1 + 1e-9) * L, b[3], b[4]), False))
    pts += [((b[0], b[1], b[2], 0.5 * (1 - 1e-9) * L, b[4]), True),
            ((b[0], b[1], b[2], 0.5 * (1 + 1e-9) * L, b[4]), False),
            ((b[0], b[1], b[2], 0.0, b[4]), False),
            ((b[0], b[1], b[2], b[3], 1e-4 * (1 + 1e-6)), True),
            ((b[0], b[1], b[2], b[3], 1e-4), False),
            ((b[0], b[1], b[2], b[3], 1.0 - 1e-9), True),
            ((b[0], b[1], b[2], b[3], 1.0), False),
            ((b[0], b[1], 1.3 * L, b[3], b[4]), True),
            ((b[0], b[1], b[2], 0.4 * L, b[4]), True)]
    for phi in (0.0, 2.5):
        c, s_ = math.cos(phi), math.sin(phi)
        pts += [(((1 - 1e-3) * c, (1 - 1e-3) * s_, *b[2:]), True), ((c, s_, *b[2:]), False),
                (((1 + 1e-9) * c, (1 + 1e-9) * s_, *b[2:]), False)]
    return pts


@pytest.mark.parametrize("kind,flux", [(1, False), (0, True)])
def test_shear_posterior_parity(bsi, kind, flux):
    """Log-posterior and gradient against the oracle within the float32 bound of
    tests/f32bound.py (derived from the library's float32 / float64 split),
    at interior points and at every edge of the hyper-prior boxes."""
    _shear_parity_case(bsi, kind, flux, 40, 300, 30 + kind)


@pytest.mark.parametrize("kind,K", [(0, 2500), (1, 1025), (1, 4000)])
def test_shear_posterior_many_samples(bsi, kind, K):
    """More samples per galaxy than a wave holds at once (K > 1024): the pass
    takes them in chunks of 512 and combines the chunks' float64 sums; the
    same oracle comparison, including the edge points whose weights force the
    fallback against the exact maximum.  K = 4000 is every draw of a
    galaxy's four chains in the benchmark's configuration."""
    _shear_parity_case(bsi, kind, True, 12, K, 60 + K)


@pytest.mark.parametrize("K", [700, 1000])
def test_shear_posterior_few_points(bsi, K):
    """At most 16 points (the shear-level sampler's chains) with more than
    512 samples per galaxy: the kernel form that takes samples in chunks of
    512 at three waves per SIMD.  Log-posterior and gradient against the
    oracle within the float32 bound."""
    _shear_parity_case(bsi, 1, False, 24, K, 90 + K, edges=False)


def _shear_parity_case(bsi, kind, flux, G, K, seed, edges=True):
    import torch
    from tests import f32bound
    _log(f"shear parity kind={kind} flux={flux} G={G} K={K}")
    rng = np.random.default_rng(seed)
    S = _shear_samples(rng, G, K)
    # e_max = 1 for the truncated Gaussian: its support is the unit disk, so the
    # disk edge of the shear prior can be probed with finite weights
    tpo = shear.TruePrior(e_kind=kind, e_max=1.0 if kind == 1 else 0.7,
                          mu_lnf=math.log(1000.0) if flux else math.nan, sig_lnf=0.5)
    tpg = bsi.TruePriorCfg(e_kind=kind, e_max=tpo.e_max, size_term=True, flux_term=flux,
                           mu_ln_f=math.log(1000.0), sigma_ln_f=0.5)
    inner = [((0.02, -0.01, math.log(0.6), 0.3, 0.2), True), ((-0.05, 0.04, -0.4, 0.25, 0.26), True),
             ((0.0, 0.0, -0.6, 0.35, 0.18), True), ((1.2, 0.0, -0.5, 0.3, 0.2), False)]
    cases = inner + (_edge_points() if edges else [])
    pts = np.array([c[0] for c in cases])
    St = [torch.tensor(a).cuda() for a in S]
    lp, gr = bsi.shear_posterior(St[0], St[1], St[2], St[3], pts, tpg, want_grad=True)
    lp, gr = lp.cpu().numpy(), gr.cpu().numpy()
    Sd = [a.astype(np.float64) for a in S]
    ip = shear.Interim()
    for j, (pt, inside) in enumerate(cases):
        if not inside:
            assert lp[j] == -np.inf, (j, pt, lp[j])
            continue
        g = complex(pt[0], pt[1])
        alpha = tuple(pt[2:])
        rl, rg = shear.log_posterior_grad(Sd, g, alpha, tpo, ip)
        tl, tg = f32bound.posterior_bounds(Sd, g, alpha, tpo, ip)
        assert np.isfinite(rl) and abs(lp[j] - rl) <= tl, (j, pt, lp[j], rl, tl)
        if j < len(inner):
            assert np.all(np.abs(gr[j] - rg) <= tg), (j, gr[j], rg, tg)


def test_shear_grid_posterior_mean(bsi):
    import torch
    _log("shear grid posterior mean")
    rng = np.random.default_rng(40)
    G, K = 16, 500
    S = _shear_samples(rng, G, K)
    g1s = np.linspace(-0.25, 0.25, 41)
    g2s = np.linspace(-0.25, 0.25, 41)
    alpha = (math.log(0.6), 0.3, 0.2)
    pts = np.array([[a, bb, *alpha] for bb in g2s for a in g1s])
    tpg = bsi.TruePriorCfg(e_kind=1, e_max=0.95)
    St = [torch.tensor(a).cuda() for a in S]
    lp = bsi.shear_posterior(St[0], St[1], St[2], St[3], pts, tpg).cpu().numpy().reshape(41, 41)
    rlp, m1, m2 = shear.grid_posterior([a.astype(np.float64) for a in S], g1s, g2s, alpha,
                                       shear.TruePrior(e_kind=1, e_max=0.95), shear.Interim())
    from tests import f32bound
    Sd = [a.astype(np.float64) for a in S]
    tp = shear.TruePrior(e_kind=1, e_max=0.95)
    tol = np.array([[f32bound.posterior_bounds(Sd, complex(a, bb), alpha, tp, shear.Interim(),
                                               want_grad=False)[0] for a in g1s] for bb in g2s])
    assert np.all(np.abs(lp - rlp) <= tol), np.max(np.abs(lp - rlp) / tol)
    # the grid mean moves by sum_p w_p (g_p - m)(d lp_p - mean d lp) to first order
    w = np.exp(lp - lp.max())
    w /= w.sum()
    G1, G2 = np.meshgrid(g1s, g2s)
    m1g, m2g = np.sum(w * G1), np.sum(w * G2)
    assert abs(m1g - m1) <= 2 * tol.max() * np.sum(w * np.abs(G1 - m1)), (m1g, m1)
    assert abs(m2g - m2) <= 2 * tol.max() * np.sum(w * np.abs(G2 - m2)), (m2g, m2)
