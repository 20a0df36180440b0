"""Slot plans: every plan with a specialised trajectory kernel (and a generic
one) keeps log L, gradient and chains at oracle parity; the autotuner
returns valid plans and the library works with them."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import hmc, render                              # noqa: E402
from workloads import gen                                    # noqa: E402
from tests import synth                                      # noqa: E402

PS = gen.PIXEL_SCALE
# every plan with a specialised kernel (the ones the autotuner chooses among),
# plus one plan per size that runs the generic kernel
PLANS = {25: (3, 1), 32: (1, 2, 4), 41: (1, 4), 53: (3, 4, 6, 2), 73: (3, 6, 8), 101: (4, 5)}


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bsi(device):
    from paper_2604_22048_amd import api
    yield api
    for n in range(8, 129):
        api.set_plan(n, 0)


def _setup(bsi, torch, N, G, C, seed):
    t, params, data, off = synth.make_population("uneven", n_gal=G, seed=seed, sizes=[N] * G)
    init = synth.init_positions(t, params, data, off, C, seed=seed + 1)
    b = bsi.Batch(n=t.n_pix, psf_fwhm=torch.tensor(t.psf_fwhm, dtype=torch.float32).cuda(),
                  sigma=torch.tensor(t.sigma, dtype=torch.float32).cuda(), pixel_scale=PS)
    return t, params, data, off, init, b


@pytest.mark.parametrize("N", sorted(PLANS))
def test_every_plan_at_parity(bsi, N):
    import torch
    G, C, L, S = 2, 2, 10, 3
    t, params, data, off, init, b = _setup(bsi, torch, N, G, C, 300 + N)
    dev = torch.tensor(data).cuda()
    ref = torch.tensor(np.stack([t.dx, t.dy], 1), dtype=torch.float32).cuda()
    p32 = params.astype(np.float32)
    for P in PLANS[N]:
        _log(f"plan N={N} P={P}")
        bsi.set_plan(N, P)
        assert bsi.get_plan(N)[0] == P
        ll, gr, _ = bsi.loglik_grad(b, dev, torch.tensor(p32).cuda())
        ll, gr = ll.cpu().numpy(), gr.cpu().numpy()
        cfg = bsi.HmcConfig(n_chains=C, n_leapfrog=L, n_warmup=0, n_samples=S, adapt=False,
                            step_size=0.003, jitter=0.1, seed=11)
        smp, _, _ = bsi.hmc_sample(b, dev, ref, torch.tensor(init, dtype=torch.float32).cuda(), cfg)
        smp = smp.cpu().numpy()
        for i in range(G):
            d = data[off[i]:off[i] + N * N].reshape(N, N).astype(np.float64)
            psf = float(np.float32(t.psf_fwhm[i]))
            rll, rg = render.loglik_grad(d, p32[i].astype(np.float64), N, PS, psf, float(t.sigma[i]))
            assert abs(ll[i] - rll) <= 1e-6 * abs(rll), (N, P, i)
            _, dT = render.spectrum(p32[i].astype(np.float64), N, PS, psf, derivs=True)
            sc = np.array([math.sqrt(np.sum(render.synthesize(dT[j], N) ** 2)) / t.sigma[i]
                           for j in range(6)])
            assert np.all(np.abs(gr[i] - rg) <= 1e-4 * (np.abs(rg) + sc)), (N, P, i)
            gal = synth.oracle_galaxy(t, data, off, i)
            r = hmc.run_chain(hmc.galaxy_potential(gal), init[i, 0].astype(np.float32), 11, i * C,
                              L, 0, S, 0.003, adapt=False, jitter=0.1)
            k = 0
            while k < S and np.max(np.abs(smp[i, 0, k] - r["samples"][k])) <= 1e-4:
                k += 1
            if k < S:      # only an accept decision taken differently may end the agreement
                moved_g = k == 0 or np.any(smp[i, 0, k] != smp[i, 0, k - 1])
                moved_o = k == 0 or np.any(r["samples"][k] != r["samples"][k - 1])
                assert moved_g != moved_o, (N, P, i, k)
    bsi.set_plan(N, 0)


def test_autotune_and_tuned_run(bsi):
    import torch
    _log("autotune")
    res = bsi.autotune([25, 41, 53, 73, 101], n_chains=4)
    for N, (P, ms) in res.items():
        assert P in (1, 2, 3, 4, 5, 6, 8)
        assert bsi.get_plan(N)[0] == P
        assert ms is None or ms > 0
    _log(f"tuned plans {res}")
    # a mixed batch with the tuned plans: graph and forked forms agree, chains finite
    sizes = [25, 41, 53, 73, 101]
    t, params, data, off = synth.make_population("uneven", n_gal=5, seed=77, sizes=sizes)
    init = synth.init_positions(t, params, data, off, 2, seed=78)
    b = bsi.Batch(n=t.n_pix, psf_fwhm=torch.tensor(t.psf_fwhm, dtype=torch.float32).cuda(),
                  sigma=torch.tensor(t.sigma, dtype=torch.float32).cuda(), pixel_scale=PS)
    ref = torch.tensor(np.stack([t.dx, t.dy], 1), dtype=torch.float32).cuda()
    base = dict(n_chains=2, n_leapfrog=8, n_warmup=4, n_samples=4, adapt=True, step_size=0.01,
                seed=3)
    a = bsi.hmc_sample(b, torch.tensor(data).cuda(), ref, torch.tensor(init, dtype=torch.float32).cuda(),
                       bsi.HmcConfig(**base))[0].cpu().numpy()
    d = bsi.hmc_sample(b, torch.tensor(data).cuda(), ref, torch.tensor(init, dtype=torch.float32).cuda(),
                       bsi.HmcConfig(use_graph=False, **base))[0].cpu().numpy()
    assert np.array_equal(a, d) and np.all(np.isfinite(a))
    for N in res:
        bsi.set_plan(N, 0)


@pytest.mark.parametrize("wpc", [2, 4])
def test_split_chains_at_parity(bsi, wpc):
    """Several waves per chain (latency form): chains follow the oracle under
    the same momenta, and two calls give bitwise equal samples."""
    import torch
    sizes = [25, 53, 73, 101]
    G, C, L, S = len(sizes), 1, 10, 3
    t, params, data, off = synth.make_population("uneven", n_gal=G, seed=500 + wpc, sizes=sizes)
    init = synth.init_positions(t, params, data, off, C, seed=501)
    b = bsi.Batch(n=t.n_pix, psf_fwhm=torch.tensor(t.psf_fwhm, dtype=torch.float32).cuda(),
                  sigma=torch.tensor(t.sigma, dtype=torch.float32).cuda(), pixel_scale=PS)
    dev = torch.tensor(data).cuda()
    ref = torch.tensor(np.stack([t.dx, t.dy], 1), dtype=torch.float32).cuda()
    cfg = bsi.HmcConfig(n_chains=C, n_leapfrog=L, n_warmup=0, n_samples=S, adapt=False,
                        step_size=0.003, jitter=0.1, seed=13, waves_per_chain=wpc)
    it = torch.tensor(init, dtype=torch.float32).cuda()
    s1 = bsi.hmc_sample(b, dev, ref, it, cfg)[0].cpu().numpy()
    s2 = bsi.hmc_sample(b, dev, ref, it, cfg)[0].cpu().numpy()
    assert np.array_equal(s1, s2)
    for i, N in enumerate(sizes):
        _log(f"split chains wpc={wpc} N={N}")
        gal = synth.oracle_galaxy(t, data, off, i)
        r = hmc.run_chain(hmc.galaxy_potential(gal), init[i, 0].astype(np.float32), 13, i, L, 0, S,
                          0.003, adapt=False, jitter=0.1)
        k = 0
        while k < S and np.max(np.abs(s1[i, 0, k] - r["samples"][k])) <= 1e-4:
            k += 1
        if k < S:
            moved_g = k == 0 or np.any(s1[i, 0, k] != s1[i, 0, k - 1])
            moved_o = k == 0 or np.any(r["samples"][k] != r["samples"][k - 1])
            assert moved_g != moved_o, (wpc, N, k)


def _restated_layout(N, P):
    """Host restatement of the pair-slot layout: npc = hc + 1 pair-columns per
    row (rows 0..hc), R = floor(64 P / npc) rows per super-row, lane l of
    iteration i holding pair-slot l + 64 i, pair-slot (j, v) holding the bins
    (+j, v) and (-j, v), column 0 as two half-weight copies.  Returns (number
    of super-rows, {bin: total squared weight}) or None for an invalid plan."""
    nc = N if N % 2 else N - 1
    hc = (nc - 1) // 2
    rows = npc = hc + 1
    R = (64 * P) // npc
    if R < 1:
        return None
    R = min(R, rows)
    nsr = -(-rows // R)
    weight = {}
    for sr in range(nsr):
        for sl in range(min(P * 64, R * npc)):
            ro, j = divmod(sl, npc)
            v = sr * R + ro
            if v > hc:
                continue
            for half in (0, 1):
                u = -j if half else j
                w = (0.5 if v == 0 else 1.0) * (0.5 if j == 0 else 1.0)
                weight[(u, v)] = weight.get((u, v), 0.0) + w
    return nsr, weight


def test_library_plans_tile_the_half_plane(bsi):
    """For every stamp side 8..128 and every plan P the library accepts
    (bsi_set_plan / bsi_get_plan), its slot count is that of the pair-slot
    layout (two stored values per pair-slot, padding included); that layout
    covers the odd core's half plane with total weight 1 per bin (row 0) or
    1 with its mirror (rows 1..hc), and the mirrors complete the DFT grid.
    The plans the library rejects are exactly those with no row per super-row,
    and its default plan has the fewest slots (ties: the smaller P)."""
    import torch  # noqa: F401  (device fixture)
    for N in range(8, 129):
        nc = N if N % 2 else N - 1
        rows = (nc - 1) // 2 + 1
        best = None
        for P in (1, 2, 3, 4, 5, 6, 8):
            lay = _restated_layout(N, P)
            if lay is None:
                with pytest.raises(bsi.BsiError):
                    bsi.set_plan(N, P)
                continue
            bsi.set_plan(N, P)
            got_P, slots = bsi.get_plan(N)
            nsr, weight = lay
            assert got_P == P and slots == 2 * nsr * P * 64, (N, P, got_P, slots)
            assert len(weight) == nc * rows, (N, P)
            for (u, v), w in weight.items():
                assert w == (0.5 if v == 0 else 1.0), (N, P, u, v, w)
            full = {(u, v) for (u, v) in weight} | {(-u, -v) for (u, v) in weight}
            assert len(full) == nc * nc, (N, P)
            if best is None or slots < best[1]:
                best = (P, slots)
        bsi.set_plan(N, 0)
        assert bsi.get_plan(N) == best, (N, bsi.get_plan(N), best)


def test_tune_cache_round_trip(bsi, tmp_path):
    """bsi_create's tuning cache: bsi_autotune writes the handle's choices;
    a new handle on the same cache starts with them; a cache written for
    another device is ignored; a cache that does not parse fails creation."""
    _log("tune cache")
    path = tmp_path / "tune.txt"
    lib = bsi.Library(0, tune_cache=str(path))
    assert not path.exists()
    bsi.set_transform(53, bsi.N.TRANSFORM_DIRECT, lib=lib)
    bsi.autotune([25, 53], n_chains=4, lib=lib)
    lines = path.read_text().splitlines()
    assert lines[0] == "bsi-tune-cache 1" and lines[1] == "library 4"
    dev = lines[2].split()
    assert dev[0] == "device" and dev[1].startswith("gfx950") and int(dev[2]) > 0
    chosen = {N: bsi.get_plan(N, lib=lib)[0] for N in (25, 53)}
    assert {f"plan {N} {P}" for N, P in chosen.items()} <= set(lines[3:])
    assert "transform 53 1" in lines[3:]
    lib.close()

    lib2 = bsi.Library(0, tune_cache=str(path))
    assert {N: bsi.get_plan(N, lib=lib2)[0] for N in (25, 53)} == chosen
    assert bsi.get_transform(53, lib=lib2) == bsi.N.TRANSFORM_DIRECT
    lib2.close()

    # a cache for this device with a plan the defaults would not pick
    mine = tmp_path / "mine.txt"
    mine.write_text("\n".join(lines[:3] + ["plan 53 6", "transform 41 1"]) + "\n")
    lib3 = bsi.Library(0, tune_cache=str(mine))
    assert bsi.get_plan(53, lib=lib3)[0] == 6 and bsi.get_transform(41, lib=lib3) == 1
    assert bsi.get_plan(25, lib=lib3)[0] == 3
    lib3.close()

    # another device's (or library version's) cache is ignored
    for hdr in (lines[:2] + [f"device {dev[1]} {int(dev[2]) + 1}"],
                ["bsi-tune-cache 1", "library 3", lines[2]]):
        other = tmp_path / "other.txt"
        other.write_text("\n".join(hdr + ["plan 53 6"]) + "\n")
        lib4 = bsi.Library(0, tune_cache=str(other))
        assert bsi.get_plan(53, lib=lib4)[0] == 3
        lib4.close()

    # malformed caches fail bsi_create with BSI_EINVAL
    for body in ("not a cache\n", "bsi-tune-cache 1\nplan 53 7\n", "bsi-tune-cache 1\nplan 300 3\n",
                 "bsi-tune-cache 1\ncolour blue\n", "bsi-tune-cache 1\ntransform 53 9\n",
                 "bsi-tune-cache 1\nplan 53 6\n"):
        bad = tmp_path / "bad.txt"
        bad.write_text(body)
        with pytest.raises(bsi.BsiError, match="BSI_EINVAL.*tune cache"):
            bsi.Library(0, tune_cache=str(bad))
