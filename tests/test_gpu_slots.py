"""The request server (bsi_slots_*): each request's samples are identical
whether it runs alone or in a changing mix of other requests of other stamp
sizes (bitwise: a chain's arithmetic and random numbers depend only on its
own data and uid), admission follows the device footprint, and every
admitted request is handed back exactly once."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import diagnostics                               # noqa: E402
from tests import synth                                      # noqa: E402
from workloads import gen                                    # noqa: E402

PS = gen.PIXEL_SCALE


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bsi(device):
    from paper_2604_22048_amd import api
    return api


def _requests(n, sizes, seed):
    t, params, data, off = synth.make_population("uneven", n_gal=n, seed=seed, sizes=sizes)
    init = synth.init_positions(t, params, data, off, 1, seed)[:, 0]
    return t, params, data, off, init


CFG = dict(n_chains=1, n_leapfrog=6, n_warmup=12, n_samples=15, adapt=True, metric=1,
           step_size=0.05, jitter=0.2, seed=9)


@pytest.mark.parametrize("pace,wpc", [(False, 1), (True, 1), (False, 4)])
def test_slots_alone_equals_mix_bitwise(bsi, pace, wpc):
    import torch
    _log(f"slots alone vs mix pace={pace} waves_per_chain={wpc}")
    rng = np.random.default_rng(70)
    n = 20
    sizes = rng.choice([25, 41, 53], n)
    t, params, data, off, init = _requests(n, sizes, 71)
    dev = torch.tensor(data).cuda()
    cfg = bsi.HmcConfig(waves_per_chain=wpc, **CFG)
    srv = bsi.Slots([25, 41, 53], cfg, hbm_budget=64 << 20, max_slots=6, pace=pace)
    ids = 1000 + np.arange(n)
    queue = list(range(n))
    got = {}
    ticks = 0
    while len(got) < n:
        while queue:
            i = queue[0]
            N = int(t.n_pix[i])
            ok = srv.admit(int(ids[i]), dev[off[i]:off[i] + N * N], float(t.psf_fwhm[i]),
                           float(t.sigma[i]), (params[i, 4], params[i, 5]), init[i])
            if not ok:
                break
            queue.pop(0)
        inf = srv.info()
        assert inf["resident"] <= 6
        srv.advance(int(rng.integers(2, 9)))
        ticks += 1
        hid, smp, st, status, nd = srv.harvest(n)
        assert np.all(nd.cpu().numpy() == CFG["n_samples"])
        for k, rid in enumerate(hid):
            assert int(rid) not in got
            got[int(rid)] = (smp[k].cpu().numpy(), st[k].cpu().numpy())
        assert ticks < 200
    inf = srv.info()
    assert inf["resident"] == 0 and inf["arena_free"] == inf["arena_bytes"]
    assert ticks > 3          # requests overlapped and queued
    # alone: a one-galaxy bsi_hmc_sample with the request's chain uid
    for i in [0, 3, 7, 12, 19]:
        N = int(t.n_pix[i])
        b = bsi.Batch(n=np.array([N]), psf_fwhm=torch.tensor([t.psf_fwhm[i]], dtype=torch.float32).cuda(),
                      sigma=torch.tensor([t.sigma[i]], dtype=torch.float32).cuda(), pixel_scale=PS)
        ref = torch.tensor([[params[i, 4], params[i, 5]]], dtype=torch.float32).cuda()
        ini = torch.tensor(init[i][None, None, :], dtype=torch.float32).cuda()
        c1 = bsi.HmcConfig(uid_base=int(ids[i]), waves_per_chain=wpc, **CFG)
        smp, st, _ = bsi.hmc_sample(b, dev[off[i]:off[i] + N * N].contiguous(), ref, ini, c1)
        assert np.array_equal(smp[0].cpu().numpy(), got[int(ids[i])][0]), i
        assert np.array_equal(st[0].cpu().numpy(), got[int(ids[i])][1]), i
    # alone in the server too
    srv1 = bsi.Slots([53, 25, 41], cfg, hbm_budget=16 << 20)
    i = 5
    N = int(t.n_pix[i])
    assert srv1.admit(int(ids[i]), dev[off[i]:off[i] + N * N], float(t.psf_fwhm[i]), float(t.sigma[i]),
                      (params[i, 4], params[i, 5]), init[i])
    srv1.advance(CFG["n_warmup"] + CFG["n_samples"])
    hid, smp, st, _, _ = srv1.harvest(4)
    assert list(hid) == [ids[i]]
    assert np.array_equal(smp[0].cpu().numpy(), got[int(ids[i])][0])
    srv.close()
    srv1.close()


def test_slots_admission_by_footprint(bsi):
    import torch
    _log("slots admission")
    cfg = bsi.HmcConfig(**CFG)
    n = 8
    t, params, data, off, init = _requests(n, [53] * n, 72)
    dev = torch.tensor(data).cuda()
    probe = bsi.Slots([53], cfg, hbm_budget=16 << 20)
    fp = probe.footprint(53)
    probe.close()
    # room for exactly three 53-pixel requests
    srv = bsi.Slots([53], cfg, hbm_budget=4 * fp, max_slots=3)
    assert srv.footprint(53) == fp
    adm = []
    for i in range(n):
        N = 53
        adm.append(srv.admit(i, dev[off[i]:off[i] + N * N], float(t.psf_fwhm[i]), float(t.sigma[i]),
                             (params[i, 4], params[i, 5]), init[i]))
    assert adm == [True] * 3 + [False] * (n - 3)
    inf = srv.info()
    assert inf["resident"] == 3 and inf["pending"] == 3
    srv.advance(CFG["n_warmup"] + CFG["n_samples"])
    hid, smp, st, status, _ = srv.harvest(2)
    assert list(hid) == [0, 1]
    assert np.all(np.isfinite(smp.cpu().numpy()))
    assert srv.info()["resident"] == 1
    assert srv.admit(3, dev[off[3]:off[3] + 2809], float(t.psf_fwhm[3]), float(t.sigma[3]),
                     (params[3, 4], params[3, 5]), init[3])
    with pytest.raises(Exception):
        srv.admit(4, dev[:25 * 25], 0.7, 1.0, (0, 0), init[4])     # size not served
    srv.close()


def test_slots_ess_target(bsi):
    """Requests asking for an ESS: each finishes at the first check (every
    20 draws after warmup) where the mean ESS over the six parameters reaches
    the target, by the oracle's ESS of the returned draws, or at the draw
    cap; draws past the stop are NaN; and the request alone in a one-galaxy
    bsi_hmc_sample with n_samples = n_draws gives the same draws and chain
    statistics bitwise (the chains wait at each check)."""
    import torch
    _log("slots ESS target")
    cfg_d = dict(CFG, n_chains=2, n_warmup=12, n_samples=120)
    every, target = 20, 45.0
    rng = np.random.default_rng(80)
    n = 14
    sizes = rng.choice([25, 41, 53], n)
    t, params, data, off = synth.make_population("uneven", n_gal=n, seed=81, sizes=sizes)
    init = synth.init_positions(t, params, data, off, 2, seed=82)
    dev = torch.tensor(data).cuda()
    cfg = bsi.HmcConfig(**cfg_d)
    srv = bsi.Slots([25, 41, 53], cfg, hbm_budget=64 << 20, max_slots=5, ess_target=target,
                    ess_every=every)
    ids = 500 + np.arange(n)
    queue = list(range(n))
    got = {}
    ticks = 0
    while len(got) < n:
        while queue:
            i = queue[0]
            N = int(t.n_pix[i])
            if not srv.admit(int(ids[i]), dev[off[i]:off[i] + N * N], float(t.psf_fwhm[i]),
                             float(t.sigma[i]), (params[i, 4], params[i, 5]), init[i]):
                break
            queue.pop(0)
        srv.advance(int(rng.integers(3, 11)))
        ticks += 1
        srv.poll()
        hid, smp, st, status, nd = srv.harvest(n)
        for k, rid in enumerate(hid):
            assert int(rid) not in got
            got[int(rid)] = (smp[k].cpu().numpy(), st[k].cpu().numpy(), int(nd[k]))
        assert ticks < 400
    inf = srv.info()
    assert inf["resident"] == 0 and inf["arena_free"] == inf["arena_bytes"]
    srv.close()
    early = 0
    for i in range(n):
        smp, st, nd = got[int(ids[i])]
        assert nd % every == 0 and every <= nd <= cfg_d["n_samples"], nd
        assert np.all(np.isfinite(smp[:, :nd])) and np.all(np.isnan(smp[:, nd:]))
        x = smp.astype(np.float64)
        e_at = np.mean(diagnostics.ess_params(x[:, :nd]))
        if nd < cfg_d["n_samples"]:
            early += 1
            assert e_at >= target * (1 - 1e-4), (i, nd, e_at)
        if nd > every:
            e_prev = np.mean(diagnostics.ess_params(x[:, :nd - every]))
            assert e_prev < target * (1 + 1e-4), (i, nd, e_prev)
        # alone, with the draws the server returned
        N = int(t.n_pix[i])
        b = bsi.Batch(n=np.array([N]), psf_fwhm=torch.tensor([t.psf_fwhm[i]], dtype=torch.float32).cuda(),
                      sigma=torch.tensor([t.sigma[i]], dtype=torch.float32).cuda(), pixel_scale=PS)
        ref = torch.tensor([[params[i, 4], params[i, 5]]], dtype=torch.float32).cuda()
        ini = torch.tensor(init[i][None], dtype=torch.float32).cuda()
        c1 = bsi.HmcConfig(uid_base=int(ids[i]) * 2, **dict(cfg_d, n_samples=nd))
        s1, st1, _ = bsi.hmc_sample(b, dev[off[i]:off[i] + N * N].contiguous(), ref, ini, c1)
        assert np.array_equal(s1[0].cpu().numpy(), smp[:, :nd]), i
        assert np.array_equal(st1[0].cpu().numpy(), st), i
    assert early >= 1


def test_serve_loop_ess_batches(bsi):
    """The request loop's ESS of returned draws: every request completes
    once, with a draw count at a check or at the cap, a finite mean ESS that
    reaches the target for requests stopped early, and the same values
    whether the kept draws are checked after every harvest or once after the
    loop."""
    import torch
    from paper_2604_22048_amd import serve
    _log("serve loop ESS batches")
    sizes_srv = [25, 41]
    n, P, C = 12, 4, 2
    every, target, cap = 20, 45.0, 120
    pool = {k: {} for k in ("stamps", "psf", "sigma", "ref", "init")}
    for N in sizes_srv:
        t, params, data, off = synth.make_population("uneven", n_gal=P, seed=90 + N,
                                                     sizes=np.full(P, N))
        init = synth.init_positions(t, params, data, off, C, seed=91 + N)
        pool["stamps"][N] = torch.tensor(data).cuda().view(P, N * N)
        pool["psf"][N] = t.psf_fwhm.astype(np.float32)
        pool["sigma"][N] = t.sigma.astype(np.float32)
        pool["ref"][N] = np.ascontiguousarray(params[:, 4:6].astype(np.float32))
        pool["init"][N] = np.ascontiguousarray(init.astype(np.float32))
    pool = serve.RequestPool(**pool)
    sizes = np.random.default_rng(92).choice(np.array(sizes_srv), n)
    cfg = bsi.HmcConfig(**dict(CFG, n_chains=C, n_samples=cap))
    out = []
    for batch_bytes in (1, 1 << 30):
        old = serve.ESS_BATCH_BYTES
        serve.ESS_BATCH_BYTES = batch_bytes
        try:
            srv = bsi.Slots(sizes_srv, cfg, hbm_budget=64 << 20, max_slots=5, ess_target=target,
                            ess_every=every)
            r = serve.serve(srv, pool, np.zeros(n), sizes, 7, time_limit=60.0, ess=True)
            srv.close()
        finally:
            serve.ESS_BATCH_BYTES = old
        assert r.n_done == n and np.all(np.isfinite(r.latency))
        assert np.all(r.n_draws % every == 0) and np.all((r.n_draws >= every) & (r.n_draws <= cap))
        assert np.all(np.isfinite(r.ess_mean))
        early = r.n_draws < cap
        assert np.all(r.ess_mean[early] >= target * (1 - 1e-3)), r.ess_mean[early]
        out.append(r)
    assert np.array_equal(out[0].n_draws, out[1].n_draws)
    assert np.array_equal(out[0].ess_mean, out[1].ess_mean)
