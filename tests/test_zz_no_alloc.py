"""The allocation-free shear posterior (bsi_shear_posterior_noalloc) against
the ordinary entry point (bsi_shear_posterior), both through the C ABI: two
calls in a row, the second with a smaller input (the scratch keeps the first
call's contents), outputs bitwise equal (same kernels and reduction order)
and within the float32 bound of the oracle; a call whose pass exceeds the
scratch fails with BSI_EINVAL before enqueueing anything."""
import ctypes as C
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import shear                  # noqa: E402
from tests import f32bound, synth         # noqa: E402


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods(device):
    import torch
    from paper_2604_22048_amd import api
    return api, torch


def _points(rng, P):
    pts = np.empty((P, 5))
    pts[:, 0] = rng.uniform(-0.06, 0.06, P)
    pts[:, 1] = rng.uniform(-0.06, 0.06, P)
    pts[:, 2] = math.log(0.6) + rng.uniform(-0.2, 0.2, P)
    pts[:, 3] = rng.uniform(0.2, 0.4, P)
    pts[:, 4] = rng.uniform(0.15, 0.3, P)
    return pts


def test_noalloc_matches_shear_posterior(mods):
    api, torch = mods
    rng = np.random.default_rng(71)
    tpo = shear.TruePrior(e_kind=1, e_max=0.95)
    tpg = api.TruePriorCfg(e_kind=1, e_max=0.95, size_term=True)
    # first call: several blocks and two point chunks; second: a smaller input
    for G, K, P in ((300, 400, 70), (40, 100, 3)):
        _log(f"noalloc G={G} K={K} P={P}")
        S = synth.interim_population(G, K, seed=G + K)
        St = [torch.tensor(a).cuda() for a in S]
        pts = _points(rng, P)
        pts_d = torch.tensor(pts, dtype=torch.float64, device="cuda")
        lp_ref, gr_ref = api.shear_posterior(St[0], St[1], St[2], None, pts_d, tpg, want_grad=True)
        lp, gr = api.shear_posterior_noalloc(St[0], St[1], St[2], None, pts_d, tpg, want_grad=True)
        torch.cuda.synchronize()
        assert torch.equal(lp, lp_ref) and torch.equal(gr, gr_ref)
        lp = lp.cpu().numpy()
        Sd = [a.astype(np.float64) for a in S]
        for j in (0, P - 1):
            g, alpha = complex(pts[j, 0], pts[j, 1]), tuple(pts[j, 2:])
            rl = shear.log_posterior(Sd, g, alpha, tpo, shear.Interim())
            tol = f32bound.posterior_bounds(Sd, g, alpha, tpo, shear.Interim(), want_grad=False)[0]
            assert abs(lp[j] - rl) <= tol, (G, j, lp[j], rl, tol)


def test_noalloc_rejects_a_pass_beyond_the_scratch(mods):
    api, torch = mods
    _log("noalloc scratch limit")
    G, K, P = 256, 8, 24000           # 16 blocks x 24000 points x 48 B > 16 MiB
    lib = api.get(0)
    e = torch.zeros(G, K, device="cuda")
    pts = torch.tensor(_points(np.random.default_rng(3), P), dtype=torch.float64, device="cuda")
    lp = torch.empty(P, dtype=torch.float64, device="cuda")
    tp = api.TruePriorCfg(e_kind=1, e_max=0.95, size_term=True).c()
    ip = api._interim(None)
    p = lambda t: C.c_void_p(t.data_ptr())
    rc = lib.lib.bsi_shear_posterior_noalloc(lib.h, G, K, p(e), p(e), p(e), None, C.byref(tp),
                                             C.byref(ip), P, p(pts), p(lp), None, None)
    assert rc == -1 and b"scratch" in lib.lib.bsi_last_error(lib.h)
