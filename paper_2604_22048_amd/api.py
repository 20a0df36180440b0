"""Python binding of the shear-inference library: same call names as the C
ABI, torch tensors for device memory and streams.  Every computation runs in
the HIP library; this module only checks shapes and passes pointers."""
from __future__ import annotations

import ctypes as C
import os
import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _native as N

PAPER_INTERIM = dict(log10f_lo=-1.0, log10f_hi=9.0, log10s_lo=-2.0, log10s_hi=1.0,
                     sigma_d=0.5, sigma_e=0.3)


class BsiError(RuntimeError):
    pass


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Library:
    """One handle on one device.  Use ``get()`` for the process-wide default.
    tune_cache: path of the handle's tuning cache (bsi_create), or None."""

    def __init__(self, device: int = 0, tune_cache: str | None = None):
        self.lib = N.load()
        self.device = device
        h = C.c_void_p()
        path = None if tune_cache is None else os.fsencode(tune_cache)
        rc = self.lib.bsi_create(C.byref(h), device, path)
        if rc != N.BSI_OK:
            raise BsiError(f"bsi_create: {N.ERRORS.get(rc, rc)}: {self.lib.bsi_last_error(None).decode()}")
        self.h = h

    def check(self, rc, what):
        if rc != N.BSI_OK:
            msg = self.lib.bsi_last_error(self.h).decode()
            raise BsiError(f"{what}: {N.ERRORS.get(rc, rc)}: {msg}")

    def close(self):
        if self.h:
            self.lib.bsi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = {}


def get(device: int = 0) -> Library:
    if device not in _default:
        _default[device] = Library(device)
    return _default[device]


@dataclass
class Batch:
    """A ragged batch of square stamps packed row-major back to back."""
    n: np.ndarray                 # int32 [G] stamp sides (host)
    psf_fwhm: torch.Tensor        # float32 [G] (device)
    sigma: torch.Tensor           # float32 [G] (device)
    pixel_scale: float = 0.2
    profile: int = N.PROFILE_EXPONENTIAL
    off: np.ndarray = field(default=None)   # int64 [G]; default: packed in order
    spergel_nu: float = 0.5       # Spergel index (profile PROFILE_SPERGEL only)
    n_exp: int = 1                # exposures per galaxy; n, psf_fwhm, sigma, off are per stamp
    noise_ps: torch.Tensor = None # float32 packed like the stamps: DFT-mode noise powers, or None

    def __post_init__(self):
        self.n = np.ascontiguousarray(self.n, dtype=np.int32)
        if self.off is None:
            sz = self.n.astype(np.int64) ** 2
            self.off = np.concatenate([[0], np.cumsum(sz)[:-1]]).astype(np.int64)
        self.off = np.ascontiguousarray(self.off, dtype=np.int64)
        self.psf_fwhm = self.psf_fwhm.contiguous().float()
        self.sigma = self.sigma.contiguous().float()
        if self.noise_ps is not None:
            self.noise_ps = self.noise_ps.contiguous().float()

    @property
    def n_gal(self):
        return int(self.n.shape[0]) // max(1, int(self.n_exp))

    @property
    def n_pixels(self):
        return int((self.off + self.n.astype(np.int64) ** 2).max()) if self.n_gal else 0

    def c(self) -> N.Batch:
        b = N.Batch()
        b.n_gal = self.n_gal
        b.n = self.n.ctypes.data_as(C.POINTER(C.c_int32))
        b.off = self.off.ctypes.data_as(C.POINTER(C.c_int64))
        b.psf_fwhm = self.psf_fwhm.data_ptr()
        b.sigma = self.sigma.data_ptr()
        b.pixel_scale = float(self.pixel_scale)
        b.profile = int(self.profile)
        b.spergel_nu = float(self.spergel_nu)
        b.n_exp = int(self.n_exp)
        b.noise_ps = None if self.noise_ps is None else self.noise_ps.data_ptr()
        return b


def _interim(d=None) -> N.Interim:
    d = dict(PAPER_INTERIM if d is None else d)
    return N.Interim(**{k: float(v) for k, v in d.items()})


def render_stamps(batch: Batch, params: torch.Tensor, lib: Library | None = None) -> torch.Tensor:
    lib = lib or get(params.device.index or 0)
    params = params.contiguous().float()
    assert params.shape == (batch.n_gal, 6)
    out = torch.zeros(batch.n_pixels, dtype=torch.float32, device=params.device)
    b = batch.c()
    lib.check(lib.lib.bsi_render_stamps(lib.h, C.byref(b), _ptr(params), _ptr(out),
                                        _stream(params.device)), "bsi_render_stamps")
    return out


def loglik_grad(batch: Batch, data: torch.Tensor, params: torch.Tensor, method: int = N.LIK_KSPACE,
                lib: Library | None = None):
    """(log L [G] float64, d log L / d params [G, 6], status [G] int32)."""
    lib = lib or get(params.device.index or 0)
    params = params.contiguous().float()
    data = data.contiguous().float()
    G = batch.n_gal
    dev = params.device
    ll = torch.empty(G, dtype=torch.float64, device=dev)
    gr = torch.empty(G, 6, dtype=torch.float32, device=dev)
    st = torch.empty(G, dtype=torch.int32, device=dev)
    b = batch.c()
    lib.check(lib.lib.bsi_loglik_grad(lib.h, C.byref(b), _ptr(data), _ptr(params), _ptr(ll), _ptr(gr),
                                      _ptr(st), int(method), _stream(dev)), "bsi_loglik_grad")
    return ll, gr, st


@dataclass
class HmcConfig:
    n_chains: int = 4
    n_leapfrog: int = 20
    n_warmup: int = 300
    n_samples: int = 1000
    adapt: bool = True
    metric: int = N.METRIC_GIVEN
    step_size: float = 0.01
    target_accept: float = 0.8
    jitter: float = 0.0
    form: int = N.FORM_BATCHED
    iters_per_launch: int = 1
    use_graph: bool = True
    seed: int = 0
    uid_base: int = 0
    waves_per_chain: int = 1
    sampler: int = N.SAMPLER_HMC      # or N.SAMPLER_NUTS (Section 3.3's sampler)
    max_tree_depth: int = 5           # NUTS doublings per transition (the paper's 5)

    def c(self, trace=None) -> N.HmcCfg:
        return N.HmcCfg(int(self.n_chains), int(self.n_leapfrog), int(self.n_warmup),
                        int(self.n_samples), int(bool(self.adapt)), int(self.metric),
                        float(self.step_size), float(self.target_accept), float(self.jitter),
                        int(self.form), int(self.iters_per_launch), int(bool(self.use_graph)),
                        int(self.seed) & 0xFFFFFFFFFFFFFFFF, int(self.uid_base) & 0xFFFFFFFFFFFFFFFF,
                        None if trace is None else trace.data_ptr(), int(self.waves_per_chain),
                        int(self.sampler), int(self.max_tree_depth))


def hmc_sample(batch: Batch, data: torch.Tensor, ref_xy: torch.Tensor, init: torch.Tensor,
               cfg: HmcConfig, interim=None, inv_mass: torch.Tensor | None = None,
               want_samples: bool = True, trace: torch.Tensor | None = None,
               lib: Library | None = None):
    """(samples [G, C, S, 6], chain_stats [G, C, 4], status [G]).

    trace: optional float32 [G, C, W + S, 4] tensor filled per iteration with
    (base step, dH, acceptance statistic, accepted)."""
    dev = data.device
    lib = lib or get(dev.index or 0)
    G, Cn, S = batch.n_gal, cfg.n_chains, cfg.n_samples
    assert init.shape == (G, Cn, 6) and ref_xy.shape == (G, 2)
    data = data.contiguous().float()
    init = init.contiguous().float()
    ref_xy = ref_xy.contiguous().float()
    if inv_mass is not None:
        inv_mass = inv_mass.contiguous().float()
        assert inv_mass.shape == (G, 6)
    samples = torch.empty(G, Cn, S, 6, dtype=torch.float32, device=dev) if want_samples else None
    stats = torch.empty(G, Cn, 4, dtype=torch.float32, device=dev)
    status = torch.empty(G, dtype=torch.int32, device=dev)
    if trace is not None:
        assert trace.shape == (G, Cn, cfg.n_warmup + S, 4) and trace.dtype == torch.float32
        assert trace.is_contiguous()
    b = batch.c()
    ip = _interim(interim)
    cc = cfg.c(trace)
    lib.check(lib.lib.bsi_hmc_sample(lib.h, C.byref(b), _ptr(data), _ptr(ref_xy), _ptr(inv_mass),
                                     _ptr(init), C.byref(ip), C.byref(cc), _ptr(samples),
                                     _ptr(stats), _ptr(status), _stream(dev)), "bsi_hmc_sample")
    return samples, stats, status


@dataclass
class TruePriorCfg:
    e_kind: int = N.E_TRUNC_GAUSS
    e_max: float = 0.7
    size_term: bool = True
    flux_term: bool = False
    mu_ln_f: float = 0.0
    sigma_ln_f: float = 1.0

    def c(self) -> N.TruePrior:
        return N.TruePrior(int(self.e_kind), float(self.e_max), int(bool(self.size_term)),
                           int(bool(self.flux_term)), float(self.mu_ln_f), float(self.sigma_ln_f))


def shear_posterior(e1p, e2p, log10s, log10f, pts, true_prior: TruePriorCfg, interim=None,
                    want_grad: bool = False, lib: Library | None = None):
    """ln P at points (g1, g2, mu_ln_s, sigma_ln_s, sigma_e); samples are [G, K] tensors."""
    dev = e1p.device
    lib = lib or get(dev.index or 0)
    G, K = e1p.shape
    e1p, e2p = e1p.contiguous().float(), e2p.contiguous().float()
    log10s = log10s.contiguous().float() if log10s is not None else None
    log10f = log10f.contiguous().float() if log10f is not None else None
    if isinstance(pts, torch.Tensor) and pts.is_cuda:
        pts_t = pts.contiguous().double()
        on_dev = 1
        P = pts_t.shape[0]
        pts_p = _ptr(pts_t)
    else:
        pts_np = np.ascontiguousarray(np.asarray(pts, dtype=np.float64).reshape(-1, 5))
        P = pts_np.shape[0]
        on_dev = 0
        pts_p = C.c_void_p(pts_np.ctypes.data)
    lp = torch.empty(P, dtype=torch.float64, device=dev)
    gr = torch.empty(P, 5, dtype=torch.float64, device=dev) if want_grad else None
    tp = true_prior.c()
    ip = _interim(interim)
    lib.check(lib.lib.bsi_shear_posterior(lib.h, G, K, _ptr(e1p), _ptr(e2p), _ptr(log10s),
                                          _ptr(log10f), C.byref(tp), C.byref(ip), P, pts_p, on_dev,
                                          _ptr(lp), _ptr(gr), _stream(dev)), "bsi_shear_posterior")
    return (lp, gr) if want_grad else lp


def shear_posterior_noalloc(e1p, e2p, log10s, log10f, pts: torch.Tensor, true_prior: TruePriorCfg,
                            interim=None, want_grad: bool = False, lib: Library | None = None):
    """bsi_shear_posterior_noalloc: as shear_posterior with device points, the
    pass's partial sums in the library's fixed device scratch (no allocation
    by the library; the outputs are allocated here by torch)."""
    dev = e1p.device
    lib = lib or get(dev.index or 0)
    G, K = e1p.shape
    e1p, e2p = e1p.contiguous().float(), e2p.contiguous().float()
    log10s = log10s.contiguous().float() if log10s is not None else None
    log10f = log10f.contiguous().float() if log10f is not None else None
    assert isinstance(pts, torch.Tensor) and pts.is_cuda, "points must be a device tensor"
    pts = pts.contiguous().double()
    P = pts.shape[0]
    lp = torch.empty(P, dtype=torch.float64, device=dev)
    gr = torch.empty(P, 5, dtype=torch.float64, device=dev) if want_grad else None
    tp = true_prior.c()
    ip = _interim(interim)
    lib.check(lib.lib.bsi_shear_posterior_noalloc(lib.h, G, K, _ptr(e1p), _ptr(e2p), _ptr(log10s),
                                                  _ptr(log10f), C.byref(tp), C.byref(ip), P, _ptr(pts),
                                                  _ptr(lp), _ptr(gr), _stream(dev)),
              "bsi_shear_posterior_noalloc")
    return (lp, gr) if want_grad else lp


def shear_galaxy_loglik(e1p, e2p, log10s, log10f, pts, true_prior: TruePriorCfg, interim=None,
                        lib: Library | None = None):
    """Per-galaxy log-marginals ell[p, n] at points (g1, g2, mu_ln_s, sigma_ln_s,
    sigma_e) (bsi_shear_galaxy_loglik); samples are [G, K] tensors."""
    dev = e1p.device
    lib = lib or get(dev.index or 0)
    G, K = e1p.shape
    e1p, e2p = e1p.contiguous().float(), e2p.contiguous().float()
    log10s = log10s.contiguous().float() if log10s is not None else None
    log10f = log10f.contiguous().float() if log10f is not None else None
    pts_t = torch.as_tensor(pts, dtype=torch.float64).reshape(-1, 5).to(dev).contiguous()
    P = pts_t.shape[0]
    ell = torch.empty(P, G, dtype=torch.float64, device=dev)
    tp = true_prior.c()
    ip = _interim(interim)
    lib.check(lib.lib.bsi_shear_galaxy_loglik(lib.h, G, K, _ptr(e1p), _ptr(e2p), _ptr(log10s),
                                              _ptr(log10f), C.byref(tp), C.byref(ip), P, _ptr(pts_t), 1,
                                              _ptr(ell), _stream(dev)), "bsi_shear_galaxy_loglik")
    return ell


def shear_bias(ell_plus, ell_minus, gpts, g_abs: float, counts=None, lib: Library | None = None):
    """m and c by shape-noise cancellation with bootstrap errors (bsi_shear_bias).
    ell_*: [P, G] float64 device tensors; gpts: [2, P, 2] (the +g dataset's grid, then the
    -g dataset's) or [P, 2] (one grid for both); counts: [B, G] int32 or None.
    Returns dict(stats=[m, c, sd(m), sd(c)], mc=[B+1, 2] (m_r, c_r), gmean=[2, B+1, 2]) as tensors."""
    dev = ell_plus.device
    lib = lib or get(dev.index or 0)
    P, G = ell_plus.shape
    ep = ell_plus.contiguous().double()
    em = ell_minus.contiguous().double()
    gp = torch.as_tensor(gpts, dtype=torch.float64).to(dev).reshape(-1, P, 2)
    gp = (gp.expand(2, P, 2) if gp.shape[0] == 1 else gp).contiguous()
    B = 0 if counts is None else int(counts.shape[0])
    cnt = None if counts is None else torch.as_tensor(counts, dtype=torch.int32).to(dev).contiguous()
    gmean = torch.empty(2, B + 1, 2, dtype=torch.float64, device=dev)
    mc = torch.empty(B + 1, 2, dtype=torch.float64, device=dev)
    stats = torch.empty(4, dtype=torch.float64, device=dev)
    lib.check(lib.lib.bsi_shear_bias(lib.h, G, P, _ptr(ep), _ptr(em), _ptr(gp), float(g_abs), B,
                                     _ptr(cnt), _ptr(gmean), _ptr(mc), _ptr(stats), _stream(dev)),
              "bsi_shear_bias")
    return {"stats": stats, "mc": mc, "gmean": gmean}


@dataclass
class ShearHmcConfig:
    n_chains: int = 4
    n_leapfrog: int = 10
    n_warmup: int = 500
    n_samples: int = 3000
    adapt: bool = True
    step_size: float = 1e-3
    target_accept: float = 0.8
    jitter: float = 0.0
    inv_mass: tuple = (1.0, 1.0, 1.0, 1.0, 1.0)
    seed: int = 0
    uid_base: int = 0
    use_graph: bool = True

    def c(self, trace=None) -> N.ShearHmcCfg:
        return N.ShearHmcCfg(int(self.n_chains), int(self.n_leapfrog), int(self.n_warmup),
                             int(self.n_samples), int(bool(self.adapt)), float(self.step_size),
                             float(self.target_accept), float(self.jitter),
                             (C.c_double * 5)(*[float(v) for v in self.inv_mass]),
                             int(self.seed) & 0xFFFFFFFFFFFFFFFF,
                             int(self.uid_base) & 0xFFFFFFFFFFFFFFFF, int(bool(self.use_graph)),
                             None if trace is None else trace.data_ptr())


def shear_hmc(e1p, e2p, log10s, log10f, true_prior: TruePriorCfg, cfg: ShearHmcConfig, init,
              interim=None, trace: torch.Tensor | None = None, want_samples: bool = True,
              lib: Library | None = None):
    """(samples [C, S, 5] float64, chain_stats [C, 4] float64) of the shear-level sampler.

    init: start points [C, 5] (host array).  trace: optional float32
    [C, W + S, 4] tensor (base step, dH, acceptance statistic, accepted)."""
    dev = e1p.device
    lib = lib or get(dev.index or 0)
    G, K = e1p.shape
    e1p, e2p = e1p.contiguous().float(), e2p.contiguous().float()
    log10s = log10s.contiguous().float() if log10s is not None else None
    log10f = log10f.contiguous().float() if log10f is not None else None
    Cn, S = cfg.n_chains, cfg.n_samples
    init_np = np.ascontiguousarray(np.asarray(init, dtype=np.float64).reshape(Cn, 5))
    samples = torch.empty(Cn, S, 5, dtype=torch.float64, device=dev) if want_samples else None
    stats = torch.empty(Cn, 4, dtype=torch.float64, device=dev)
    if trace is not None:
        assert trace.shape == (Cn, cfg.n_warmup + S, 4) and trace.dtype == torch.float32
        assert trace.is_contiguous()
    tp = true_prior.c()
    ip = _interim(interim)
    cc = cfg.c(trace)
    lib.check(lib.lib.bsi_shear_hmc(lib.h, G, K, _ptr(e1p), _ptr(e2p), _ptr(log10s), _ptr(log10f),
                                    C.byref(tp), C.byref(ip), C.byref(cc),
                                    C.c_void_p(init_np.ctypes.data), _ptr(samples), _ptr(stats),
                                    _stream(dev)), "bsi_shear_hmc")
    return samples, stats


class Slots:
    """Request server (bsi_slots_*): admit galaxy-fit requests while their
    device footprint fits, advance all resident chains, harvest finished
    requests.  Work is ordered on the stream current at creation.

    ess_target > 0: each request asks for that many effective samples; it is
    checked every ess_every draws after warmup and finishes at the first check
    that reaches the target (or after cfg.n_samples draws)."""

    def __init__(self, sizes, cfg: HmcConfig, hbm_budget: int, max_slots: int = 0, interim=None,
                 pixel_scale: float = 0.2, profile: int = N.PROFILE_EXPONENTIAL,
                 pace: bool = False, ess_target: float = 0.0, ess_every: int = 100, device: int = 0,
                 lib: Library | None = None, spergel_nu: float = 0.5):
        self.lib = lib or get(device)
        self.device = torch.device("cuda", device)
        self.cfg = cfg
        self._sizes = (C.c_int32 * len(sizes))(*[int(x) for x in sizes])
        c = N.SlotsCfg(len(sizes), C.cast(self._sizes, C.POINTER(C.c_int32)), int(hbm_budget),
                       int(max_slots), cfg.c(), _interim(interim), float(pixel_scale), int(profile),
                       float(spergel_nu), int(bool(pace)), float(ess_target), int(ess_every))
        self._stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        self.lib.check(self.lib.lib.bsi_slots_create(self.lib.h, C.byref(c),
                                                     C.c_void_p(self._stream.cuda_stream),
                                                     C.byref(h)), "bsi_slots_create")
        self.h = h
        self._keep = []          # stamps referenced by not yet advanced admissions

    def footprint(self, n: int) -> int:
        b = C.c_int64()
        self.lib.check(self.lib.lib.bsi_slots_footprint(self.h, int(n), C.byref(b)), "bsi_slots_footprint")
        return int(b.value)

    def admit(self, rid: int, stamp: torch.Tensor, psf_fwhm: float, sigma: float, ref_xy, init) -> bool:
        n = int(round(math.sqrt(stamp.numel())))
        assert stamp.is_cuda and stamp.dtype == torch.float32 and stamp.is_contiguous()
        ini = np.ascontiguousarray(np.asarray(init, dtype=np.float32).reshape(self.cfg.n_chains, 6))
        r = N.Request(int(rid), n, stamp.data_ptr(), float(psf_fwhm), float(sigma), float(ref_xy[0]),
                      float(ref_xy[1]), ini.ctypes.data_as(C.POINTER(C.c_float)))
        ok = C.c_int32(0)
        self.lib.check(self.lib.lib.bsi_slots_admit(self.h, C.byref(r), C.byref(ok)), "bsi_slots_admit")
        if ok.value:
            self._keep.append(stamp)
        return bool(ok.value)

    # numpy view of bsi_request (same field offsets as the C struct)
    REQUEST_DTYPE = np.dtype({"names": ["id", "n", "stamp", "psf_fwhm", "sigma", "ref_x", "ref_y", "init"],
                              "formats": [np.uint64, np.int32, np.uint64, np.float32, np.float32,
                                          np.float32, np.float32, np.uint64],
                              "offsets": [N.Request.id.offset, N.Request.n.offset, N.Request.stamp.offset,
                                          N.Request.psf_fwhm.offset, N.Request.sigma.offset,
                                          N.Request.ref_x.offset, N.Request.ref_y.offset,
                                          N.Request.init.offset],
                              "itemsize": C.sizeof(N.Request)})

    def admit_many(self, reqs: np.ndarray, keep=None) -> int:
        """Admit requests (a REQUEST_DTYPE array) in order until one does not
        fit; returns how many were admitted.  `keep` holds whatever owns the
        stamps and start positions until the next advance has run."""
        reqs = np.ascontiguousarray(reqs, dtype=self.REQUEST_DTYPE)
        n = C.c_int32(0)
        self.lib.check(self.lib.lib.bsi_slots_admit_many(self.h, int(reqs.shape[0]),
                                                         C.c_void_p(reqs.ctypes.data), C.byref(n)),
                       "bsi_slots_admit_many")
        if n.value and keep is not None:
            self._keep.append(keep)
        return int(n.value)

    def advance(self, n_iter: int):
        self.lib.check(self.lib.lib.bsi_slots_advance(self.h, int(n_iter)), "bsi_slots_advance")
        self._keep_prev, self._keep = self._keep, []

    def poll(self) -> int:
        """Wait for the server's work; number of finished, unharvested requests."""
        n = C.c_int32(0)
        self.lib.check(self.lib.lib.bsi_slots_poll(self.h, C.byref(n)), "bsi_slots_poll")
        return int(n.value)

    def harvest(self, max_n: int, want_samples: bool = True):
        """(ids [n] uint64 numpy, samples [n, C, S, 6], chain_stats [n, C, 4],
        status [n], n_draws [n]); draws past a request's n_draws are NaN."""
        Cn, S = self.cfg.n_chains, self.cfg.n_samples
        smp = torch.empty(max_n, Cn, S, 6, dtype=torch.float32, device=self.device) if want_samples else None
        st = torch.empty(max_n, Cn, 4, dtype=torch.float32, device=self.device)
        stat = torch.empty(max_n, dtype=torch.int32, device=self.device)
        nd = torch.empty(max_n, dtype=torch.int32, device=self.device)
        ids = (C.c_uint64 * max(max_n, 1))()
        n = C.c_int32(0)
        self.lib.check(self.lib.lib.bsi_slots_harvest(self.h, int(max_n), ids, _ptr(smp), _ptr(st),
                                                      _ptr(stat), _ptr(nd), C.byref(n)),
                       "bsi_slots_harvest")
        k = n.value
        self._keep_prev = []
        out_ids = np.array(ids[:k], dtype=np.uint64)
        return out_ids, (smp[:k] if smp is not None else None), st[:k], stat[:k], nd[:k]

    def info(self) -> dict:
        i = N.SlotsInfo()
        self.lib.check(self.lib.lib.bsi_slots_get_info(self.h, C.byref(i)), "bsi_slots_get_info")
        return {f: getattr(i, f) for f, _ in N.SlotsInfo._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.lib.bsi_slots_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_plan(n: int, P: int, lib: Library | None = None):
    """Slot plan P for stamp side n on the handle (0 = default)."""
    lib = lib or get()
    lib.check(lib.lib.bsi_set_plan(lib.h, int(n), int(P)), "bsi_set_plan")


def get_plan(n: int, lib: Library | None = None):
    """(P, slots) of stamp side n on the handle."""
    lib = lib or get()
    P, sl = C.c_int32(), C.c_int32()
    lib.check(lib.lib.bsi_get_plan(lib.h, int(n), C.byref(P), C.byref(sl)), "bsi_get_plan")
    return P.value, sl.value


def autotune(sizes, n_chains: int = 4, lib: Library | None = None):
    """Measure the candidate slot plans of each size and keep the fastest:
    {N: (P, ms per 20-step launch or None when there was one candidate)}."""
    lib = lib or get()
    n = len(sizes)
    sz = (C.c_int32 * max(n, 1))(*[int(x) for x in sizes])
    ch = (C.c_int32 * max(n, 1))()
    ms = (C.c_float * max(n, 1))()
    lib.check(lib.lib.bsi_autotune(lib.h, n, sz, int(n_chains), ch, ms), "bsi_autotune")
    return {int(sizes[i]): (int(ch[i]), float(ms[i]) if ms[i] >= 0 else None) for i in range(n)}


def set_transform(n: int, method: int, lib: Library | None = None):
    """Render transform for stamp side n (N.TRANSFORM_*; DEFAULT resets)."""
    lib = lib or get()
    lib.check(lib.lib.bsi_set_transform(lib.h, int(n), int(method)), "bsi_set_transform")


def get_transform(n: int, lib: Library | None = None) -> int:
    lib = lib or get()
    m = C.c_int32()
    lib.check(lib.lib.bsi_get_transform(lib.h, int(n), C.byref(m)), "bsi_get_transform")
    return int(m.value)


def autotune_transform(sizes, n_gal: int = 10000, lib: Library | None = None):
    """Time both transforms per size (render and forward DFT of n_gal stamps)
    and keep the faster: {N: (method, ms render direct, render MFMA, forward
    direct, forward MFMA)}."""
    lib = lib or get()
    n = len(sizes)
    sz = (C.c_int32 * max(n, 1))(*[int(x) for x in sizes])
    ch = (C.c_int32 * max(n, 1))()
    ms = (C.c_float * max(4 * n, 4))()
    lib.check(lib.lib.bsi_autotune_transform(lib.h, n, sz, int(n_gal), ch, ms), "bsi_autotune_transform")
    return {int(sizes[i]): (int(ch[i]), *[float(ms[4 * i + m]) for m in range(4)]) for i in range(n)}


def reserve(max_stamps: int = 0, max_n: int = 8, max_chains: int = 0, weighted: bool = False,
            pixel_method: bool = False, max_shear_gal: int = 0, max_points: int = 0, bias: bool = False,
            max_boot: int = 0, lib: Library | None = None):
    """bsi_reserve: size the handle's workspace so that calls within the
    limits neither allocate nor fail under graph capture."""
    lib = lib or get()
    cfg = N.ReserveCfg(int(max_stamps), int(max_n), int(max_chains), int(bool(weighted)),
                       int(bool(pixel_method)), int(max_shear_gal), int(max_points), int(bool(bias)),
                       int(max_boot))
    lib.check(lib.lib.bsi_reserve(lib.h, C.byref(cfg)), "bsi_reserve")


def ess(samples: torch.Tensor, lib: Library | None = None, split: bool = False):
    """(ESS [G, P], R-hat [G, P]) of samples [G, C, S, P]; with split=True
    also the split R-hat [G, P] as a third element."""
    dev = samples.device
    lib = lib or get(dev.index or 0)
    samples = samples.contiguous().float()
    G, Cn, S, P = samples.shape
    e = torch.empty(G, P, dtype=torch.float32, device=dev)
    r = torch.empty(G, P, dtype=torch.float32, device=dev)
    rs = torch.empty(G, P, dtype=torch.float32, device=dev) if split else None
    lib.check(lib.lib.bsi_ess(lib.h, G, Cn, S, P, _ptr(samples), _ptr(e), _ptr(r), _ptr(rs),
                              _stream(dev)), "bsi_ess")
    return (e, r, rs) if split else (e, r)
