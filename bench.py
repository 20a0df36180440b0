"""Benchmark: galaxies/s at 300 effective samples on the batched uniform
workload (10,000 galaxies, 53x53 stamps, PSF FWHM 0.7", 4 chains, 20 leapfrog
steps, 300 dual-averaging warmup iterations + 1,000 draws), one MI355X.

One step = the whole hot path on one synthetic batch: data transform, chain
initialisation, warmup + sampling (one persistent launch per trajectory,
replayed from a HIP graph), ESS/R-hat, and the shear posterior of the interim
samples on a 41x41 grid.  Time per galaxy follows Section 4.1:
    T_warmup / G + T_sampling / (G * n_eff) * 300,
with T_warmup from a warmup-only call and T_sampling = T_hmc - T_warmup.

Prints one JSON line (rank 0).  `--gpus` above 1 is rejected: the benchmark
runs on one GPU (the sharding across GPUs is a design, not code).
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from workloads import gen  # noqa: E402

TARGET_ESS = 300.0
PS = gen.PIXEL_SCALE


FP32_PEAK_TFLOPS = 157.3      # MI355X published FP32 peak (vector, packed / matrix)
VALU_ISSUE_TFLOPS = 78.6      # one wave64 FMA per CU per cycle (non-packed issue): 256 x 64 x 2 x 2.4 GHz
CLOCK_HZ = 2.4e9
N_CU = 256


def half_plane_bins(N: int) -> int:
    """Distinct bins of the Hermitian half plane (the even-N Nyquist bins combined)."""
    return (N * N + 1) // 2 if N % 2 else N * N // 2 + 2


def flops_per_eval(N: int, L: int = 20, chi2_every_step: bool = False, weighted: bool = False) -> float:
    """Algorithmic float32 operations of one gradient evaluation in the k-space
    form, counted from the trajectory kernel's pair loop as it executes (an FMA
    counts 2; a reciprocal square root, logarithm or exponential 1).

    One pair of bins (+kx, ky), (-kx, ky) costs 62 operations for the gradient:
    the two profile arguments 6, the profile powers G and G/(1 + r0^2 q) 8 (two
    rsqrt and three products each; the Spergel form's log2/exp2 pair costs the
    same), the separable factors X Y and conj(X) Y 10, the residuals 8,
    conj(R) X Y 12, and the shape and centroid accumulations 18 (the flux sum
    is not accumulated: it follows from the shape sums after the loop).  Sum
    |R|^2 adds 8 per pair; fixed-length HMC forms it on the last leapfrog step
    of a trajectory only (1 in L evaluations), NUTS on every step.  Stationary
    noise weights scale the two bins' G factors: 4 more per pair.  Per bin
    that is 31 (+4 for Sum |R|^2, +2 for the weights), counted over the
    distinct half-plane bins (the lane layout's duplicated column-0 and
    padding slots are not counted).  Per evaluation also: the separable
    PSF-sinc-phase tables (6 per x frequency, 8 per row), the per-column
    constants and post-loop sums and products (10 per column), and 152 for
    the shape constants, the flux sum, reductions, gradient assembly, prior
    and leapfrog update."""
    h = N // 2
    per_bin = 31.0 + (4.0 if chi2_every_step else 4.0 / L) + (2.0 if weighted else 0.0)
    return per_bin * half_plane_bins(N) + 6.0 * (2 * h + 1) + 8.0 * (h + 1) + 10.0 * (h + 1) + 152.0


KERNEL_SOURCES = {
    "hmc": ("hmc.hip", "kspace.h", "bsi_device.h", "bsi_kernels.h"),
    "shear": ("shear.hip", "bsi_device.h", "bsi_kernels.h"),
}


def kernel_source_hash(kernel: str = "hmc") -> str:
    """Digest of the sources a kernel is compiled from (its profile's key)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(f.encode())
        h.update(open(os.path.join(ROOT, "paper_2604_22048_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def recorded_counter(profile="hmc_kernel_uniform53.txt", kernel="hmc", key="traffic_bytes_per_launch"):
    """A per-launch figure from a committed counter summary (key: value lines),
    or None when the kernel's sources have changed since the counters were
    taken or the summary lacks the key."""
    path = os.path.join(ROOT, "profiles", profile)
    try:
        kv = dict(line.split(": ", 1) for line in open(path).read().splitlines() if ": " in line)
    except OSError:
        return None
    if kv.get("source_sha256", "").strip() != kernel_source_hash(kernel) or key not in kv:
        return None
    return float(kv[key])


def recorded_traffic(profile="hmc_kernel_uniform53.txt", kernel="hmc"):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None."""
    return recorded_counter(profile, kernel, "traffic_bytes_per_launch")


def valu_issue_frac(launch_s, profile="hmc_kernel_uniform53.txt", kernel="hmc"):
    """Wave64 VALU instructions issued per CU per cycle (the non-packed issue
    ceiling is 1): the counter summary's SQ_INSTS_VALU per launch over the
    live launch duration at 2.4 GHz, or None."""
    n = recorded_counter(profile, kernel, "valu_insts_per_launch")
    return None if n is None else round(n / N_CU / (launch_s * CLOCK_HZ), 4)


def executed_frac(launch_s, profile="hmc_kernel_uniform53.txt", kernel="hmc"):
    """FP32 flops the hardware counted per launch (SQ_INSTS_VALU_FLOPS_FP32,
    in units of 64 lane-flops, from the counter summary) over the live launch
    duration, as a fraction of the FP32 peak, or None.  It exceeds the
    algorithmic fraction by the work the count leaves out (padding lanes,
    per-chain work every lane of a chain repeats)."""
    n = recorded_counter(profile, kernel, "fp32_flops_executed_per_launch")
    return None if n is None else round(n / launch_s / 1e12 / FP32_PEAK_TFLOPS, 4)


# ---------------------------------------------------------------- CPU baseline
def _oracle_chain(args):
    """One single-threaded float64 oracle chain on one galaxy of a workload:
    (stamp side, seconds, gradient evaluations)."""
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)            # one BLAS thread per worker process
    name, idx, n_warmup, n_samples, size = args
    from oracle import hmc, render, shear
    cfg = gen.CONFIGS[name]
    t = gen.draw_truth(cfg, n_gal=1, seed=gen.data_seed(cfg.index) + 1000 + idx,
                       size_override=None if size is None else np.array([size]))
    ep = shear.shear_forward(t.e1 + 1j * t.e2, complex(*cfg.g_true))
    prm = np.array([t.flux[0], t.hlr[0], ep.real[0], ep.imag[0], t.dx[0], t.dy[0]])
    rng = np.random.default_rng(idx)
    N = int(t.n_pix[0])
    d = render.render_one(prm, N, PS, t.psf_fwhm[0]) + rng.normal(0, 1, (N, N))
    gal = hmc.Galaxy(data=d, N=N, pixel_scale=PS, psf_fwhm=float(t.psf_fwhm[0]), sigma=1.0,
                     ref_xy=(float(t.dx[0]), float(t.dy[0])))
    th0 = hmc.init_chain(d, 1.0, math.log10(prm[1]), (prm[2], prm[3]), 7, idx)
    t0 = time.perf_counter()
    if cfg.adapt:
        hmc.run_chain(hmc.galaxy_potential(gal), th0, 7, idx, cfg.leapfrog, n_warmup, n_samples, 0.01,
                      adapt=True, jitter=0.2)
    else:
        hmc.run_chain(hmc.galaxy_potential(gal), th0, 7, idx, cfg.leapfrog, n_warmup, n_samples,
                      cfg.step_size, adapt=False)
    return N, time.perf_counter() - t0, (n_warmup + n_samples) * cfg.leapfrog


CPU_ITERS = 600     # per worker: about 15 s of oracle work
# Worker processes for the oracle baseline: one per usable core, at most 16,
# the host cores that come with one GPU when a node's cores are divided among
# its GPUs (the affinity mask of a process can list the whole host).
CPU_WORKER_CAP = 16
UNEVEN_ORACLE_GAL = 16      # oracle chains per size class of the uneven mix
UNEVEN_ORACLE_ITERS = 20    # warmup iterations each (bounded sample)


def oracle_workers() -> int:
    return min(len(os.sched_getaffinity(0)), CPU_WORKER_CAP)


def oracle_pool(tasks):
    """Oracle chains [(workload, index, warmup, draws, side or None)] on one
    single-threaded worker process per usable core (CPU_WORKER_CAP at most).
    Forks, so it runs before the process touches the GPU.  Returns (results,
    cores, wall seconds)."""
    import multiprocessing as mp
    cores = oracle_workers()
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_chain, tasks, chunksize=1)
    return res, cores, time.perf_counter() - t0


def cpu_baseline_eval_rate(n_iter=CPU_ITERS):
    """Oracle gradient evaluations per second on the host for the uniform
    workload: one 53-pixel warmup chain of n_iter iterations per worker."""
    res, cores, wall = oracle_pool([("uniform", i, n_iter, 0, None) for i in range(oracle_workers())])
    evals = sum(r[2] for r in res)
    return evals / wall, cores, evals, wall


def cpu_oracle_per_size(name="uneven", n_gal=UNEVEN_ORACLE_GAL, n_iter=UNEVEN_ORACLE_ITERS):
    """Oracle seconds per gradient evaluation on one core for each stamp size
    of the mixed-size workloads: n_gal galaxies of each size from the
    workload's distributions, n_iter warmup iterations each."""
    tasks = [(name, 100 * N + i, n_iter, 0, N) for N in gen.SIZE_CLASSES for i in range(n_gal)]
    res, cores, wall = oracle_pool(tasks)
    sec = {N: 0.0 for N in gen.SIZE_CLASSES}
    ev = {N: 0 for N in gen.SIZE_CLASSES}
    for N, s_, e_ in res:
        sec[N] += s_
        ev[N] += e_
    return {"s_per_eval": {N: sec[N] / ev[N] for N in gen.SIZE_CLASSES}, "evals": sum(ev.values()),
            "cores": cores, "wall": wall,
            "sample": f"{n_gal} galaxies per stamp size (25/41/53/73/101 px), one {n_iter}-iteration "
                      f"warmup chain of {gen.CONFIGS[name].leapfrog} leapfrog steps each"}


def cpu_oracle_tiny():
    """The plain tiny workload in full on the oracle: every galaxy's whole
    chain (burn-in and draws), one galaxy per worker."""
    cfg = gen.CONFIGS["tiny"]
    res, cores, wall = oracle_pool([("tiny", i, cfg.warmup, cfg.samples, None) for i in range(cfg.n_gal)])
    evals = sum(r[2] for r in res)
    return {"s_per_eval": sum(r[1] for r in res) / evals, "evals": evals, "cores": cores, "wall": wall}


def mix_cpu_baseline(orc, weights, evals_per_gal, note):
    """cpu_baseline of a mixed-size workload from the oracle's per-size
    seconds per evaluation: cores / (the mix's mean oracle seconds per
    galaxy), with evals_per_gal[N] gradient evaluations per galaxy of side N."""
    tot = sum(weights.values())
    mean_s = sum(w * evals_per_gal[N] * orc["s_per_eval"][N] for N, w in weights.items()) / tot
    return {"value": round(orc["cores"] / mean_s, 6), "unit": "galaxies/s", "cores": orc["cores"],
            "kind": "oracle",
            "ms_per_eval_by_size": {N: round(v * 1e3, 4) for N, v in orc["s_per_eval"].items()},
            "s_per_galaxy_by_size": {N: round(evals_per_gal[N] * orc["s_per_eval"][N], 1) for N in weights},
            "sample": f"{orc['sample']} ({orc['evals']:,} evaluations in {orc['wall']:.1f} s); {note}"}


# ---------------------------------------------------------------- GPU workload
def lens(e1, e2, g):
    """Shear response of the reduced-shear ellipticity (simulation input)."""
    e = e1 + 1j * e2
    gg = complex(*g)
    ep = (e + gg) / (1.0 + np.conj(gg) * e)
    return ep.real, ep.imag


def make_inputs(api, torch, n_gal, cfg, seed_offset=0, sizes=None, chains=None, g=None):
    """Seeded synthetic galaxies of workload cfg rendered on the device, with
    pixel noise, reference centroids and chain starts (eq. initialize); g
    overrides the applied shear (same galaxies and noise)."""
    dev = torch.device("cuda:0")
    t = gen.draw_truth(cfg, n_gal=n_gal, seed=gen.data_seed(cfg.index) + seed_offset,
                       size_override=sizes)
    e1p, e2p = lens(t.e1, t.e2, cfg.g_true if g is None else g)
    params = np.stack([t.flux, t.hlr, e1p, e2p, t.dx, t.dy], axis=1).astype(np.float32)
    b = api.Batch(n=t.n_pix, psf_fwhm=torch.tensor(t.psf_fwhm, dtype=torch.float32, device=dev),
                  sigma=torch.tensor(t.sigma, dtype=torch.float32, device=dev), pixel_scale=PS)
    model = api.render_stamps(b, torch.tensor(params, device=dev))
    noise, off = gen.draw_noise(t, gen.data_seed(cfg.index) + 7 + seed_offset)
    data = (model + torch.tensor(noise, device=dev)).contiguous()
    # chain starts (eq. initialize): flux from the stamp sum, size and shape
    # jittered around the truth, centroid offsets zero
    rng = np.random.default_rng(gen.chain_seed(cfg.index) + seed_offset)
    npix = t.n_pix.astype(np.int64)
    cs = torch.cumsum(data.double(), 0)
    end = torch.tensor(off + npix * npix - 1, device=dev)
    start = torch.tensor(off - 1, device=dev)
    sums = (cs[end] - torch.where(start >= 0, cs[start.clamp(min=0)], torch.zeros_like(cs[end])))
    sums = sums.cpu().numpy()
    C = cfg.chains if chains is None else chains
    init = np.zeros((n_gal, C, 6), np.float32)
    init[:, :, 0] = np.log10(np.maximum(sums, t.sigma * npix))[:, None]
    init[:, :, 1] = np.log10(t.hlr)[:, None] + rng.uniform(-0.015, 0.015, (n_gal, C))
    for c in range(C):
        e1 = e1p + rng.uniform(-0.1, 0.1, n_gal)
        e2 = e2p + rng.uniform(-0.1, 0.1, n_gal)
        bad = e1 * e1 + e2 * e2 >= 0.95 ** 2
        e1[bad], e2[bad] = e1p[bad], e2p[bad]
        init[:, c, 2], init[:, c, 3] = e1, e2
    ref = torch.tensor(np.stack([t.dx, t.dy], 1), dtype=torch.float32, device=dev)
    return t, b, data, ref, torch.tensor(init, device=dev)


def timed(torch, fn, stream):
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record(stream)
    out = fn()
    e.record(stream)
    e.synchronize()
    return out, s.elapsed_time(e) * 1e-3


def shear_leg(api, torch, stream, smp, G, K, seed, cpu=False):
    """Shear-level HMC over (g1, g2, mu_ln_s, sigma_ln_s, sigma_e) on the
    interim samples of the uniform step (every 4th draw of the 4 chains: K =
    1000 per galaxy, 10^7 in all): 4 chains, 10 leapfrog steps, 500 warmup +
    3000 draws, and the HBM roofline of one evaluation pass."""
    th = smp[:, :, 3::4, :].reshape(G, K, 6)
    e1p, e2p, l10s = th[..., 2].contiguous(), th[..., 3].contiguous(), th[..., 1].contiguous()
    return shear_hmc_run(api, torch, stream, e1p, e2p, l10s, G, K, seed, cpu)


def shear_oracle_point(e1p, e2p, l10s, x):
    """The oracle's log posterior and gradient at one point x = (g1, g2,
    mu_ln_s, sigma_ln_s, sigma_e) over all samples, single process: (seconds,
    log posterior)."""
    from oracle import shear as oshear
    h = [v.cpu().numpy() for v in (e1p, e2p, l10s)]
    tpo = oshear.TruePrior(e_kind=1, e_max=0.7, size_term=True)
    t0 = time.perf_counter()
    lp, _ = oshear.log_posterior_grad((h[0], h[1], h[2], h[2]), complex(x[0], x[1]), tuple(x[2:]), tpo,
                                      oshear.Interim())
    return time.perf_counter() - t0, lp


def shear_hmc_run(api, torch, stream, e1p, e2p, l10s, G, K, seed, cpu=False):
    """The shear-level HMC leg on interim samples (e1', e2', log10 s) [G, K];
    cpu: also time the oracle at one point over all samples."""
    dev = torch.device("cuda:0")
    tp = api.TruePriorCfg(e_kind=1, e_max=0.7, size_term=True)
    dcfg = gen.CONFIGS["diff"].extra
    Cs = 4
    rng = np.random.default_rng(seed)
    x0 = np.array([0.0, 0.0, math.log(0.6), 0.3, 0.2]) + rng.normal(0, 0.003, (Cs, 5))
    cfg = api.ShearHmcConfig(n_chains=Cs, n_leapfrog=dcfg["shear_leapfrog"],
                             n_warmup=dcfg["shear_warmup"], n_samples=dcfg["shear_samples"],
                             adapt=True, step_size=1e-3, jitter=0.1, seed=seed)
    (ss, sst), t_tot = timed(torch, lambda: api.shear_hmc(e1p, e2p, l10s, None, tp, cfg, x0), stream)
    n_eval = 1 + (cfg.n_warmup + cfg.n_samples) * cfg.n_leapfrog
    e, rh = api.ess(ss.float()[None])
    ssn = ss.cpu().numpy()
    # one evaluation pass at the chains' final points, timed alone
    pts = torch.tensor(ssn[:, -1, :], dtype=torch.float64, device=dev)
    api.shear_posterior(e1p, e2p, l10s, None, pts, tp, want_grad=True)
    reps = 20
    _, t_pass = timed(torch, lambda: [api.shear_posterior(e1p, e2p, l10s, None, pts, tp, want_grad=True)
                                      for _ in range(reps)], stream)
    t_pass /= reps
    bytes_pass = G * K * 12.0                  # e1', e2', log10 s as float32
    gbs = bytes_pass / t_pass / 1e9
    out = {"n_gal": G, "K": K, "chains": Cs, "leapfrog": cfg.n_leapfrog, "warmup": cfg.n_warmup,
           "samples": cfg.n_samples, "t_s": round(t_tot, 4), "n_eval": n_eval,
           "us_per_eval": round(t_tot / n_eval * 1e6, 2),
           "g_mean": [round(float(ssn[..., 0].mean()), 5), round(float(ssn[..., 1].mean()), 5)],
           "g_sd": [round(float(ssn[..., 0].std()), 5), round(float(ssn[..., 1].std()), 5)],
           "g_true": list(gen.CONFIGS["uniform"].g_true),
           "ess_g": [round(float(e[0, 0]), 1), round(float(e[0, 1]), 1)],
           "rhat_max": round(float(rh.max()), 4),
           "accept_rate": round(float(sst[:, 0].mean()), 4),
           "eval_pass_us": round(t_pass * 1e6, 2),
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
                        "frac": round(gbs / 8000.0, 4),
                        "traffic": recorded_traffic("shear_kernel_diff_1e7.txt", "shear"),
                        "kernel": "shear_kernel + shear_reduce_kernel (4 points, with gradient)",
                        "alg_bytes_per_pass": bytes_pass}}
    if cpu:
        t_pt, _ = shear_oracle_point(e1p, e2p, l10s, ssn[0, -1, :])
        out["cpu_baseline"] = {
            "value": round(t_pt * Cs * n_eval, 1), "unit": "s", "cores": 1, "kind": "oracle",
            "s_per_point": round(t_pt, 3),
            "sample": f"one point (g, alpha) with gradient over all {G * K:,} samples on one core "
                      f"in {t_pt:.2f} s; the run = {n_eval:,} passes x {Cs} points"}
    return out


def render_flops(N):
    """(algorithmic, executed) flops of one stamp's render as two dense DFT
    products: pass 1 complex (rows v = 0..h) x (u = -h..h) x (x), 8 flops per
    complex multiply-add; pass 2 real, 4 flops per (y, x, v).  Executed: the
    MFMA tiles the kernel issues (16 x 16 x 4, 2048 flops each), padding
    included."""
    h = N // 2
    ntab, nrow = 2 * h + 1, h + 1
    alg = 8 * nrow * ntab * N + 4 * N * N * nrow
    ldT, nrow4, Np = (ntab + 3) // 4 * 4, (nrow + 3) // 4 * 4, (N + 15) // 16 * 16
    n1 = ((nrow + 15) // 16) * (Np // 16) * (ldT // 4) * 4
    n2 = (Np // 16) ** 2 * (nrow4 // 4) * 2
    return alg, (n1 + n2) * 2048


def transform_leg(api, sizes=(25, 41, 53, 73, 101), n_gal=10_000):
    """Render of n_gal stamps per size with each transform (direct float64
    sums vs FP32 DFT-as-GEMM on MFMA), best of five, and the choice kept."""
    res = api.autotune_transform(list(sizes), n_gal=n_gal)
    out = {}
    for N, (m, t_d, t_m, f_d, f_m) in res.items():
        alg, exe = render_flops(N)
        out[N] = {"direct_ms": round(t_d, 4), "mfma_ms": round(t_m, 4),
                  "forward_direct_ms": round(f_d, 4), "forward_mfma_ms": round(f_m, 4),
                  "chosen": "mfma" if m == api.N.TRANSFORM_MFMA else "direct",
                  "mfma_alg_tflops": round(alg * n_gal / (t_m * 1e-3) / 1e12, 2),
                  "mfma_exec_tflops": round(exe * n_gal / (t_m * 1e-3) / 1e12, 2),
                  "mfma_exec_frac_fp32_peak": round(exe * n_gal / (t_m * 1e-3) / 157.3e12, 4)}
    return {"n_gal": n_gal, "by_size": out}


def shear_pass_leg(api, torch, stream, reps, G=10_000, K=1000):
    """One evaluation pass of the shear-level sampler (4 points with gradient)
    over G x K synthetic interim samples, repeated `reps` times without a
    graph (the counter runs profile this form)."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(gen.data_seed(3))
    e1p = (0.25 * torch.randn(G, K, generator=g, device=dev)).clamp(-0.9, 0.9)
    e2p = (0.25 * torch.randn(G, K, generator=g, device=dev)).clamp(-0.9, 0.9)
    l10s = math.log10(0.6) + 0.13 * torch.randn(G, K, generator=g, device=dev)
    tp = api.TruePriorCfg(e_kind=1, e_max=0.95, size_term=True)
    pts = torch.tensor([[0.02, 0.0, math.log(0.6), 0.3, 0.2], [0.0, 0.01, -0.5, 0.3, 0.21],
                        [0.01, -0.01, -0.55, 0.28, 0.2], [-0.01, 0.0, -0.5, 0.32, 0.19]],
                       dtype=torch.float64, device=dev)
    api.shear_posterior(e1p, e2p, l10s, None, pts, tp, want_grad=True)
    _, t = timed(torch, lambda: [api.shear_posterior(e1p, e2p, l10s, None, pts, tp, want_grad=True)
                                 for _ in range(reps)], stream)
    t /= reps
    by = G * K * 12.0
    return {"reps": reps, "pass_us": round(t * 1e6, 2), "alg_bytes_per_pass": by,
            "gb_per_s": round(by / t / 1e9, 1), "frac_hbm_peak": round(by / t / 8e12, 4)}


SERVING_SIZES = gen.SIZE_CLASSES


def make_request_pool(api, torch, per_size, seed_offset=0):
    """Device-resident request payloads per stamp size (serving workload)."""
    from paper_2604_22048_amd import serve
    cfg = gen.CONFIGS["serving"]
    P = {k: {} for k in ("stamps", "psf", "sigma", "ref", "init")}
    for N in SERVING_SIZES:
        t, b, data, ref, init = make_inputs(api, torch, per_size, cfg, seed_offset=seed_offset + N,
                                            sizes=np.full(per_size, N), chains=1)
        P["stamps"][N] = data.view(per_size, N * N)
        P["psf"][N] = t.psf_fwhm.astype(np.float32)
        P["sigma"][N] = t.sigma.astype(np.float32)
        P["ref"][N] = ref.cpu().numpy()
        P["init"][N] = np.ascontiguousarray(init.cpu().numpy())
    return serve.RequestPool(**P)


def serving_leg(api, torch, rate, window_s, cap_requests, seed, n_draws=1500, iters_per_tick=60,
                paced_iters_per_tick=15, budget=4 << 30, extra_rates=(), pace=True, split=4,
                ess_target=300.0, ess_every=60, log=None, oracle=None):
    """Poisson request stream at `rate` for `window_s` seconds of arrivals
    (sizes 25/41/53/73/101 with weights .3/.3/.2/.15/.05, 1 chain, 300
    warmup iterations of 20 leapfrog steps, then draws until the request's
    ESS reaches ess_target at a check every ess_every draws, at most n_draws),
    then the capacity: cap_requests requests all present at the start.
    The paced run advances paced_iters_per_tick base iterations per call (its
    per-size counts are scaled from them), the others iters_per_tick."""
    from paper_2604_22048_amd import serve
    cfg = gen.CONFIGS["serving"]
    hc = api.HmcConfig(n_chains=1, n_leapfrog=cfg.leapfrog, n_warmup=cfg.warmup, n_samples=n_draws,
                       adapt=True, metric=api.N.METRIC_FISHER, step_size=0.5, target_accept=0.8,
                       jitter=0.2, seed=gen.chain_seed(cfg.index))
    plans = api.autotune(list(SERVING_SIZES), n_chains=1)
    pool = make_request_pool(api, torch, 512)
    w = np.array(cfg.extra["size_weights"])

    def run(arr, tag, ess, paced, wpc=0):
        sizes = np.random.default_rng(seed + arr.shape[0]).choice(np.array(SERVING_SIZES),
                                                                  size=arr.shape[0], p=w)
        hc.waves_per_chain = wpc
        srv = api.Slots(list(SERVING_SIZES), hc, hbm_budget=budget, pace=paced, ess_target=ess_target,
                        ess_every=ess_every)
        r = serve.serve(srv, pool, arr, sizes, paced_iters_per_tick if paced else iters_per_tick, ess=ess,
                        progress=log)
        srv.close()
        if log:
            log(f"[serve] {tag}: {r.n_done} requests in {r.wall:.2f} s")
        return r, sizes

    def lat_stats(r):
        lat = r.latency[np.isfinite(r.latency)]
        return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
                "mean_ms": round(float(lat.mean()) * 1e3, 2)}

    # warm the kernels and the allocator
    run(np.zeros(64), "warm", False, False)
    n_req = int(rate * window_s)
    arr = gen.draw_requests(n_req, rate, gen.data_seed(cfg.index))
    r, sizes = run(arr, f"{rate:.0f}/s", True, False)
    em = r.ess_mean[np.isfinite(r.ess_mean)]
    by_size = lambda rr, sz: {int(N): round(float(np.nanpercentile(rr.latency[sz == N], 50)) * 1e3, 2)
                              for N in SERVING_SIZES}
    out = {"rate_req_per_s": rate, "window_s": window_s, "n_requests": n_req, "completed": r.n_done,
           "galaxies_per_s": round(r.n_done / r.wall, 1), **lat_stats(r),
           "max_resident": r.max_resident, "ticks": r.ticks, "iters_per_tick": iters_per_tick,
           "tick_ms": {"p50": round(float(np.percentile(r.tick_s, 50)) * 1e3, 3),
                       "p99": round(float(np.percentile(r.tick_s, 99)) * 1e3, 3),
                       "max": round(float(r.tick_s.max()) * 1e3, 1),
                       "n_over_20ms": int(np.sum(r.tick_s > 0.02))},
           "warmup": cfg.warmup, "ess_target": ess_target, "ess_every": ess_every,
           "max_draws": n_draws, "leapfrog": cfg.leapfrog,
           "draws_median": float(np.median(r.n_draws[r.n_draws > 0])),
           "draws_p99": float(np.percentile(r.n_draws[r.n_draws > 0], 99)),
           "frac_at_max_draws": round(float(np.mean(r.n_draws[r.n_draws > 0] >= n_draws)), 4),
           "slot_plans": {N: P for N, (P, _) in plans.items()},
           "ess_mean_median": round(float(np.median(em)), 1),
           "frac_ess_ge_300": round(float(np.mean(em >= 300.0)), 4),
           "p50_ms_by_size": by_size(r, sizes)}
    if oracle:
        # one request per size on one oracle core: its warmup and the median
        # number of draws this run needed
        epr = cfg.leapfrog * (cfg.warmup + out["draws_median"])
        cb = mix_cpu_baseline(oracle, dict(zip(SERVING_SIZES, w)), {N: epr for N in SERVING_SIZES},
                              "one request per size = warmup + the run's median draws; galaxies/s "
                              "= cores / the size-weighted mean request time on one core")
        cb["request_s_by_size"] = cb.pop("s_per_galaxy_by_size")
        out["cpu_baseline"] = cb
    if pace:
        rp, sp = run(arr, f"{rate:.0f}/s paced", False, True)
        out["paced_by_size"] = {"galaxies_per_s": round(rp.n_done / rp.wall, 1), **lat_stats(rp),
                                "ticks": rp.ticks, "iters_per_tick": paced_iters_per_tick,
                                "p50_ms_by_size": by_size(rp, sp)}
    if split:
        # chains split over waves run on the default slot plans
        for N in SERVING_SIZES:
            api.set_plan(N, 0)
        run(np.zeros(64), "warm split", False, False, split)
        rs, ss = run(arr, f"{rate:.0f}/s {split} waves per chain", False, False, split)
        for N, (P, _) in plans.items():
            api.set_plan(N, P)
        out["split_chains"] = {"waves_per_chain": split, "galaxies_per_s": round(rs.n_done / rs.wall, 1),
                               **lat_stats(rs), "ticks": rs.ticks, "p50_ms_by_size": by_size(rs, ss)}
    rc, _ = run(np.zeros(cap_requests), "capacity", False, False)
    cap = rc.n_done / rc.wall
    out["capacity_req_per_s"] = round(cap, 1)
    out["capacity_requests"] = cap_requests
    for frac in extra_rates:
        rr = frac * cap
        n2 = int(rr * window_s)
        r2, _ = run(gen.draw_requests(n2, rr, gen.data_seed(cfg.index) + 1), f"{frac:.1f}x capacity",
                    False, False)
        out[f"at_{frac:.1f}x_capacity"] = {"rate_req_per_s": round(rr, 1), "n_requests": n2,
                                           "galaxies_per_s": round(r2.n_done / r2.wall, 1),
                                           **lat_stats(r2)}
    return out


def tiny_leg(api, torch, stream, log=None, oracle=None):
    """The plain tiny workload: 16 galaxies of 32 x 32, 1 chain, 10 leapfrog
    steps at the fixed step 0.005, 100 burn-in + 500 draws.  Batched (one
    launch per iteration, graph-replayed) and plain (one galaxy and one
    leapfrog step per launch, run in full), galaxies/s at 300 ESS for both,
    then the 41 x 41 shear grid on [-0.25, 0.25]^2 over the draws."""
    cfg = gen.CONFIGS["tiny"]
    say = log or (lambda m: None)
    G, C, L, W, S = cfg.n_gal, cfg.chains, cfg.leapfrog, cfg.warmup, cfg.samples
    t, b, data, ref, init = make_inputs(api, torch, G, cfg)
    hcfg = api.HmcConfig(n_chains=C, n_leapfrog=L, n_warmup=W, n_samples=S, adapt=False,
                         step_size=cfg.step_size, use_graph=True, seed=gen.chain_seed(cfg.index))
    wcfg = api.HmcConfig(**{**hcfg.__dict__, "n_samples": 0})
    pcfg = api.HmcConfig(**{**hcfg.__dict__, "form": api.N.FORM_PLAIN, "use_graph": False})
    api.hmc_sample(b, data, ref, init, hcfg)                               # warm
    (smp, st, status), t_hmc = timed(torch, lambda: api.hmc_sample(b, data, ref, init, hcfg), stream)
    _, t_w = timed(torch, lambda: api.hmc_sample(b, data, ref, init, wcfg, want_samples=False), stream)
    (psmp, _, _), t_plain = timed(torch, lambda: api.hmc_sample(b, data, ref, init, pcfg), stream)
    say(f"[tiny] batched {t_hmc:.3f} s, plain {t_plain:.3f} s")
    e, _ = api.ess(smp)
    n_eff = float(e.mean(dim=1).mean())
    t_s = t_hmc - t_w
    tpg = t_w / G + t_s / (G * n_eff) * TARGET_ESS
    plain_tpg = t_plain / (G * (W + S)) * (W + S * TARGET_ESS / n_eff)
    n1 = cfg.extra["grid_n"]
    gs = np.linspace(cfg.extra["grid_lo"], cfg.extra["grid_hi"], n1)
    pts = torch.tensor([[a, bb, math.log(0.6), 0.3, 0.2] for bb in gs for a in gs], dtype=torch.float64,
                       device=data.device)
    th = smp.reshape(G, C * S, 6)
    tp = api.TruePriorCfg(e_kind=1, e_max=0.7, size_term=True)
    grid = lambda: api.shear_posterior(th[..., 2].contiguous(), th[..., 3].contiguous(),
                                       th[..., 1].contiguous(), None, pts, tp)
    grid()
    lp, t_grid = timed(torch, grid, stream)
    lpn = lp.cpu().numpy().reshape(n1, n1)
    wgt = np.exp(lpn - lpn.max())
    G1, G2 = np.meshgrid(gs, gs)
    out = {"n_gal": G, "stamp": cfg.n_pix, "chains": C, "leapfrog": L, "step_size": cfg.step_size,
           "burn_in": W, "samples": S, "t_hmc_s": round(t_hmc, 4), "t_burn_in_s": round(t_w, 4),
           "t_plain_s": round(t_plain, 4), "plain_launches": G * (W + S) * L,
           "plain_equals_batched": bool(torch.equal(smp, psmp)),
           "n_eff_mean": round(n_eff, 1), "galaxies_per_s": round(1.0 / tpg, 2),
           "plain_galaxies_per_s": round(1.0 / plain_tpg, 2),
           "accept_rate": round(float(st[..., 0].mean()), 4),
           "grid": f"{n1}x{n1}", "t_grid_s": round(t_grid, 5),
           "g_mean": [round(float((wgt * G1).sum() / wgt.sum()), 5),
                      round(float((wgt * G2).sum() / wgt.sum()), 5)]}
    if oracle:
        epg = C * L * (W + S * TARGET_ESS / n_eff)
        out["cpu_baseline"] = {
            "value": round(oracle["cores"] / (epg * oracle["s_per_eval"]), 6), "unit": "galaxies/s",
            "cores": oracle["cores"], "kind": "oracle",
            "sample": f"the whole workload: {G} chains of {W} + {S} iterations, one per galaxy "
                      f"({oracle['evals']:,} evaluations, {oracle['wall']:.1f} s wall on "
                      f"{oracle['cores']} cores); galaxies/s with the GPU run's n_eff"}
    return out


def uneven_leg(api, torch, stream, n_gal, log=None, per_size_runs=True, oracle=None):
    """Batched uneven workload: n_gal galaxies, stamp side from the size rule
    (25-101), PSF FWHM ~ U(0.6, 0.9), SNR 10-200, 4 chains, 20 leapfrog
    steps, 300 warmup + 1000 draws.  Timed in the direct form (each
    iteration's per-size launches concurrent on forked streams), and in the
    graph form (the per-size launches in sequence, replayed from a graph) for
    comparison.  per_size_runs: also time each size class alone
    (uneven_per_size)."""
    cfg = gen.CONFIGS["uneven"]
    say = log or (lambda m: None)
    plans = api.autotune(list(gen.SIZE_CLASSES), n_chains=cfg.chains)
    say(f"[uneven] plans {plans}")
    t, b, data, ref, init = make_inputs(api, torch, n_gal, cfg)
    say(f"[uneven] {n_gal} galaxies rendered")
    C, L, W, S = cfg.chains, cfg.leapfrog, cfg.warmup, cfg.samples
    hcfg = api.HmcConfig(n_chains=C, n_leapfrog=L, n_warmup=W, n_samples=S, adapt=True,
                         metric=api.N.METRIC_FISHER, step_size=0.5, target_accept=0.8, jitter=0.2,
                         use_graph=True, seed=gen.chain_seed(cfg.index))
    dcfg = api.HmcConfig(**{**hcfg.__dict__, "use_graph": False})
    run = lambda cfg_, n_s, want: api.hmc_sample(b, data, ref, init,
                                                 api.HmcConfig(**{**cfg_.__dict__, "n_samples": n_s}),
                                                 want_samples=want)
    run(hcfg, 0, False)                                                # warm
    run(dcfg, 0, False)
    (smp, st, status), t_hmc = timed(torch, lambda: run(dcfg, S, True), stream)
    say(f"[uneven] sampler call {t_hmc:.3f} s (direct)")
    (e, rh), _ = timed(torch, lambda: api.ess(smp), stream)
    _, t_w = timed(torch, lambda: run(dcfg, 0, False), stream)
    _, t_hmc_g = timed(torch, lambda: run(hcfg, S, True), stream)
    _, t_w_g = timed(torch, lambda: run(hcfg, 0, False), stream)
    say(f"[uneven] sampler call {t_hmc_g:.3f} s (graph)")
    n_eff = float(e.mean(dim=1).mean())
    acc = st[..., 0].mean()
    n_flag = int((status != 0).sum())
    tpg = t_w / n_gal + (t_hmc - t_w) / (n_gal * n_eff) * TARGET_ESS
    tpg_g = t_w_g / n_gal + (t_hmc_g - t_w_g) / (n_gal * n_eff) * TARGET_ESS
    counts = {int(N): int(np.sum(t.n_pix == N)) for N in np.unique(t.n_pix)}
    flop = sum(flops_per_eval(N) * k for N, k in counts.items()) * C * L * (W + S)
    del smp, st, e, rh, data
    per_size = uneven_per_size(api, torch, stream, cfg, counts, hcfg, log=say) if per_size_runs else None
    out = {"n_gal": n_gal, "size_counts": counts, "slot_plans": {N: P for N, (P, _) in plans.items()},
           "launch_form": "direct (per-size launches concurrent on forked streams)",
           "t_hmc_s": round(t_hmc, 4), "t_warmup_s": round(t_w, 4),
           "n_eff_mean": round(n_eff, 1),
           "galaxies_per_s": round(1.0 / tpg, 1),
           "achieved_tflops": round(flop / t_hmc / 1e12, 3),
           "frac_fp32_peak": round(flop / t_hmc / 1e12 / FP32_PEAK_TFLOPS, 4),
           "graph_form": {"t_hmc_s": round(t_hmc_g, 4), "t_warmup_s": round(t_w_g, 4),
                          "galaxies_per_s": round(1.0 / tpg_g, 1)},
           "accept_rate": round(float(acc), 4),
           "status_nonzero": n_flag,
           "per_size": per_size}
    if oracle:
        epg = C * L * (W + S * TARGET_ESS / n_eff)
        out["cpu_baseline"] = mix_cpu_baseline(
            oracle, counts, {N: epg for N in counts},
            "galaxies/s = cores / the mix's mean oracle seconds per galaxy at 300 ESS with the GPU "
            "run's n_eff")
    return out


def uneven_per_size(api, torch, stream, cfg, counts, hcfg, n1=20, n2=60, log=None):
    """Trajectory-kernel time per launch of each size class of the uneven
    batch, alone on the device: a batch of that many galaxies of that size
    (drawn from the uneven population with the stamp side forced), timed as
    the difference of two warmup-only calls of n2 and n1 iterations (one
    launch per iteration, replayed from a graph), so that the chain start and
    data transform cancel.  Fractions use the algorithmic flop count per
    evaluation of that size."""
    out = {}
    for N, k in sorted(counts.items()):
        t, b, data, ref, init = make_inputs(api, torch, k, cfg, seed_offset=1000 + N,
                                            sizes=np.full(k, N, dtype=np.int32))
        ts = []
        for n in (n1, n2):
            c = api.HmcConfig(**{**hcfg.__dict__, "n_warmup": n, "n_samples": 0})
            api.hmc_sample(b, data, ref, init, c, want_samples=False)          # warm
            _, dt = timed(torch, lambda: api.hmc_sample(b, data, ref, init, c, want_samples=False),
                          stream)
            ts.append(dt)
        t_launch = (ts[1] - ts[0]) / (n2 - n1)
        tf = flops_per_eval(N, hcfg.n_leapfrog) * k * hcfg.n_chains * hcfg.n_leapfrog / t_launch / 1e12
        if log:
            log(f"[uneven] {N} px alone: {t_launch * 1e3:.4f} ms per launch")
        out[N] = {"n_gal": k, "launch_ms": round(t_launch * 1e3, 4), "achieved_tflops": round(tf, 3),
                  "frac_fp32_peak": round(tf / FP32_PEAK_TFLOPS, 4),
                  "frac_of_nonpacked_issue_ceiling": round(tf / VALU_ISSUE_TFLOPS, 4)}
        del t, b, data, ref, init
    return out


def spergel_leg(api, torch, stream, n_gal, nu, log=None):
    """Model-bias fit (Appendix B): the uniform workload's exponential galaxies
    (53-pixel stamps) fitted with a Spergel profile of fixed index nu, same
    sampler settings as the headline line."""
    cfg = gen.CONFIGS["uniform"]
    t, b, data, ref, init = make_inputs(api, torch, n_gal, cfg)
    bs = api.Batch(n=b.n, psf_fwhm=b.psf_fwhm, sigma=b.sigma, pixel_scale=b.pixel_scale,
                   profile=api.N.PROFILE_SPERGEL, spergel_nu=nu)
    C, L, W, S = cfg.chains, cfg.leapfrog, cfg.warmup, cfg.samples
    hcfg = api.HmcConfig(n_chains=C, n_leapfrog=L, n_warmup=W, n_samples=S, adapt=True,
                         metric=api.N.METRIC_FISHER, step_size=0.5, target_accept=0.8, jitter=0.2,
                         use_graph=True, seed=gen.chain_seed(cfg.index))
    wcfg = api.HmcConfig(**{**hcfg.__dict__, "n_samples": 0})
    api.hmc_sample(bs, data, ref, init, wcfg, want_samples=False)      # warm
    (smp, st, status), t_hmc = timed(torch, lambda: api.hmc_sample(bs, data, ref, init, hcfg), stream)
    (e, rh), _ = timed(torch, lambda: api.ess(smp), stream)
    _, t_w = timed(torch, lambda: api.hmc_sample(bs, data, ref, init, wcfg, want_samples=False), stream)
    n_eff = float(e.mean(dim=1).mean())
    t_s = t_hmc - t_w
    tpg = t_w / n_gal + t_s / (n_gal * n_eff) * TARGET_ESS
    flop = flops_per_eval(cfg.n_pix) * n_gal * C * L * (W + S)
    return {"n_gal": n_gal, "spergel_nu": nu, "t_hmc_s": round(t_hmc, 4), "t_warmup_s": round(t_w, 4),
            "n_eff_mean": round(n_eff, 1), "galaxies_per_s": round(1.0 / tpg, 1),
            "achieved_tflops": round(flop / t_hmc / 1e12, 3),
            "frac_fp32_peak": round(flop / t_hmc / 1e12 / FP32_PEAK_TFLOPS, 4),
            "accept_rate": round(float(st[..., 0].mean()), 4),
            "status_nonzero": int((status != 0).sum())}


def bias_leg(api, torch, stream, n_gal, n_boot, log, sampler="hmc", depth=5):
    """Multiplicative and additive shear bias by shape-noise cancellation with
    bootstrap errors (Section 3.5; Table 2's all-fixed setting): the uniform
    workload's galaxies and noise sheared by +g and by -g, every property
    sampled (4 chains, 300 warmup + 1000 draws; fixed-length HMC with 20
    leapfrog steps, or NUTS of the given maximum tree depth with all
    transitions in one launch), the shear phase with the population parameters
    at their true values on a 33 x 33 grid of g around each dataset's shear
    (K = 1000: every 4th draw), n_boot resamples of the galaxies."""
    import math
    cfg = gen.CONFIGS["uniform"]
    dev = torch.device("cuda:0")
    C, L, W, S = cfg.chains, cfg.leapfrog, cfg.warmup, cfg.samples
    if sampler == "nuts":
        hcfg = api.HmcConfig(n_chains=C, n_warmup=W, n_samples=S, adapt=True,
                             metric=api.N.METRIC_FISHER, step_size=0.5, target_accept=0.8,
                             iters_per_launch=W + S, use_graph=True, seed=gen.chain_seed(cfg.index),
                             sampler=api.N.SAMPLER_NUTS, max_tree_depth=depth)
    else:
        hcfg = api.HmcConfig(n_chains=C, n_leapfrog=L, n_warmup=W, n_samples=S, adapt=True,
                             metric=api.N.METRIC_FISHER, step_size=0.5, target_accept=0.8, jitter=0.2,
                             use_graph=True, seed=gen.chain_seed(cfg.index))
    g_abs = cfg.g_true[0]
    mu_f, sd_f = gen.flux_lognormal(*cfg.snr, cfg.sigma)
    tp = api.TruePriorCfg(e_kind=1, e_max=0.7, size_term=True, flux_term=True, mu_ln_f=mu_f,
                          sigma_ln_f=sd_f)
    alpha = (math.log(0.6), 0.3, 0.2)
    n1, half = 33, 0.03
    g1 = np.linspace(g_abs - half, g_abs + half, n1)
    g2 = np.linspace(-half, half, n1)
    G1, G2 = np.meshgrid(g1, g2)
    gpp = np.stack([G1.ravel(), G2.ravel()], axis=1)
    gpm = gpp * [-1.0, 1.0]
    K = 1000
    ells, t_hmc, t_ell, acc = [], [], [], []
    for sgn, gp in ((1.0, gpp), (-1.0, gpm)):
        t, b, data, ref, init = make_inputs(api, torch, n_gal, cfg, g=(sgn * g_abs, 0.0))
        (smp, st, status), th = timed(torch, lambda: api.hmc_sample(b, data, ref, init, hcfg), stream)
        thn = smp[:, :, 3::4, :].reshape(n_gal, K, 6)
        pts = np.array([[a, bb, *alpha] for a, bb in gp])
        ell, tl = timed(torch, lambda: api.shear_galaxy_loglik(thn[..., 2], thn[..., 3], thn[..., 1],
                                                               thn[..., 0], pts, tp), stream)
        ells.append(ell)
        t_hmc.append(th)
        t_ell.append(tl)
        acc.append(float(st[..., 0].mean()))
        log(f"[bench] bias: dataset g1 = {sgn * g_abs:+.2f}: hmc {th:.3f} s, shear table {tl:.3f} s")
    counts = torch.tensor(gen.bootstrap_counts(n_boot, n_gal, gen.chain_seed(cfg.index) + 5), device=dev)
    gps = torch.tensor(np.stack([gpp, gpm]), device=dev)
    api.shear_bias(ells[0], ells[1], gps, g_abs, counts)          # warm
    res, t_boot = timed(torch, lambda: api.shear_bias(ells[0], ells[1], gps, g_abs, counts), stream)
    st = res["stats"].cpu().numpy()
    P = n1 * n1
    boot_flop = 2.0 * (n_boot + 1) * 2 * P * n_gal
    total = sum(t_hmc) + sum(t_ell) + t_boot
    return {"n_gal": n_gal, "n_boot": n_boot, "grid": f"{n1}x{n1}", "K": K, "sampler": sampler,
            "m": float(st[0]), "c": float(st[1]), "m_err_3sigma": 3 * float(st[2]),
            "c_err_3sigma": 3 * float(st[3]),
            "t_hmc_s": [round(x, 4) for x in t_hmc], "t_shear_table_s": [round(x, 4) for x in t_ell],
            "t_bootstrap_s": round(t_boot, 5), "bootstrap_tflops": round(boot_flop / t_boot / 1e12, 3),
            "accept_rate": [round(a, 4) for a in acc], "t_total_s": round(total, 3),
            "galaxy_pairs_per_s": round(n_gal / total, 1)}


def nuts_leg(api, torch, stream, n_gal, depth, ipl, log):
    """The paper's sampler (Section 3.3: NUTS, maximum tree depth 5) on the
    uniform workload with the headline's warmup and draws, beside fixed-length
    HMC on the same galaxies: galaxies/s at 300 ESS, leapfrog steps per
    transition (from the per-iteration trace) and the kernels' algorithmic rate."""
    cfg = gen.CONFIGS["uniform"]
    t, b, data, ref, init = make_inputs(api, torch, n_gal, cfg)
    C, W, S = cfg.chains, cfg.warmup, cfg.samples
    dev = torch.device("cuda:0")
    ipl = ipl if ipl > 0 else W + S
    ncfg = api.HmcConfig(n_chains=C, n_warmup=W, n_samples=S, adapt=True,
                         metric=api.N.METRIC_FISHER, step_size=0.5, target_accept=0.8,
                         iters_per_launch=ipl, use_graph=True, seed=gen.chain_seed(cfg.index),
                         sampler=api.N.SAMPLER_NUTS, max_tree_depth=depth)
    wcfg = api.HmcConfig(**{**ncfg.__dict__, "n_samples": 0})
    trace = torch.zeros(n_gal, C, W + S, 4, dtype=torch.float32, device=dev)
    api.hmc_sample(b, data, ref, init, wcfg, want_samples=False)      # warm
    (smp, st, status), t_all = timed(torch, lambda: api.hmc_sample(b, data, ref, init, ncfg, trace=trace),
                                     stream)
    (e, rh), _ = timed(torch, lambda: api.ess(smp), stream)
    _, t_w = timed(torch, lambda: api.hmc_sample(b, data, ref, init, wcfg, want_samples=False), stream)
    n_eff = float(e.mean(dim=1).mean())
    t_s = t_all - t_w
    tpg = t_w / n_gal + t_s / (n_gal * n_eff) * TARGET_ESS
    nlf = trace[..., 1]
    steps = float(nlf.sum())
    steps_w = float(nlf[:, :, :W].sum())
    depth_hist = torch.bincount(trace[..., 3].reshape(-1).long(), minlength=depth + 1).cpu().tolist()
    flop = flops_per_eval(cfg.n_pix, chi2_every_step=True) * steps
    log(f"[bench] nuts: depth {depth}, {ipl} per launch: {t_all:.3f} s, {steps / (n_gal * C * (W + S)):.2f} "
        f"leapfrog steps per transition, n_eff {n_eff:.0f}")
    return {"n_gal": n_gal, "max_tree_depth": depth, "iters_per_launch": ipl,
            "t_sampler_s": round(t_all, 4), "t_warmup_s": round(t_w, 4), "n_eff_mean": round(n_eff, 1),
            "galaxies_per_s": round(1.0 / tpg, 1),
            "leapfrog_per_transition": round(steps / (n_gal * C * (W + S)), 3),
            "leapfrog_per_transition_sampling": round((steps - steps_w) / (n_gal * C * S), 3),
            "depth_histogram": depth_hist,
            "ess_per_gradient_eval": round(n_eff / ((steps - steps_w) / n_gal), 4),
            "achieved_tflops": round(flop / t_all / 1e12, 3),
            "frac_fp32_peak": round(flop / t_all / 1e12 / FP32_PEAK_TFLOPS, 4),
            "accept_stat_mean": round(float(trace[:, :, W:, 2].mean()), 4),
            "status_nonzero": int((status != 0).sum())}


def exposures_leg(api, torch, stream, n_gal, E, log, sampler="hmc", depth=5):
    """Appendix C likelihood: the uniform workload's galaxies (53-pixel stamps)
    each seen in E exposures with their own PSF FWHM ~ U(0.6", 0.9"), noise
    sigma ~ U(0.8, 1.2) and stationary correlated noise (exposure j: a 3 x 3
    correlation kernel shared by all galaxies), sampled with the headline
    settings on the 53-pixel kernels of the default plan (fixed-length HMC; or
    NUTS of the given maximum tree depth, all transitions in one launch)."""
    cfg = gen.CONFIGS["uniform"]
    dev = torch.device("cuda:0")
    N = cfg.n_pix
    rng = np.random.default_rng(gen.data_seed(cfg.index) + 31)
    t = gen.draw_truth(cfg, n_gal=n_gal, seed=gen.data_seed(cfg.index))
    e1p, e2p = lens(t.e1, t.e2, cfg.g_true)
    params = np.stack([t.flux, t.hlr, e1p, e2p, t.dx, t.dy], axis=1).astype(np.float32)
    S = n_gal * E
    n = np.full(S, N, np.int32)
    psf = rng.uniform(0.6, 0.9, S).astype(np.float32)
    sig = rng.uniform(0.8, 1.2, S).astype(np.float32)
    kern = [gen.noise_kernel_ps(rng, N) for _ in range(E)]
    ps = np.stack([kern[s % E][0] for s in range(S)]).astype(np.float32)       # [S, N, N]
    noise = np.empty((S, N, N), np.float32)
    for j in range(E):
        noise[j::E] = gen.correlated_noise(rng, kern[j][1], 1.0, n=n_gal) * sig[j::E, None, None]
    b = api.Batch(n=n, psf_fwhm=torch.tensor(psf, device=dev), sigma=torch.tensor(sig, device=dev),
                  pixel_scale=PS, n_exp=E, noise_ps=torch.tensor(ps.ravel(), device=dev))
    model = api.render_stamps(b, torch.tensor(params, device=dev))
    data = (model + torch.tensor(noise.ravel(), device=dev)).contiguous()
    del noise
    C, L, W, Sd = cfg.chains, cfg.leapfrog, cfg.warmup, cfg.samples
    init = np.zeros((n_gal, C, 6), np.float32)
    init[:, :, 0] = np.log10(t.flux)[:, None] + rng.uniform(-0.02, 0.02, (n_gal, C))
    init[:, :, 1] = np.log10(t.hlr)[:, None] + rng.uniform(-0.015, 0.015, (n_gal, C))
    init[:, :, 2] = e1p[:, None] + rng.uniform(-0.1, 0.1, (n_gal, C))
    init[:, :, 3] = e2p[:, None] + rng.uniform(-0.1, 0.1, (n_gal, C))
    init = torch.tensor(init, device=dev)
    ref = torch.tensor(np.stack([t.dx, t.dy], axis=1).astype(np.float32), device=dev)
    hcfg = api.HmcConfig(n_chains=C, n_leapfrog=L, n_warmup=W, n_samples=Sd, adapt=True,
                         metric=api.N.METRIC_FISHER, step_size=0.5, target_accept=0.8, jitter=0.2,
                         use_graph=True, seed=gen.chain_seed(cfg.index))
    if sampler == "nuts":
        hcfg = api.HmcConfig(**{**hcfg.__dict__, "sampler": api.N.SAMPLER_NUTS, "max_tree_depth": depth,
                                "iters_per_launch": W + Sd})
    wcfg = api.HmcConfig(**{**hcfg.__dict__, "n_samples": 0})
    api.hmc_sample(b, data, ref, init, wcfg, want_samples=False)      # warm
    (smp, st, status), t_hmc = timed(torch, lambda: api.hmc_sample(b, data, ref, init, hcfg), stream)
    (e, rh), _ = timed(torch, lambda: api.ess(smp), stream)
    _, t_w = timed(torch, lambda: api.hmc_sample(b, data, ref, init, wcfg, want_samples=False), stream)
    n_eff = float(e.mean(dim=1).mean())
    t_s = t_hmc - t_w
    tpg = t_w / n_gal + t_s / (n_gal * n_eff) * TARGET_ESS
    flop = flops_per_eval(N, L, weighted=True) * E * n_gal * C * L * (W + Sd) if sampler == "hmc" else None
    log(f"[bench] exposures: E = {E}, {sampler} {t_hmc:.3f} s, warmup {t_w:.3f} s, n_eff {n_eff:.0f}")
    return {"n_gal": n_gal, "n_exp": E, "sampler": sampler, "t_hmc_s": round(t_hmc, 4),
            "t_warmup_s": round(t_w, 4), "n_eff_mean": round(n_eff, 1), "galaxies_per_s": round(1.0 / tpg, 1),
            "achieved_tflops": round(flop / t_hmc / 1e12, 3) if flop else None,
            "frac_fp32_peak": round(flop / t_hmc / 1e12 / FP32_PEAK_TFLOPS, 4) if flop else None,
            "accept_rate": round(float(st[..., 0].mean()), 4),
            "status_nonzero": int((status != 0).sum())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-gal", type=int, default=None, help="override galaxy count (profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-gal", type=int, default=4)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES of device memory 4 times (calibrates HBM counters)")
    ap.add_argument("--workload", choices=["uniform", "uneven", "serving", "shear-pass", "shear-hmc",
                                           "spergel", "bias", "exposures", "nuts", "tiny"],
                    default="uniform",
                    help="uniform: the headline line (with shear-level HMC and serving legs); "
                         "uneven / serving: the mixed-size batch or the extended serving study")
    ap.add_argument("--no-legs", action="store_true", help="uniform workload without the shear and "
                    "serving legs (profiling)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg (profiling)")
    ap.add_argument("--serve-window", type=float, default=8.0, help="seconds of request arrivals")
    ap.add_argument("--n-boot", type=int, default=500, help="--workload bias: bootstrap resamples")
    ap.add_argument("--n-exp", type=int, default=4, help="--workload exposures: exposures per galaxy")
    ap.add_argument("--depth", type=int, default=5, help="--workload nuts / bias: maximum tree depth")
    ap.add_argument("--sampler", choices=["hmc", "nuts"], default="hmc",
                    help="--workload bias / exposures: per-galaxy sampler")
    ap.add_argument("--ipl", type=int, default=0,
                    help="--workload nuts: transitions per launch (0: all in one launch)")
    ap.add_argument("--spergel-nu", type=float, default=-0.6,
                    help="--workload spergel: the fixed Spergel index of the fit")
    ap.add_argument("--plan", type=int, default=0,
                    help="uniform workload: this slot plan P for the 53-pixel kernel instead of autotuning")
    ap.add_argument("--transform-only", action="store_true",
                    help="only the render-transform comparison (both transforms, workload sizes)")
    ap.add_argument("--shear-k", type=int, default=1000,
                    help="--workload shear-pass: interim samples per galaxy (above 1024: chunked)")
    ap.add_argument("--serve-requests", type=int, default=0,
                    help="--workload serving: this many Poisson requests at 2000/s (overrides "
                         "--serve-window; only the ESS-targeted run and the capacity are measured)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda:0")
        for _ in range(4):
            b = a.clone()
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "copies": 4}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    if args.transform_only:
        import torch
        from paper_2604_22048_amd import api
        torch.cuda.init()
        print(json.dumps({"transform": transform_leg(api)}), flush=True)
        return
    # oracle timings fork worker processes, so they run before anything
    # touches the GPU
    orc = {}
    if not args.no_cpu_baseline:
        legs_on = args.workload == "uniform" and not args.no_legs
        if args.workload in ("uneven", "serving") or legs_on:
            orc["sizes"] = cpu_oracle_per_size()
            log(f"[bench] oracle per size: {orc['sizes']['evals']} evaluations in "
                f"{orc['sizes']['wall']:.1f} s")
        if args.workload == "tiny" or legs_on:
            orc["tiny"] = cpu_oracle_tiny()
            log(f"[bench] oracle tiny workload: {orc['tiny']['evals']} evaluations in "
                f"{orc['tiny']['wall']:.1f} s")
    if args.workload != "uniform":
        import torch
        from paper_2604_22048_amd import api
        torch.cuda.init()
        stream = torch.cuda.current_stream(torch.device("cuda:0"))
        if args.workload == "shear-hmc":
            G, K = args.n_gal or 10_000, 1000
            S = [torch.tensor(a, device="cuda:0") for a in gen.draw_interim_samples(G, K, gen.data_seed(3))]
            shear_hmc_run(api, torch, stream, *S, G, K, gen.chain_seed(3))          # warm
            res = shear_hmc_run(api, torch, stream, *S, G, K, gen.chain_seed(3),
                                cpu=not args.no_cpu_baseline)
            out = {"metric": "shear-level HMC (500 warmup + 3000 draws, L = 10, 4 chains)",
                   "value": res["t_s"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
                   "dtype": "f32+f64", "data": "synthetic",
                   "config": {"workload": f"{G} galaxies x {K} stand-in interim samples"}, **res}
            print(json.dumps(out), flush=True)
            return
        if args.workload == "shear-pass":
            G = args.n_gal or 10_000
            K = args.shear_k
            res = shear_pass_leg(api, torch, stream, args.steps, G=G, K=K)
            out = {"metric": "shear posterior evaluation pass (4 points, with gradient)",
                   "value": res["gb_per_s"], "unit": "GB/s", "n_gpus": 1, "higher_is_better": True,
                   "dtype": "f32", "data": "synthetic",
                   "config": {"workload": f"{G:,} galaxies x {K:,} interim samples, 4 points"}, **res}
            print(json.dumps(out), flush=True)
            return
        if args.workload == "nuts":
            G = args.n_gal or gen.CONFIGS["uniform"].n_gal
            res = nuts_leg(api, torch, stream, G, args.depth, args.ipl, log)
            out = {"metric": "galaxies/sec at 300 ESS (NUTS, Section 3.3's sampler)",
                   "value": res["galaxies_per_s"], "unit": "galaxies/s", "n_gpus": 1,
                   "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                   "config": {"workload": f"batched uniform: {G} galaxies, 53x53, 4 chains, NUTS max "
                                          f"tree depth {args.depth}, 300 warmup + 1000 draws, "
                                          f"{res['iters_per_launch']} transitions per launch"}, **res}
        elif args.workload == "exposures":
            G = args.n_gal or gen.CONFIGS["uniform"].n_gal
            res = exposures_leg(api, torch, stream, G, args.n_exp, log, args.sampler, args.depth)
            out = {"metric": "galaxies/sec at 300 ESS (several exposures, correlated noise)",
                   "value": res["galaxies_per_s"], "unit": "galaxies/s", "n_gpus": 1,
                   "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                   "config": {"workload": f"{G} galaxies x {args.n_exp} exposures of 53 x 53, PSF FWHM "
                                          "U(0.6, 0.9)in, stationary correlated noise, 4 chains, "
                                          + ("20 leapfrog steps" if args.sampler == "hmc" else
                                             f"NUTS max tree depth {args.depth}")
                                          + ", 300 warmup + 1000 draws"}, **res}
        elif args.workload == "bias":
            G = args.n_gal or gen.CONFIGS["uniform"].n_gal
            res = bias_leg(api, torch, stream, G, args.n_boot, log, args.sampler, args.depth)
            out = {"metric": "m/c bias study by shape-noise cancellation (galaxy pairs/s, end to end)",
                   "value": res["galaxy_pairs_per_s"], "unit": "galaxy pairs/s", "n_gpus": 1,
                   "higher_is_better": True, "dtype": "f32+f64", "data": "synthetic",
                   "config": {"workload": f"{G} 53-pixel galaxies sheared by +-(0.02, 0), same noise; "
                                          f"{args.sampler.upper()}, 4 chains x (300 + 1000), K = 1000, "
                                          f"33 x 33 grid, {args.n_boot} bootstrap resamples"}, **res}
        elif args.workload == "spergel":
            G = args.n_gal or gen.CONFIGS["uniform"].n_gal
            res = spergel_leg(api, torch, stream, G, args.spergel_nu, log)
            out = {"metric": "galaxies/sec at 300 ESS (Spergel-profile fit of exponential galaxies)",
                   "value": res["galaxies_per_s"], "unit": "galaxies/s", "n_gpus": 1,
                   "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                   "config": {"workload": f"model-bias fit: 53-pixel exponential galaxies, Spergel "
                                          f"nu = {args.spergel_nu}, 4 chains, 20 leapfrog steps, "
                                          "300 warmup + 1000 draws"}, **res}
        elif args.workload == "tiny":
            res = tiny_leg(api, torch, stream, log, oracle=orc.get("tiny"))
            out = {"metric": "galaxies/sec at 300 ESS (plain tiny workload), batched vs plain",
                   "value": res["galaxies_per_s"], "unit": "galaxies/s", "n_gpus": 1,
                   "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                   "config": {"workload": "plain tiny: 16 galaxies, 32x32 stamps, PSF FWHM 0.7in, "
                                          "SNR 15-100, 1 chain, 10 leapfrog steps at step 0.005, "
                                          "100 burn-in + 500 draws, shear grid 41x41 on "
                                          "[-0.25, 0.25]^2"}, **res}
        elif args.workload == "uneven":
            G = args.n_gal or gen.CONFIGS["uneven"].n_gal
            res = uneven_leg(api, torch, stream, G, log, oracle=orc.get("sizes"))
            out = {"metric": "galaxies/sec at 300 ESS (uneven stamps 25-101 px)",
                   "value": res["galaxies_per_s"], "unit": "galaxies/s", "n_gpus": 1,
                   "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                   "config": {"workload": "batched uneven: stamp side from the size rule, PSF FWHM "
                                          "U(0.6, 0.9)in, SNR 10-200, 4 chains, 20 leapfrog steps, "
                                          "300 warmup + 1000 draws"}, **res}
        else:
            if args.serve_requests:
                res = serving_leg(api, torch, 2000.0, args.serve_requests / 2000.0, 60000, 5, pace=False,
                                  split=0, log=log, oracle=orc.get("sizes"))
            else:
                res = serving_leg(api, torch, 2000.0, args.serve_window, 60000, 5,
                                  extra_rates=(0.5, 0.9), log=log, oracle=orc.get("sizes"))
            out = {"metric": "p50/p99 fit latency and galaxies/s, Poisson requests",
                   "value": res["galaxies_per_s"], "unit": "galaxies/s", "n_gpus": 1,
                   "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                   "config": {"workload": "serving: Poisson arrivals at 2000 req/s, stamp sizes "
                                          "25/41/53/73/101 (weights .3/.3/.2/.15/.05), 1 chain, 20 "
                                          "leapfrog steps, 300 warmup, then draws until 300 ESS "
                                          "(checked every 60 draws, at most 1500)"}, **res}
        print(json.dumps(out), flush=True)
        return
    cfg = gen.CONFIGS["uniform"]
    G = args.n_gal or cfg.n_gal

    cpu = None
    if not args.no_cpu_baseline:
        rate, cores, evals, wall = cpu_baseline_eval_rate()
        cpu = dict(rate=rate, cores=cores, evals=evals, wall=wall,
                   visible=len(os.sched_getaffinity(0)))
        print(f"[bench] oracle: {evals} gradient evaluations on {cores} cores in {wall:.1f} s",
              file=sys.stderr, flush=True)

    import torch
    from paper_2604_22048_amd import api
    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if args.plan:
        api.set_plan(cfg.n_pix, args.plan)          # fixed slot plan (profiling runs)
        plans = {cfg.n_pix: (args.plan, None)}
    else:
        plans = api.autotune([cfg.n_pix], n_chains=cfg.chains)
    log(f"[bench] slot plans {plans}")
    t, b, data, ref, init = make_inputs(api, torch, G, cfg)
    N = cfg.n_pix
    C, L, W, S = cfg.chains, cfg.leapfrog, cfg.warmup, cfg.samples
    hcfg = api.HmcConfig(n_chains=C, n_leapfrog=L, n_warmup=W, n_samples=S, adapt=True,
                         metric=api.N.METRIC_FISHER, step_size=0.5, target_accept=0.8, jitter=0.2,
                         iters_per_launch=1, use_graph=True, seed=gen.chain_seed(cfg.index))
    wcfg = api.HmcConfig(**{**hcfg.__dict__, "n_samples": 0})
    g1s = np.linspace(-0.1, 0.1, 41)
    alpha = (math.log(0.6), 0.3, 0.2)
    pts = torch.tensor([[a, bb, *alpha] for bb in g1s for a in g1s], dtype=torch.float64, device=dev)
    tp = api.TruePriorCfg(e_kind=1, e_max=0.7, size_term=True)
    K = 1000

    def step():
        (smp, stats, status), t_hmc = timed(torch, lambda: api.hmc_sample(b, data, ref, init, hcfg),
                                            stream)
        (ess, rh, rhs), t_ess = timed(torch, lambda: api.ess(smp, split=True), stream)
        # interim samples for the shear phase: every 4th draw of the 4 chains
        def shear_step():
            th = smp[:, :, 3::4, :].reshape(G, K, 6)
            return api.shear_posterior(th[..., 2], th[..., 3], th[..., 1], th[..., 0], pts, tp)
        lp, t_shear = timed(torch, shear_step, stream)
        return dict(smp=smp, stats=stats, status=status, ess=ess, rhat=rh, rhat_split=rhs, lp=lp,
                    t_hmc=t_hmc,
                    t_ess=t_ess, t_shear=t_shear)

    for i in range(args.warmup):
        step()
        print(f"[bench] warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(step())
        print(f"[bench] step {i + 1}/{args.steps}: hmc {results[-1]['t_hmc']:.3f} s", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    r = results[-1]
    # warmup-only call: splits T_hmc into warmup and sampling
    _, t_w = timed(torch, lambda: api.hmc_sample(b, data, ref, init, wcfg, want_samples=False), stream)
    t_hmc = float(np.mean([x["t_hmc"] for x in results]))
    t_s = t_hmc - t_w
    ess = r["ess"].cpu().numpy()
    n_eff = ess.mean(axis=1)                  # mean over the six properties (Section 4.1)
    n_eff_mean = float(n_eff.mean())
    tpg = t_w / G + t_s / (G * n_eff_mean) * TARGET_ESS
    value = 1.0 / tpg
    stats = r["stats"].cpu().numpy()
    rhat = r["rhat"].cpu().numpy()
    rhat_split = r["rhat_split"].cpu().numpy()
    flagged = (r["status"] != 0).cpu().numpy()

    # plain form: one galaxy and one leapfrog step per launch, on a subset
    Gp = args.plain_gal
    pt, pb, pdata, pref, pinit = make_inputs(api, torch, Gp, cfg, seed_offset=99)
    it_p = 2
    pcfg = api.HmcConfig(**{**hcfg.__dict__, "form": api.N.FORM_PLAIN, "n_warmup": it_p,
                            "n_samples": 0, "use_graph": False})
    _, t_plain = timed(torch, lambda: api.hmc_sample(pb, pdata, pref, pinit, pcfg, want_samples=False),
                       stream)
    per_iter_gal = t_plain / (Gp * it_p)        # seconds per galaxy-iteration (C chains)
    plain_tpg = per_iter_gal * (W + S * TARGET_ESS / n_eff_mean)
    plain_value = 1.0 / plain_tpg

    # roofline of the trajectory kernel: one launch = one iteration of every chain
    n_launch = W + S
    t_launch = t_hmc / n_launch
    alg = flops_per_eval(N, L) * G * C * L
    achieved = alg / t_launch / 1e12
    peak = FP32_PEAK_TFLOPS
    legs = {}
    if not args.no_legs:
        legs["shear_hmc"] = shear_leg(api, torch, stream, r["smp"], G, K, gen.chain_seed(3),
                                      cpu=cpu is not None)
        log(f"[bench] shear-level HMC: {legs['shear_hmc']['t_s']} s")
        del results, r["smp"]
        legs["uneven"] = uneven_leg(api, torch, stream, gen.CONFIGS["uneven"].n_gal, log,
                                    oracle=orc.get("sizes"))
        log(f"[bench] uneven: {legs['uneven']['galaxies_per_s']} galaxies/s, per size "
            f"{ {N: v['frac_fp32_peak'] for N, v in legs['uneven']['per_size'].items()} }")
        legs["transform"] = transform_leg(api)
        log(f"[bench] render transforms: {legs['transform']}")
        legs["tiny"] = tiny_leg(api, torch, stream, log, oracle=orc.get("tiny"))
        log(f"[bench] tiny: {legs['tiny']['galaxies_per_s']} galaxies/s batched, "
            f"{legs['tiny']['plain_galaxies_per_s']} plain")
        if not args.no_serving:
            legs["serving"] = serving_leg(api, torch, 2000.0, args.serve_window, 20000, 5, log=log,
                                          oracle=orc.get("sizes"))
    out = {
        "metric": "galaxies/sec at 300 ESS (53x53 stamps), batched vs plain; p50/p99 fit latency",
        "value": round(value, 3),
        "unit": "galaxies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched uniform: 10,000 galaxies, 53x53 stamps, PSF FWHM 0.7in, "
                               "SNR 15-100, 4 chains, 20 leapfrog steps, 300 dual-averaging warmup "
                               "+ 1000 draws, shear grid 41x41",
                   "n_gal": G, "stamp": N, "chains": C, "leapfrog": L, "warmup_iters": W,
                   "samples": S, "metric_kind": "fisher-diagonal", "jitter": 0.2,
                   "slot_plan_P": plans[N][0]},
        "plain_value": round(plain_value, 4),
        "batched_over_plain": round(value / plain_value, 1),
        "t_warmup_s": round(t_w, 4),
        "t_sampling_s": round(t_s, 4),
        "t_ess_s": round(r["t_ess"], 4),
        "t_shear_grid_s": round(r["t_shear"], 4),
        "n_eff_mean": round(n_eff_mean, 1),
        "n_eff_min_param_mean": round(float(ess.min(axis=1).mean()), 1),
        "ess_per_s": round(float(ess.mean(axis=1).sum()) / t_s, 1),
        "accept_rate": round(float(stats[..., 0].mean()), 4),
        "rhat_max": round(float(np.nanmax(rhat)), 4),
        "frac_rhat_lt_1.01": round(float(np.mean(rhat.max(axis=1) < 1.01)), 4),
        "rhat_split_max": round(float(np.nanmax(rhat_split)), 4),
        "frac_rhat_split_lt_1.01": round(float(np.mean(rhat_split.max(axis=1) < 1.01)), 4),
        "n_eff_mean_unflagged": round(float(n_eff[~flagged].mean()), 1),
        "frac_status_nonzero": round(float((r["status"] != 0).float().mean()), 4),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "traffic": recorded_traffic(),
                     "kernel": "hmc_kernel (advance)", "launch_ms": round(t_launch * 1e3, 4),
                     "alg_flop_per_eval": flops_per_eval(N, L), "evals_per_launch": G * C * L,
                     "alg_flop_per_launch": alg,
                     "valu_issue_frac": valu_issue_frac(t_launch),
                     "executed_frac": executed_frac(t_launch),
                     "frac_of_nonpacked_issue_ceiling": round(achieved / VALU_ISSUE_TFLOPS, 4)},
        **legs,
    }
    if cpu:
        evals_per_gal = C * L * (W + S * TARGET_ESS / n_eff_mean)
        out["cpu_baseline"] = {"value": round(cpu["rate"] / evals_per_gal, 6), "unit": "galaxies/s",
                               "cores": cpu["cores"], "kind": "oracle",
                               "cores_visible": cpu["visible"],
                               "cores_note": f"one worker per usable core, capped at {CPU_WORKER_CAP} "
                                             "(the host cores that come with one GPU of a shared node)",
                               "sample": f"{cpu['evals']} float64 oracle gradient evaluations (53x53, "
                                         f"one {CPU_ITERS}-iteration warmup chain per core) in "
                                         f"{cpu['wall']:.1f} s; galaxies/s = eval rate / evaluations "
                                         f"per galaxy at 300 ESS with the GPU run's n_eff"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
