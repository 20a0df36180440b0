"""Request loop over the library's slot server (bsi_slots_*): requests arrive
at given wall-clock times, wait in a first-come-first-served queue, are
admitted while their device footprint fits, run concurrently with everything
else resident, and are handed back when their chains have finished.  The
latency of a request is the time from its arrival to the moment its samples
are back in caller memory.

Only host bookkeeping happens here; every computation runs in the library.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import api

# finished requests' draws held on the device for the ESS check before a batch is checked
ESS_BATCH_BYTES = 64 << 20


@dataclass
class RequestPool:
    """Request payloads (stamp on the device, PSF, noise, centroid, start
    positions) for each served stamp size; request j of size N uses payload
    j mod len(pool[N])."""
    stamps: dict          # N -> float32 device tensor [P, N * N]
    psf: dict             # N -> float32 [P]
    sigma: dict           # N -> float32 [P]
    ref: dict             # N -> float32 [P, 2]
    init: dict            # N -> float32 [P, C, 6] (host, contiguous)

    def build(self, ids: np.ndarray, sizes: np.ndarray, slot: np.ndarray) -> np.ndarray:
        """bsi_request records for requests `ids` with stamp sides `sizes`,
        payload indices `slot` (per size)."""
        rec = np.zeros(ids.shape[0], dtype=api.Slots.REQUEST_DTYPE)
        rec["id"] = ids
        rec["n"] = sizes
        for N in np.unique(sizes):
            m = sizes == N
            P = self.stamps[int(N)].shape[0]
            j = slot[m] % P
            rec["stamp"][m] = self.stamps[int(N)].data_ptr() + j.astype(np.uint64) * (int(N) * int(N) * 4)
            rec["psf_fwhm"][m] = self.psf[int(N)][j]
            rec["sigma"][m] = self.sigma[int(N)][j]
            rec["ref_x"][m] = self.ref[int(N)][j, 0]
            rec["ref_y"][m] = self.ref[int(N)][j, 1]
            ini = self.init[int(N)]
            rec["init"][m] = ini.ctypes.data + j.astype(np.uint64) * ini[0].nbytes
        return rec


@dataclass
class ServeResult:
    latency: np.ndarray       # seconds, per request (NaN if not completed)
    finish: np.ndarray        # completion time from the start, per request
    wall: float               # seconds from the first arrival to the last completion
    n_done: int
    ticks: int
    max_resident: int
    ess_mean: np.ndarray | None   # mean over the six properties, per completed request
    n_draws: np.ndarray           # draws per chain returned, per request (0 if not completed)
    tick_s: np.ndarray | None = None   # duration of each loop turn that advanced, ESS bookkeeping included [s]


def serve(srv: api.Slots, pool: RequestPool, arrivals: np.ndarray, sizes: np.ndarray,
          n_iter: int, time_limit: float = 600.0, ess: bool = False, progress=None) -> ServeResult:
    """Run the request loop in real time until every request has completed.

    arrivals: nondecreasing arrival times [s] relative to the start of the
    loop; sizes: stamp side of each request.  Each loop turn admits every
    arrived request that fits (in arrival order), enqueues n_iter iterations
    for all resident requests, and collects the finished ones.  ess: also
    the ESS of each request's returned draws (mean over the six properties),
    computed off the requests' critical path: the finished requests' draws are
    kept on the device and checked in batches (once they pass ESS_BATCH_BYTES,
    and after the loop) on a side stream that the loop does not wait for."""
    n = arrivals.shape[0]
    ids = np.arange(n, dtype=np.uint64)
    slot = np.zeros(n, dtype=np.int64)
    for N in np.unique(sizes):
        m = sizes == N
        slot[m] = np.arange(int(m.sum()))
    records = pool.build(ids, sizes.astype(np.int32), slot)
    lat = np.full(n, np.nan)
    fin = np.full(n, np.nan)
    ess_out = np.full(n, np.nan) if ess else None
    draws = np.zeros(n, dtype=np.int32)
    # finished requests' draws for the ESS check, by draw count: count -> [(ids, samples)]
    kept: dict = {}
    kept_bytes = 0
    side = torch.cuda.Stream(device=pool.stamps[int(sizes[0])].device) if ess and n else None
    checked = []       # (ids, device ESS means) of the batches queued so far
    in_use = []        # inputs of the batch on the side stream, held until it has run

    def check_kept():
        # one ESS call per distinct draw count over everything kept, queued on
        # a side stream so that the loop does not wait for it
        side.synchronize()
        in_use.clear()
        side.wait_stream(torch.cuda.current_stream(side.device))
        with torch.cuda.stream(side):
            for v, parts in kept.items():
                x = torch.cat([x for _, x in parts])
                e, _ = api.ess(x)
                checked.append((np.concatenate([h for h, _ in parts]), e.mean(dim=1)))
        in_use.append(kept.copy())
        kept.clear()

    queue_head = 0
    done = 0
    ticks = 0
    resident = 0
    max_res = 0
    next_report = 5.0
    tick_s = []
    t0 = time.perf_counter()
    while done < n:
        now = time.perf_counter() - t0
        if now > time_limit:
            break
        arrived = int(np.searchsorted(arrivals, now, side="right"))
        if queue_head < arrived:
            k = srv.admit_many(records[queue_head:arrived])
            queue_head += k
            resident += k
        if resident == 0:
            # idle: wait for the next arrival
            if queue_head < n:
                time.sleep(max(0.0, min(arrivals[queue_head] - now, 0.01)))
            continue
        max_res = max(max_res, resident)
        srv.advance(n_iter)
        ticks += 1
        n_fin = srv.poll()
        hid, smp, _, _, nd = srv.harvest(n_fin, want_samples=ess)
        t_done = time.perf_counter() - t0
        if hid.size:
            h = hid.astype(np.int64)
            fin[h] = t_done
            lat[h] = t_done - arrivals[h]
            done += h.size
            resident -= h.size
            ndh = nd.cpu().numpy()
            draws[h] = ndh
            if ess:
                # the returned draws (a prefix of each request's draws for
                # requests finished at a check) are checked in batches, off
                # the requests' critical path
                for v in np.unique(ndh):
                    m = np.nonzero(ndh == v)[0]
                    x = smp[torch.from_numpy(m).to(smp.device), :, :int(v)].contiguous()
                    kept.setdefault(int(v), []).append((h[m], x))
                    kept_bytes += x.numel() * x.element_size()
                if kept_bytes > ESS_BATCH_BYTES:
                    check_kept()
                    kept_bytes = 0
        tick_s.append(time.perf_counter() - t0 - now)
        if progress and t_done > next_report:
            progress(f"[serve] t={t_done:.1f}s done={done}/{n} resident={resident} "
                     f"queued={arrived - queue_head}")
            next_report = t_done + 5.0
    if side is not None:
        check_kept()
        side.synchronize()
        for h, em in checked:
            ess_out[h] = em.cpu().numpy()
    wall = float(np.nanmax(fin) - arrivals[0]) if done else float("nan")
    return ServeResult(latency=lat, finish=fin, wall=wall, n_done=done, ticks=ticks,
                       max_resident=max_res, ess_mean=None if ess_out is None else ess_out,
                       n_draws=draws, tick_s=np.array(tick_s))
