"""Open- and closed-loop drivers for the energy-density serving loop.

A job is (cell, one frequency, a block of coarse points); arrivals follow a
seeded Poisson process over a seeded mix of cells.  Latency is completion
minus arrival (host steady clock of the server)."""
from __future__ import annotations

import time

import numpy as np


def make_jobs(n_jobs, cells, mix, omegas, block, seed):
    """[(cell index, omega, points)] drawn from the mix with a seeded stream.
    cells: list of (cell_id, coarse_points); mix: probabilities per cell."""
    rng = np.random.default_rng(seed)
    perms = [rng.permutation(pts) for _, pts in cells]
    cursor = [0] * len(cells)
    jobs = []
    for _ in range(n_jobs):
        c = int(rng.choice(len(cells), p=mix))
        w = float(rng.choice(omegas))
        pts = perms[c]
        i0 = cursor[c] % max(1, len(pts) - block + 1)
        cursor[c] += block
        jobs.append((c, w, np.sort(pts[i0:i0 + block])))
    return jobs


class DeviceMemoryPeak:
    """Largest device memory in use (all allocations on the GPU, free memory
    reported by the runtime), sampled when jobs complete; no-op without a GPU."""

    def __init__(self):
        self.used_max = 0
        try:
            import torch
            self._info = torch.cuda.mem_get_info if torch.cuda.is_available() else None
        except ImportError:
            self._info = None

    def sample(self):
        if self._info is not None:
            free, total = self._info()
            self.used_max = max(self.used_max, total - free)


def run_closed(server, cells, jobs, n_lanczos, depth, mem=None, log=None, every=10):
    """Keep `depth` jobs in flight; returns (seconds, infos).  log(msg), if
    given, is called after every `every` completions."""
    t0 = time.perf_counter()
    inflight, infos, k = [], [], 0
    while k < len(jobs) or inflight:
        while k < len(jobs) and len(inflight) < depth:
            c, w, pts = jobs[k]
            inflight.append(server.submit(cells[c][0], w, pts, n_lanczos))
            k += 1
        _, info = server.wait(inflight.pop(0))
        infos.append(info)
        if mem is not None:
            mem.sample()
        if log is not None and len(infos) % every == 0:
            log(f"closed loop: {len(infos)}/{len(jobs)} jobs done at {time.perf_counter() - t0:.1f}s")
    return time.perf_counter() - t0, infos


def run_open(server, cells, jobs, n_lanczos, rate, seed, mem=None, log=None, every=10):
    """Submit at Poisson arrival times of the given rate (jobs/s); returns
    (seconds, infos) with latency = finish - submit.  log(msg), if given, is
    called after every `every` submissions and completions."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=len(jobs))
    t0 = time.perf_counter()
    t_next = t0
    ids = []
    for (c, w, pts), g in zip(jobs, gaps):
        t_next += g
        dt = t_next - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        ids.append(server.submit(cells[c][0], w, pts, n_lanczos))
        if log is not None and len(ids) % every == 0:
            log(f"open loop: {len(ids)}/{len(jobs)} jobs submitted at {time.perf_counter() - t0:.1f}s")
    infos = []
    for j in ids:
        infos.append(server.wait(j)[1])
        if mem is not None:
            mem.sample()
        if log is not None and len(infos) % every == 0:
            log(f"open loop: {len(infos)}/{len(jobs)} jobs done at {time.perf_counter() - t0:.1f}s")
    return time.perf_counter() - t0, infos


def summarize(infos, seconds, warm=0):
    lat = np.array([i["latency"] for i in infos[warm:]])
    pts = sum(i["stats"]["n_systems"] for i in infos)   # systems, for reference
    return {"jobs": len(infos), "seconds": seconds,
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "jobs_per_s": len(infos) / seconds}
