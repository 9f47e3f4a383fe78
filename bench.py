#!/usr/bin/env python3
"""Benchmark of the RPA energy-density hot path on one MI355X.

One step = one batch of 64 Lanczos start vectors (8 coarse points x 8
frequencies) through the whole path: nu^1/2 -> Galerkin guess -> batched
Sternheimer COCG (FP32 + FP64 refinement) -> density accumulation -> nu^1/2 ->
Lanczos recurrence with full reorthogonalisation -> tridiagonal quadrature,
then tricubic interpolation of the resident coarse field and frequency
integration.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RPA energy-density points/s, Si64 FP32+refine vs FP64; stencil GB/s; p99 latency"
HBM_PEAK_GBPS = 8000.0
# the kernel's traffic also depends on the engine's defaults (reliable-update
# factor, processing order), so the engine source is part of the key
COCG_SRC = [os.path.join(ROOT, "paper_2609_16408_amd", "csrc", f)
            for f in ("cocg_impl.h", "precond_impl.h", "internal.h", "cocg.hip", "cocg_nl.hip",
                      "cocg_pc.hip", "engine.hip")]
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_cocg_si64_hbm_traffic.md")
CALIB_BYTES = 1 << 30

# workload name -> synthetic cell preset and method settings
WORKLOADS = {
    # Galerkin guess widened by the 384 eigenpairs above the occupied ones;
    # preconditioned solves for 0.5 <= omega <= 20, where the kinetic
    # preconditioner's fewer iterations outweigh its per-iteration cost,
    # plain COCG at the other nodes
    "si64": dict(preset="si64", n_lanczos=8, tol=1e-6, stride=2, interp="tricubic", every=3,
                 pts_per_step=8, precond_window=(0.5, 20.0), n_extra=384,
                 desc="Si64-like 2x2x2 cell, 48^3 grid, 128 orbitals"),
    "si8": dict(preset="si8", n_lanczos=8, tol=1e-6, stride=2, interp="tricubic", every=3,
                pts_per_step=8, desc="Si8-like cell, 24^3 grid, 16 orbitals"),
    "tiny": dict(preset="tiny", n_lanczos=8, tol=1e-6, stride=2, interp="tricubic", every=1,
                 pts_per_step=8, desc="tiny 12^3 cell, 4 orbitals"),
    # largest configuration: 2 points x 8 frequencies = 16 start vectors per step
    # (x alone is 41 GB); every 9th coarse point per axis
    "si216": dict(preset="si216", n_lanczos=8, tol=1e-6, stride=2, interp="tricubic", every=9,
                  pts_per_step=2, progress=True,
                  desc="Si216-like 3x3x3 cell, 72^3 grid, 432 orbitals, 864 nonlocal projectors"),
    # the plain FP64 method on the Si8-like cell at its own settings: N_l = 30,
    # tol 1e-8, trilinear interpolation, every stride-2 coarse point (54 steps
    # of 32 points x 8 frequencies cover all 1728)
    "si8c2": dict(preset="si8", n_lanczos=30, tol=1e-8, stride=2, interp="trilinear", every=1,
                  pts_per_step=32, precision="fp64",
                  desc="Si8-like cell, 24^3 grid, 16 orbitals, plain FP64 method (N_l 30, tol 1e-8)"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def nl_support_points(proj) -> int:
    """Grid points gathered per projection of one vector: the support of each
    group of consecutive projectors with identical support (as the library
    groups them, at most 4 per group)."""
    if proj is None:
        return 0
    import numpy as np
    ptr, idx = proj["ptr"], proj["idx"]
    total, q, n = 0, 0, len(ptr) - 1
    while q < n:
        a, b = ptr[q], ptr[q + 1]
        k = 1
        while k < 4 and q + k < n and ptr[q + k + 1] - ptr[q + k] == b - a and \
                np.array_equal(idx[ptr[q + k]:ptr[q + k + 1]], idx[a:b]):
            k += 1
        total += int(b - a)
        q += k
    return total


def cocg_algorithmic_bytes(st: dict, N: int, precision: str, nl_support: int = 0) -> float:
    """HBM bytes the batched Sternheimer launches must move.

    FP32+refine, per system: 80 B/pt per COCG iteration (sweep A reads r, p_old
    and writes p, q; sweep B reads p, q, r, d and writes d, r: 10 complex FP32
    vectors), 40 B/pt per FP64 residual sweep (read x64, psi, u; write r32) and
    40 B/pt per fold x64 += d, one residual sweep per system plus one per cycle.
    FP64: 160 B/pt per iteration and 48 B/pt for the initial residual.
    """
    if precision == "fp32_refine":
        per_pt = 80.0 * st["cocg_iters_total"] + 80.0 * st["refine_cycles"] + 40.0 * st["n_systems"]
        # nonlocal projections: gather p (8 B) per support point and iteration,
        # x64 (16 B) per residual sweep; the shared projector tables are not counted
        nl = nl_support * (8.0 * st["cocg_iters_total"] +
                           16.0 * (st["refine_cycles"] + st["n_systems"]))
    else:
        per_pt = 160.0 * st["cocg_iters_total"] + 48.0 * st["n_systems"]
        nl = nl_support * 16.0 * (st["cocg_iters_total"] + st["n_systems"])
    return per_pt * N + nl


def precond_algorithmic(st: dict, n, precision: str) -> tuple[float, float]:
    """HBM bytes and MFMA flops of the preconditioner applications on top of
    cocg_algorithmic_bytes, one application per COCG iteration: three complex
    passes (yz forward r -> t, x forward/scale/inverse t -> t, yz inverse
    t -> z), each reading and writing one vector (48 B/pt FP32, 96 B/pt FP64),
    and a real n_d x n_d basis applied to both parts of the complex vector
    along each axis, forward and inverse: 8 (n_x + n_y + n_z) flops per point."""
    N = float(n[0] * n[1] * n[2])
    its = st["cocg_iters_total"]
    per_pt = 48.0 if precision == "fp32_refine" else 96.0
    return per_pt * its * N, 8.0 * float(sum(n)) * its * N


def kind_totals(per_omega, precond: bool, window) -> dict:
    """Per-frequency COCG totals split by the launch that ran them: the plain
    kernel (kind 0) and the preconditioned one (kind 1), from the pooled
    per-frequency statistics (a solve handed over to FP64 is counted with its
    FP32 launch)."""
    out = {k: {"n_systems": 0, "cocg_iters_total": 0, "refine_cycles": 0} for k in (0, 1)}
    lo, hi = (window if window is not None else (0.0, 0.0))
    for r in per_omega:
        inside = precond and (window is None or (r["omega"] >= lo and (hi <= 0 or r["omega"] <= hi)))
        o = out[1 if inside else 0]
        o["n_systems"] += r["solves"]
        o["cocg_iters_total"] += r["iters_total"]
        o["refine_cycles"] += r["refine_cycles"]
    return out


def source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in COCG_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def cocg_mode(precond: bool, window) -> str:
    if not precond:
        return "plain"
    return "precond" if window is None else f"precond_window {window[0]:g} {window[1]:g}"


def pmc_traffic(workload, precond=False, window=None, n_extra=0):
    """HBM bytes per launch of the dominant Sternheimer kernel from the
    committed rocprofv3 --pmc summary, or None when it is missing, for another
    workload, solver mode or Galerkin space, or for another version of the
    kernel source."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    vals = {}
    for line in open(PMC_SUMMARY):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("workload") != workload or vals.get("cocg_source_sha") != source_sha() or \
            vals.get("mode", "plain") != cocg_mode(precond, window) or \
            int(vals.get("galerkin_extra", "0")) != int(n_extra):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def calibrate_copy():
    """Plain device-to-device copy of CALIB_BYTES (the rocprofv3 --pmc scale reference)."""
    import torch
    src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": CALIB_BYTES, "copies": 3}), flush=True)


def load_or_make_cell(sc, preset, cache, n_extra=0):
    """Synthetic cell (with n_extra converged eigenpairs above the occupied
    ones); with `cache`, orbitals are reused from (or saved to) an .npz."""
    import numpy as np
    if cache and os.path.exists(cache):
        z = np.load(cache)
        cached = int(z["n_extra"]) if "n_extra" in z.files else 0
        if cached == n_extra:
            cell = sc.preset(preset, orbitals=False)
            cell.psi, cell.eps = z["psi"], z["eps"]
            cell.gap, cell.eig_residual = float(z["gap"]), float(z["res"])
            if n_extra > 0:
                cell.psi_extra, cell.eps_extra = z["psi_extra"], z["eps_extra"]
            return cell
    # the orbital solver reports progress on large cells (a long silent setup
    # would look hung)
    cell = sc.preset(preset, device="cuda", verbose=2 if preset == "si216" else False, n_extra=n_extra)
    if cache:
        extra = {"psi_extra": cell.psi_extra, "eps_extra": cell.eps_extra} if n_extra > 0 else {}
        np.savez(cache, psi=cell.psi, eps=cell.eps, gap=cell.gap, res=cell.eig_residual,
                 n_extra=n_extra, **extra)
    return cell


def stencil_gbps(P, h, cell, torch, nvec=512, reps=5):
    """Plain FP32 H-apply on nvec complex vectors: algorithmic 16 B/pt (read + write)."""
    N = cell.N_d
    x = torch.randn((nvec, N), dtype=torch.complex64, device="cuda")
    shifts = [complex(-0.4, 0.1 * (i + 1)) for i in range(nvec)]
    h.hamiltonian_apply(shifts, x, precision="fp32_refine")
    ms = []
    for _ in range(reps):
        h.hamiltonian_apply(shifts, x, precision="fp32_refine")
        ms.append(h.last_cocg_timing()["ms"])
    t = sorted(ms)[len(ms) // 2]
    return 16.0 * nvec * N / (t * 1e-3) / 1e9, t


def _cpu_init(root, spec):
    import numpy as np
    sys.path.insert(0, root)
    from threadpoolctl import threadpool_limits
    _CPU["lim"] = threadpool_limits(limits=1)
    import oracle as O
    _CPU["O"] = O
    _CPU["psi"] = np.load(spec["psi"], mmap_mode="r")
    _CPU["eps"] = np.load(spec["eps"])
    _CPU["ham"] = O.Hamiltonian(spec["n"], spec["L"], np.load(spec["v"]), proj=spec["proj"])
    _CPU["u"] = np.load(spec["u"])


def _cpu_unit(args):
    """One Sternheimer solve of the oracle (an (omega, orbital) unit of one
    Lanczos matrix-vector product); returns its seconds and iterations."""
    omega, n, tol = args
    st = {}
    t = time.perf_counter()
    _CPU["O"].chi0_apply(_CPU["ham"], _CPU["psi"], _CPU["eps"], _CPU["u"], omega, tol=tol,
                         orbitals=[n], stats=st)
    return time.perf_counter() - t, st["iters"][0]


_CPU = {}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cell, cfg, omegas, workers=None):
    """The oracle timed on the host, one single-threaded process per core (at
    most 16): the first Lanczos matrix-vector product of one coarse point
    (nu^1/2 e_j, then every occupied orbital's Sternheimer solve at the
    benchmark's tolerance) at all 8 frequencies, (frequency, orbital) units
    dealt round-robin over the processes.  Those 8 matrix-vector products are
    the first of the n_lanczos each of the 8 points (j, omega_k) needs; the
    rate is extrapolated over the remaining Lanczos steps only."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import shutil
    import tempfile
    import numpy as np
    import oracle as O
    workers = int(workers or min(16, os.cpu_count() or 1))
    j = int(sc_sublattice_first(cell, cfg))
    q = np.zeros(cell.N_d)
    q[j] = 1.0
    u = O.Coulomb(cell.n, cell.L).half(q)
    d = tempfile.mkdtemp(prefix="cpu_baseline_")
    spec = {"n": tuple(cell.n), "L": tuple(cell.L), "proj": cell.proj}
    for k, arr in (("v", cell.v_loc), ("psi", cell.psi), ("eps", cell.eps), ("u", u)):
        spec[k] = os.path.join(d, k + ".npy")
        np.save(spec[k], np.ascontiguousarray(arr, dtype=np.float64))
    units = [(float(w), n, cfg["tol"]) for n in range(cell.n_occ) for w in omegas]
    # the longest solves (smallest omega, highest orbitals) first
    units.sort(key=lambda t: (t[0], -t[1]))
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"),
                                    initializer=_cpu_init, initargs=(ROOT, spec)) as ex:
            list(ex.map(abs, range(workers)))          # start every worker before timing
            t0 = time.perf_counter()
            res = []
            for r in ex.map(_cpu_unit, units, chunksize=1):
                res.append(r)
                if len(res) % max(1, len(units) // 4) == 0:
                    log(f"[bench] cpu baseline: {len(res)}/{len(units)} solves after "
                        f"{time.perf_counter() - t0:.0f}s")
            wall = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
        shutil.rmtree(d, ignore_errors=True)
    cpu_s = sum(r[0] for r in res)
    its = [r[1] for r in res]
    points = len(omegas)                                  # (j, omega_k) pairs
    per_point_s = wall * cfg["n_lanczos"] / points
    return {"value": 1.0 / per_point_s, "unit": "points/s", "cores": workers, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "core_seconds_per_point": cpu_s * cfg["n_lanczos"] / points,
            "sample": (f"first Lanczos matrix-vector product of coarse point {j} at all {points} "
                       f"frequencies: {len(units)} Sternheimer solves (all {cell.n_occ} orbitals), "
                       f"tol {cfg['tol']}, mean {np.mean(its):.1f} COCG iterations, on {workers} "
                       f"single-threaded processes: {wall:.1f} s wall, {cpu_s:.0f} core-s; "
                       f"extrapolated x{cfg['n_lanczos']} Lanczos steps")}


def sc_sublattice_first(cell, cfg):
    import synthcell as sc
    return sc.sublattice_points(cell.n, cfg["stride"], cfg["every"])[0]


def serving_run(P, sc, si64_cell, omega, log_fn, n_closed=12, n_open=20, warm=2, n_lanczos=3,
                tol=0.1, block=256, budget_gb=250.0):
    """Energy-density serving: seeded job mix over resident cells, 3 workers,
    closed-loop saturation, then Poisson arrivals at 0.5x and 0.9x of it.
    The defaults are the light block the default benchmark run includes."""
    import numpy as np
    from paper_2609_16408_amd import serve
    t0 = time.perf_counter()
    pool = [sc.preset("si8", seed=401, device="cuda"), sc.preset("si8", seed=402, device="cuda"),
            sc.preset("si16", seed=411, device="cuda"), sc.preset("si16", seed=412, device="cuda"),
            si64_cell]
    mix = [0.25, 0.25, 0.15, 0.15, 0.20]
    server = P.Server(n_workers=3, hbm_budget=int(budget_gb * 10 ** 9))
    cells = [(server.add_cell(c.n, c.L, c.v_loc, c.psi, c.eps, precision="fp32_refine",
                              stern_tol=tol), sc.coarse_points(c.n, 2)) for c in pool]
    log_fn(f"[bench] serving pool ready in {time.perf_counter() - t0:.1f}s")
    jobs = serve.make_jobs(n_closed + 2 * n_open, cells, mix, omega, block, seed=4000)
    mem = serve.DeviceMemoryPeak()
    say = lambda m: log_fn("[bench] serving " + m)
    secs, infos = serve.run_closed(server, cells, jobs[:n_closed], n_lanczos, depth=6, mem=mem,
                                   log=say)
    sat = len(infos) / secs
    out = {"workload": f"jobs of {block} coarse points at one frequency; 50% Si8-like (24^3, 16 orb), "
                       "30% Si16-like (24x24x48, 32 orb), 20% Si64-like (48^3, 128 orb); "
                       f"FP32+refine, N_l={n_lanczos}, tol {tol:g}; 3 workers",
           "jobs_closed_loop": n_closed, "jobs_per_load": n_open, "warmup_jobs_excluded": warm,
           "saturation_jobs_per_s": sat}
    log_fn(f"[bench] serving saturation {sat:.3f} jobs/s")
    for name, frac, lo in (("load_0.5", 0.5, n_closed), ("load_0.9", 0.9, n_closed + n_open)):
        secs, infos = serve.run_open(server, cells, jobs[lo:lo + n_open], n_lanczos,
                                     rate=frac * sat, seed=4100 + int(10 * frac), mem=mem, log=say)
        r = serve.summarize(infos, secs, warm=warm)
        r["points_per_s"] = n_open * block / secs
        out[name] = r
        log_fn(f"[bench] serving {name}: p50 {r['p50_latency_s']:.2f}s p99 {r['p99_latency_s']:.2f}s")
    st = server.status()
    # admission model (resident cells + admitted workspace estimates) and the
    # device memory actually in use at job completions (whole GPU)
    out["hbm_admitted_high_water_gb"] = st["high_water"] / 1e9
    out["hbm_used_max_gb"] = mem.used_max / 1e9
    out["hbm_budget_gb"] = budget_gb
    server.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="si64", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32_refine", choices=["fp32_refine", "fp64"])
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--slots-per-cu", type=int, default=0)
    ap.add_argument("--tile-y", type=int, default=0)
    ap.add_argument("--use-graph", action="store_true",
                    help="replay each batch's kernel sequence as a captured HIP graph")
    ap.add_argument("--autotune", action="store_true",
                    help="choose tile rows and workgroups per CU with rpa_autotune first")
    ap.add_argument("--inner-tol", type=float, default=0.0,
                    help="reliable-update factor of the FP32 COCG (0: library default)")
    ap.add_argument("--orbital-cache", default="", help="npz file to reuse/save the orbitals")
    ap.add_argument("--precond", action="store_true",
                    help="preconditioned Sternheimer solves (shifted kinetic operator) at every "
                         "frequency")
    ap.add_argument("--precond-window", type=float, nargs=2, default=None, metavar=("LO", "HI"),
                    help="precondition only the solves with LO <= omega <= HI (HI 0: no bound)")
    ap.add_argument("--plain", action="store_true",
                    help="plain COCG at every frequency (overrides the workload's default window)")
    ap.add_argument("--extra", type=int, default=None,
                    help="extra eigenpairs above the occupied ones in the Galerkin guess "
                         "(default: the workload's)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-only", action="store_true",
                    help="only the serving measurement, at the settings below; prints its own JSON line")
    ap.add_argument("--serve-nl", type=int, default=8)
    ap.add_argument("--serve-tol", type=float, default=1e-6)
    ap.add_argument("--serve-block", type=int, default=32, help="coarse points per job")
    ap.add_argument("--serve-jobs", type=int, default=110, help="open-loop jobs per load level")
    ap.add_argument("--serve-closed", type=int, default=24, help="closed-loop jobs (saturation)")
    ap.add_argument("--serve-budget-gb", type=float, default=288.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the plain copy used to scale HBM counters")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the per-point work "
              "is independent, so N GPUs would shard the (point, frequency) list with no "
              "communication inside a frequency and one all-gather of the coarse diagonals per "
              "frequency.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2609_16408_amd as P
    import synthcell as sc

    cfg = WORKLOADS[args.workload]
    if "precision" in cfg:
        args.precision = cfg["precision"]
    if args.plain:
        args.precond, args.precond_window = False, None
    elif args.precond_window is None and not args.precond and "precond_window" in cfg:
        args.precond_window = list(cfg["precond_window"])
    if args.precond_window is not None:
        args.precond = True
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    log(f"[bench] building the {cfg['preset']} cell")
    if args.extra is None:
        args.extra = int(cfg.get("n_extra", 0))
    cell = load_or_make_cell(sc, cfg["preset"], args.orbital_cache, args.extra)
    log(f"[bench] cell {cfg['preset']} n={cell.n} N_s={cell.n_occ} gap={cell.gap:.2e} "
        f"eig residual={cell.eig_residual:.1e} setup {time.perf_counter() - t0:.1f}s")
    omega, weight = P.frequency_rule(8)
    if args.serving_only:
        # the serving protocol at the given settings (the Si64-like cell of
        # this workload is the pool's large cell)
        r = serving_run(P, sc, cell, omega, log, n_closed=args.serve_closed, n_open=args.serve_jobs,
                        warm=10, n_lanczos=args.serve_nl, tol=args.serve_tol, block=args.serve_block,
                        budget_gb=args.serve_budget_gb)
        print(json.dumps({"serving": r, "data": "synthetic", "n_gpus": 1}), flush=True)
        return
    stride = cfg["stride"]
    coarse = sc.coarse_points(cell.n, stride)
    subset = sc.sublattice_points(cell.n, stride, cfg["every"])
    pos_in_coarse = np.searchsorted(coarse, subset)
    assert np.array_equal(coarse[pos_in_coarse], subset)
    pps = cfg["pts_per_step"]
    n_batches = len(subset) // pps
    needed = args.warmup + args.steps
    assert needed <= n_batches, "not enough distinct point batches"

    def make_handle(precision, plain=False):
        return P.handle_for_cell(cell, precision=precision, stern_tol=cfg["tol"],
                                 stern_maxit=20000, batch=pps * 8, slots_per_cu=args.slots_per_cu,
                                 tile_y=args.tile_y, inner_tol=args.inner_tol,
                                 use_graph=args.use_graph, precond=args.precond and not plain,
                                 precond_window=None if plain else args.precond_window,
                                 progress=bool(cfg.get("progress", False)),
                                 extra=(cell.psi_extra, cell.eps_extra) if args.extra > 0 and not plain
                                 else None)

    h = make_handle(args.precision)
    tuned = None
    if args.autotune:
        tuned = h.autotune(n_lanczos=cfg["n_lanczos"])
        log(f"[bench] autotune: {tuned}")
    d_coarse = torch.zeros((8, coarse.size), dtype=torch.float64, device="cuda")

    def step(hd, i):
        pts = subset[i * pps:(i + 1) * pps]
        d, st = hd.lanczos_energy_density(omega, pts, cfg["n_lanczos"])
        idx = torch.from_numpy(pos_in_coarse[i * pps:(i + 1) * pps]).to("cuda")
        d_coarse.index_copy_(1, idx, d)
        e_c, _ = hd.energy_from_coarse(weight, stride, cfg["interp"], d_coarse, want_fine=True)
        tm = hd.last_cocg_timing()
        tm["split"] = hd.last_cocg_split()
        st["per_omega"] = hd.last_iteration_stats()
        return st, tm, e_c

    def pool_omega(stats_list):
        """Per-frequency COCG iteration statistics pooled over steps."""
        acc = {}
        for st in stats_list:
            for r in st["per_omega"]:
                a = acc.setdefault(r["omega"], [0, 0.0, 0.0, None, 0, 0])
                a[0] += r["solves"]
                a[1] += r["mean"] * r["solves"]
                a[2] += (r["std"] ** 2 + r["mean"] ** 2) * r["solves"]
                a[3] = r["min"] if a[3] is None else min(a[3], r["min"])
                a[4] = max(a[4], r["max"])
                a[5] += r["refine_cycles"]
        out = []
        for w in sorted(acc):
            c, s1, s2, mn, mx, cyc = acc[w]
            m = s1 / c
            out.append({"omega": w, "solves": c, "mean": round(m, 2),
                        "std": round(math.sqrt(max(0.0, s2 / c - m * m)), 2), "min": mn, "max": mx,
                        "iters_total": int(round(s1)), "refine_cycles": cyc})
        return out

    for i in range(args.warmup):
        st, tm, _ = step(h, i)
        log(f"[bench] warmup {i}: {st['seconds']:.2f}s iters/system "
            f"{st['cocg_iters_total'] / st['n_systems']:.1f} max {st['cocg_iters_max']}")
    torch.cuda.synchronize()
    stats, cocg_ms, cocg_launches = [], 0.0, 0
    split_ms = {"plain": 0.0, "precond": 0.0, "followup": 0.0}
    t_start = time.perf_counter()
    for i in range(args.warmup, needed):
        st, tm, e_c = step(h, i)
        stats.append(st)
        cocg_ms += tm["ms"]
        cocg_launches += tm["launches"]
        for k in split_ms:
            split_ms[k] += tm["split"][k]
        log(f"[bench] step {i}: {st['seconds']:.2f}s iters/system "
            f"{st['cocg_iters_total'] / st['n_systems']:.1f} max {st['cocg_iters_max']} "
            f"cycles {st['refine_cycles']} noconv {st['n_noconv']}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    n_points = args.steps * pps * 8
    value = n_points / elapsed
    tot = {k: sum(s[k] for s in stats) for k in ("n_systems", "cocg_iters_total", "refine_cycles",
                                                 "n_noconv", "n_breakdown")}
    nl_sup = nl_support_points(cell.proj)
    per_omega = pool_omega(stats)
    kt = kind_totals(per_omega, args.precond, args.precond_window)
    timing = h.last_cocg_timing()
    # one roofline entry per Sternheimer kernel that ran: algorithmic bytes (and
    # for the preconditioned kernel also MFMA flops) over that kernel's own
    # event-timed launches; the FP64 follow-up launch of handed-over solves is
    # added to the kernel whose solves it finishes
    kernels = []
    for kind, name, ms in ((0, "k_cocg (batched Sternheimer COCG)", split_ms["plain"]),
                           (1, "k_cocg preconditioned (batched Sternheimer PCOCG)", split_ms["precond"])):
        t = kt[kind]
        if t["n_systems"] == 0:
            continue
        if kind == (1 if args.precond else 0):
            ms += split_ms["followup"]
        b = cocg_algorithmic_bytes(t, cell.N_d, args.precision, nl_sup)
        e = {"kernel": name, "ms": ms, "launches": cocg_launches, "systems": t["n_systems"],
             "iters_per_system": t["cocg_iters_total"] / t["n_systems"]}
        if kind == 1:
            pb, pf = precond_algorithmic(t, cell.n, args.precision)
            b += pb
            mfma_peak = 157.3 if args.precision == "fp32_refine" else 78.6
            e["mfma"] = {"achieved": pf / (ms * 1e-3) / 1e12 if ms > 0 else None, "peak": mfma_peak,
                         "unit": "TFLOP/s", "flops_per_launch": pf / cocg_launches}
            e["mfma"]["frac"] = e["mfma"]["achieved"] / mfma_peak if ms > 0 else None
        e["algorithmic_bytes_per_launch"] = b / cocg_launches
        # graph replay records no per-kernel events: no kernel rate then
        e["achieved_gbps"] = b / (ms * 1e-3) / 1e9 if ms > 0 else None
        e["hbm_frac"] = e["achieved_gbps"] / HBM_PEAK_GBPS if ms > 0 else None
        kernels.append(e)
    dom = max(kernels, key=lambda e: e["ms"])
    alg_bytes = dom["algorithmic_bytes_per_launch"] * cocg_launches
    achieved = dom["achieved_gbps"]
    # the preconditioned kernel is priced against whichever ceiling it is closer to
    use_mfma = "mfma" in dom and dom["mfma"]["frac"] is not None and dom["hbm_frac"] is not None \
        and dom["mfma"]["frac"] > dom["hbm_frac"]
    traffic = pmc_traffic(args.workload, args.precond, args.precond_window, args.extra) \
        if args.precision == "fp32_refine" else None

    extra = {}
    if not args.no_fp64_compare and args.precision == "fp32_refine":
        # the plain FP64 GPU form (no preconditioner) on the same point
        # batches: one untimed warm-up step, then up to two timed ones
        h64 = make_handle("fp64", plain=True)
        n64 = max(1, min(args.steps, 2))
        st64, _, _ = step(h64, 0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sts64, ms64 = [], 0.0
        for i in range(args.warmup, args.warmup + n64):
            st, tm, _ = step(h64, i)
            sts64.append(st)
            ms64 += tm["ms"]
            log(f"[bench] fp64 step {i}: {st['seconds']:.2f}s iters/system "
                f"{st['cocg_iters_total'] / st['n_systems']:.1f} max {st['cocg_iters_max']}")
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        tot64 = {k: sum(x[k] for x in sts64) for k in ("n_systems", "cocg_iters_total", "refine_cycles")}
        extra["fp64_points_per_s"] = n64 * pps * 8 / t64
        extra["fp64_steps"] = n64
        extra["speedup_vs_fp64"] = value / extra["fp64_points_per_s"]
        extra["fp64_cocg_gbps"] = cocg_algorithmic_bytes(tot64, cell.N_d, "fp64", nl_sup) / (ms64 * 1e-3) / 1e9
        extra["fp64_iters_per_system"] = tot64["cocg_iters_total"] / tot64["n_systems"]
        h64.close()
    sgbps, sms = stencil_gbps(P, h, cell, torch)
    extra["stencil_fp32_gbps"] = sgbps
    extra["stencil_fp32_frac"] = sgbps / HBM_PEAK_GBPS
    h.close()

    if not args.no_serving and args.workload == "si64":
        try:
            extra["serving"] = serving_run(P, sc, cell, omega, log)
            extra["p99_latency_s"] = extra["serving"]["load_0.9"]["p99_latency_s"]
        except Exception as e:  # serving must not hide the main measurement
            log(f"[bench] serving failed: {e!r}")

    cpu = None
    if not args.no_cpu_baseline:
        try:
            log("[bench] cpu baseline (oracle, one process per core)")
            cpu = cpu_baseline(cell, cfg, [float(w) for w in omega])
            log(f"[bench] cpu baseline: {cpu['value']:.3g} points/s; {cpu['sample']}")
        except Exception as e:  # the baseline must not hide the GPU result
            log(f"[bench] cpu baseline failed: {e!r}")

    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "fp32_refine" else "f64",
        "data": "synthetic",
        "config": {"workload": cfg["desc"], "precision": args.precision,
                   "n_lanczos": cfg["n_lanczos"], "stern_tol": cfg["tol"], "n_omega": 8,
                   "points_per_step": pps * 8, "coarse_stride": stride,
                   "interp": cfg["interp"], "precond": bool(args.precond),
                   "precond_window": args.precond_window,
                   "sternheimer_mode": cocg_mode(args.precond, args.precond_window),
                   "galerkin_extra_states": args.extra,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma" if use_mfma else "hbm",
                     "achieved": dom["mfma"]["achieved"] if use_mfma else achieved,
                     "peak": dom["mfma"]["peak"] if use_mfma else HBM_PEAK_GBPS,
                     "unit": "TFLOP/s" if use_mfma else "GB/s",
                     "frac": dom["mfma"]["frac"] if use_mfma else (achieved / HBM_PEAK_GBPS if achieved else None),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": alg_bytes / cocg_launches if cocg_launches else None,
                     "kernel": dom["kernel"], "cocg_source_sha": source_sha(),
                     "launches": cocg_launches, "avg_launch_ms": dom["ms"] / max(1, cocg_launches),
                     "all_cocg_avg_launch_ms": cocg_ms / max(1, cocg_launches),
                     "kernels": kernels,
                     "grid": timing["grid"], "block": timing["block"], "tile_y": timing["tile_y"]},
        "cpu_baseline": cpu,
        "launch": {"use_graph": bool(args.use_graph), "autotuned": tuned},
        "cocg": {"iters_per_system": tot["cocg_iters_total"] / max(1, tot["n_systems"]),
                 "refine_cycles_per_system": tot["refine_cycles"] / max(1, tot["n_systems"]),
                 "noconv": tot["n_noconv"], "E_c_partial": e_c,
                 "E_c_complete": bool(needed * pps >= len(subset) and cfg["every"] == 1),
                 "per_omega": per_omega},
    }
    rec.update(extra)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
