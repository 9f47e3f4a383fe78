"""Host-side logic of bench.py: the solver-mode key, the split of the
per-frequency COCG totals between the plain and the preconditioned kernel,
the preconditioner's algorithmic bytes and flops, the algorithmic bytes of
the COCG launches, and the lookup of the committed counter-traffic summary."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_solver_mode_key():
    assert bench.cocg_mode(False, None) == "plain"
    assert bench.cocg_mode(True, None) == "precond"
    assert bench.cocg_mode(True, [0.5, 20.0]) == "precond_window 0.5 20"


def _per_omega():
    om = [0.0203, 0.113, 0.311, 0.69, 1.45, 3.22, 8.84, 49.4]
    return [{"omega": w, "solves": 10, "iters_total": 100 * (i + 1), "refine_cycles": 3 * (i + 1)}
            for i, w in enumerate(om)]


def test_kind_totals_follow_the_window():
    po = _per_omega()
    t = bench.kind_totals(po, True, [0.5, 20.0])
    # preconditioned: 0.69, 1.45, 3.22, 8.84 (entries 4..7 of the list, 1-based)
    assert t[1]["n_systems"] == 40 and t[1]["cocg_iters_total"] == 100 * (4 + 5 + 6 + 7)
    assert t[0]["n_systems"] == 40 and t[0]["cocg_iters_total"] == 100 * (1 + 2 + 3 + 8)
    assert t[0]["refine_cycles"] + t[1]["refine_cycles"] == 3 * 36
    everything = bench.kind_totals(po, True, None)
    assert everything[0]["n_systems"] == 0 and everything[1]["n_systems"] == 80
    plain = bench.kind_totals(po, False, None)
    assert plain[1]["n_systems"] == 0 and plain[0]["cocg_iters_total"] == 3600
    open_top = bench.kind_totals(po, True, [0.5, 0.0])          # no upper bound
    assert open_top[1]["n_systems"] == 50


def test_algorithmic_counts():
    st = {"n_systems": 2, "cocg_iters_total": 10, "refine_cycles": 3}
    N = 1000
    # FP32 + refinement: 80 B/pt per iteration and per reliable update, 40 per system
    assert bench.cocg_algorithmic_bytes(st, N, "fp32_refine") == (800 + 240 + 80) * N
    # FP64: 160 B/pt per iteration, 48 per system
    assert bench.cocg_algorithmic_bytes(st, N, "fp64") == (1600 + 96) * N
    b, f = bench.precond_algorithmic(st, (10, 10, 10), "fp32_refine")
    assert b == 48.0 * 10 * N and f == 8.0 * 30 * 10 * N
    b64, _ = bench.precond_algorithmic(st, (10, 10, 10), "fp64")
    assert b64 == 2 * b


def test_traffic_summary_lookup_is_keyed():
    path = bench.PMC_SUMMARY
    assert os.path.exists(path)
    vals = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    mode = vals["mode"]
    window = None
    if mode.startswith("precond_window"):
        window = [float(x) for x in mode.split()[1:]]
    extra = int(vals.get("galerkin_extra", "0"))
    precond = mode != "plain"
    hit = bench.pmc_traffic(vals["workload"], precond, window, extra)
    if vals["cocg_source_sha"] == bench.source_sha():
        assert hit == float(vals["hbm_bytes_per_launch"])
    else:
        assert hit is None
    assert bench.pmc_traffic("si8", precond, window, extra) is None
    assert bench.pmc_traffic(vals["workload"], precond, window, extra + 1) is None
