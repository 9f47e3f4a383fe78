"""Host-side tests of the serving loop's scheduler (fake executor: jobs sleep
instead of computing, so admission, ordering and latency accounting are
checked without a GPU)."""
import numpy as np
import pytest

import paper_2609_16408_amd as P
from paper_2609_16408_amd import serve

US = 30000  # fake job length (microseconds)


def _server(workers, budget=0):
    s = P.Server(n_workers=workers, hbm_budget=budget, fake_executor_us=US)
    cid = s.add_cell((24, 24, 24), (10.26,) * 3, None, None, np.linspace(-0.5, -0.4, 16))
    return s, cid


def _overlaps(infos):
    """Largest number of jobs running at the same time (event sweep)."""
    ev = sorted([(i["t_start"], 1) for i in infos] + [(i["t_finish"], -1) for i in infos],
                key=lambda e: (e[0], e[1]))
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


def test_concurrent_jobs_overlap_up_to_the_worker_count():
    s, cid = _server(3)
    ids = [s.submit(cid, 0.5, np.arange(16), 4) for _ in range(6)]
    infos = [s.wait(j)[1] for j in ids]
    s.close()
    assert all(i["status"] == 0 for i in infos)
    assert _overlaps(infos) == 3
    assert all(i["latency"] >= US * 1e-6 for i in infos)


def test_admission_respects_the_hbm_budget():
    s0, cid0 = _server(1)
    fp = s0.wait(s0.submit(cid0, 0.5, np.arange(16), 4))[1]["footprint"]
    s0.close()
    N = 24 ** 3
    worker = N * 8 * 17 + N * (4 + 2 * 8) + 16 * 8 + 3 * 24 * 24 * 8   # what rpa_setup keeps
    resident = N * 8 * 17 + 3 * worker       # server's V + 16 orbitals, 3 worker copies
    s, cid = _server(3, budget=resident + int(1.5 * fp))   # room for one job at a time
    ids = [s.submit(cid, 0.5, np.arange(16), 4) for _ in range(4)]
    infos = [s.wait(j)[1] for j in ids]
    s.close()
    assert _overlaps(infos) == 1
    # oldest first: start times follow submission order
    starts = [i["t_start"] for i in infos]
    assert starts == sorted(starts)


def test_job_that_can_never_fit_is_refused():
    s, cid = _server(2, budget=1 << 20)
    with pytest.raises(P.RPAError) as e:
        s.submit(cid, 0.5, np.arange(16), 4)
    assert e.value.status == P.RPA_E_OOM
    s.close()


@pytest.mark.parametrize("bad", [dict(omega=0.0), dict(points=[24 ** 3]), dict(n_lanczos=0),
                                 dict(cell=7)])
def test_invalid_jobs_are_rejected(bad):
    s, cid = _server(1)
    kw = dict(cell=cid, omega=0.5, points=[0, 1], n_lanczos=4)
    kw.update(bad)
    with pytest.raises(P.RPAError) as e:
        s.submit(kw["cell"], kw["omega"], kw["points"], kw["n_lanczos"])
    assert e.value.status == P.RPA_E_ARG
    s.close()


def test_open_loop_driver_reports_latency_percentiles():
    s, cid = _server(2)
    cells = [(cid, np.arange(0, 24 ** 3, 8))]
    jobs = serve.make_jobs(12, cells, [1.0], [0.5, 3.2], 16, seed=4000)
    secs, infos = serve.run_open(s, cells, jobs, 4, rate=40.0, seed=4001)
    s.close()
    r = serve.summarize(infos, secs)
    assert r["jobs"] == 12 and r["p99_latency_s"] >= r["p50_latency_s"] >= US * 1e-6


def test_status_reports_admission_high_water():
    """The high-water mark covers resident cell data plus every admitted job's
    workspace estimate at its peak."""
    s = P.Server(n_workers=2, fake_executor_us=20000)
    cid = s.add_cell((24, 24, 24), (10.26,) * 3, None, None, np.linspace(-1, -0.5, 16),
                     precision="fp32_refine")
    idle = s.status()
    assert idle["in_use"] == 0 and idle["high_water"] > 0     # resident data only
    jobs = [s.submit(cid, 0.5, np.arange(64 * k, 64 * k + 64), 4) for k in range(4)]
    infos = [s.wait(j)[1] for j in jobs]
    st = s.status()
    assert st["in_use"] == 0
    assert st["high_water"] >= idle["high_water"] + max(i["footprint"] for i in infos)
    s.close()


def test_cells_added_while_jobs_run():
    """Cells added while workers run jobs of earlier cells: every job
    finishes, on the cell it names (workers keep the cell they took under the
    server's lock, so growing the cell table cannot move it under them)."""
    s, cid = _server(3)
    ids = [(cid, s.submit(cid, 0.5, np.arange(16), 4)) for _ in range(3)]
    for k in range(40):
        c = s.add_cell((24, 24, 24 + 12 * (k % 2)), (10.26,) * 3, None, None,
                       np.linspace(-0.5, -0.4, 16))
        ids.append((c, s.submit(c, 0.5, np.arange(8), 2)))
    infos = [(c, s.wait(j)[1]) for c, j in ids]
    s.close()
    assert all(i["status"] == 0 for _, i in infos)
    # footprints follow the grid of the cell each job named
    fp = {}
    for c, i in infos[3:]:
        fp.setdefault(c % 2, set()).add(i["footprint"])
    assert len(fp) == 2 and all(len(v) == 1 for v in fp.values()) and fp[0] != fp[1]
