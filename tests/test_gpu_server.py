"""Serving loop on the GPU: a job's result is the same alone and in a mix of
concurrent jobs on other cells and frequencies (batching happens inside a job
only and every reduction has a fixed order, so the match is bit for bit)."""
import numpy as np
import pytest

import synthcell as sc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2609_16408_amd as P
    assert torch.cuda.is_available()
    return P


@pytest.fixture(scope="module")
def cells():
    return sc.preset("tiny"), sc.preset("si8")


def _add(server, c):
    return server.add_cell(c.n, c.L, c.v_loc, c.psi, c.eps, precision="fp32_refine",
                           stern_tol=1e-8)


def test_job_result_identical_alone_in_mix_and_direct(P, cells):
    tiny, si8 = cells
    pts_a = sc.coarse_points(tiny.n, 2)[5:25]
    pts_b = sc.coarse_points(si8.n, 2)[100:140]
    # alone
    s1 = P.Server(n_workers=1)
    a_id, b_id = _add(s1, tiny), _add(s1, si8)
    d_a_alone, info = s1.wait(s1.submit(a_id, 0.31, pts_a, 4))
    assert info["status"] == 0
    d_b_alone, _ = s1.wait(s1.submit(b_id, 1.45, pts_b, 4))
    s1.close()
    # in a mix of concurrent jobs (3 workers, 6 jobs in flight)
    s3 = P.Server(n_workers=3)
    a3, b3 = _add(s3, tiny), _add(s3, si8)
    jobs = [s3.submit(b3, 0.02, pts_b[:16], 4), s3.submit(a3, 0.31, pts_a, 4),
            s3.submit(b3, 1.45, pts_b, 4), s3.submit(a3, 8.8, pts_a[:8], 4),
            s3.submit(b3, 0.69, pts_b[8:30], 4), s3.submit(a3, 0.31, pts_a, 4)]
    res = [s3.wait(j) for j in jobs]
    s3.close()
    assert all(r[1]["status"] == 0 for r in res)
    starts = sorted((r[1]["t_start"], r[1]["t_finish"]) for r in res)
    assert any(b[0] < a[1] for a, b in zip(starts, starts[1:])), "jobs did not overlap"
    assert torch.equal(res[1][0], d_a_alone) and torch.equal(res[5][0], d_a_alone)
    assert torch.equal(res[2][0], d_b_alone)
    # and the same as the plain handle path
    h = P.handle_for_cell(tiny, precision="fp32_refine", stern_tol=1e-8)
    d_direct, _ = h.lanczos_energy_density([0.31], pts_a, 4)
    h.close()
    assert torch.equal(d_direct[0], d_a_alone)


def test_server_job_with_projectors_matches_direct_handle(P):
    """A cell with nonlocal projectors goes through the serving loop unchanged."""
    c = sc.preset("tiny", with_projectors=True, proj_seed=201)
    pts = sc.coarse_points(c.n, 2)[:24]
    s = P.Server(n_workers=2)
    cid = s.add_cell(c.n, c.L, c.v_loc, c.psi, c.eps, precision="fp32_refine", stern_tol=1e-8,
                     proj=c.proj)
    d_a, info = s.wait(s.submit(cid, 0.69, pts, 4))
    s.close()
    assert info["status"] == 0
    h = P.handle_for_cell(c, precision="fp32_refine", stern_tol=1e-8)
    d_b, _ = h.lanczos_energy_density([0.69], pts, 4)
    h.close()
    assert torch.equal(d_b[0], d_a)
