"""Widened Galerkin initial guess (extra eigenpairs above the occupied ones,
rpa_setup_params.n_extra): the Sternheimer solutions and chi0 are those of
the plain guess (same stopping rule), checked against the oracle's chi0
with and without the widened space (oracle.chi0_apply psi_extra/eps_extra),
and the COCG iterations at small omega drop."""
import numpy as np
import pytest

import oracle as O
import synthcell as sc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2609_16408_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.lib()
    return P


@pytest.fixture(scope="module")
def tiny_x():
    return sc.preset("tiny", n_extra=8)


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_widened_galerkin_guess_keeps_chi0_and_cuts_iterations(P, tiny_x, precision):
    c = tiny_x
    ham, coul = O.Hamiltonian(c.n, c.L, c.v_loc), O.Coulomb(c.n, c.L)
    tol = 1e-10 if precision == "fp64" else 1e-8
    u = np.random.default_rng(71).standard_normal((2, c.N_d))
    out, its = {}, {}
    for key, extra in (("plain", None), ("wide", (c.psi_extra, c.eps_extra))):
        h = P.handle_for_cell(c, precision=precision, stern_tol=tol, batch=2, extra=extra)
        y, st = h.chi0_apply(0.0203, torch.from_numpy(u))
        its[key] = h.last_iteration_stats()[0]["mean"]
        h.close()
        assert st["n_noconv"] == 0
        out[key] = y.cpu().numpy()
    ref = np.stack([O.chi0_apply(ham, c.psi, c.eps, u[i], 0.0203, tol=1e-12) for i in range(2)])
    ref_w = np.stack([O.chi0_apply(ham, c.psi, c.eps, u[i], 0.0203, tol=1e-12, psi_extra=c.psi_extra,
                                   eps_extra=c.eps_extra) for i in range(2)])
    scale = np.abs(ref).max()
    err_w = np.abs(out["wide"] - ref).max() / scale
    err_p = np.abs(out["plain"] - ref).max() / scale
    print(f"{precision}: iterations plain {its['plain']:.1f}, widened {its['wide']:.1f}; "
          f"relative chi0 error plain {err_p:.1e}, widened {err_w:.1e}; "
          f"oracle widened vs plain {np.abs(ref_w - ref).max() / scale:.1e}", flush=True)
    lim = 1e-7 if precision == "fp64" else 1e-5
    assert err_w <= lim and err_p <= lim
    assert np.abs(ref_w - ref).max() / scale <= 1e-9
    assert its["wide"] < its["plain"]


def test_si64_benchmark_configuration_matches_plain_fp64(P):
    """The benchmark's Si64 configuration (FP32 + refinement, 384 extra
    eigenpairs in the Galerkin guess, preconditioned solves for
    0.5 <= omega <= 20) against the plain FP64 form (occupied Galerkin space,
    no preconditioner) on one batch of 8 points x 8 frequencies: every
    diagonal <= 0 and the energy difference, extrapolated over all N_d fine
    points, within 1e-5 Ha/atom; the widened guess must also cut the COCG
    iterations at the smallest frequency."""
    import math
    c = sc.preset("si64", device="cuda", n_extra=384)
    om, w = P.frequency_rule(8)
    pts = sc.sublattice_points(c.n, 2, 3)[:8]
    h = P.handle_for_cell(c, precision="fp32_refine", stern_tol=1e-6, batch=64,
                          precond=True, precond_window=(0.5, 20.0), extra=(c.psi_extra, c.eps_extra))
    d32, st32 = h.lanczos_energy_density(om, pts, 8)
    s32 = h.last_iteration_stats()
    h.close()
    h = P.handle_for_cell(c, precision="fp64", stern_tol=1e-6, batch=64)
    d64, st64 = h.lanczos_energy_density(om, pts, 8)
    s64 = h.last_iteration_stats()
    h.close()
    assert st32["n_noconv"] == 0 and st64["n_noconv"] == 0
    d32, d64 = d32.cpu().numpy(), d64.cpu().numpy()
    assert (d32 <= 0).all() and (d64 <= 0).all()
    dE = (c.N_d / len(pts)) * float(np.abs(w @ (d32 - d64)).sum()) / (2 * math.pi) / c.n_atoms
    print(f"si64 benchmark configuration vs plain FP64: max |dd| = {np.abs(d32 - d64).max():.2e}, "
          f"extrapolated |dE|/atom = {dE:.2e}; iterations at omega = {s32[0]['omega']:.4g}: "
          f"{s32[0]['mean']:.1f} (plain FP64 {s64[0]['mean']:.1f})", flush=True)
    assert dE <= 1e-5, dE
    assert s32[0]["mean"] < 0.5 * s64[0]["mean"]
