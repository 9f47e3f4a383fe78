"""Shifted kinetic preconditioner (rpa_kinetic_precond_apply) against the oracle.

The preconditioner of preconditioned Sternheimer solves (Conclusions and Future
Work): (-1/2 Lap_h + sigma)^-1 in the per-axis eigenbasis of the FD Laplacian.
"""
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


def _handle(P, grid, L):
    atoms = sc.diamond_atoms((1, 1, 1), seed=7) * np.array(L) / 10.26
    v = sc.gaussian_vloc(grid, L, atoms)
    N = int(np.prod(grid))
    psi = np.zeros((1, N))
    psi[0, 0] = 1.0
    return P.Handle(grid, L, v, psi, np.array([-0.5]))


@pytest.mark.parametrize("grid", [(12, 12, 12), (14, 12, 10), (9, 24, 72), (48, 48, 48)])
def test_kinetic_precond_matches_oracle(P, grid):
    L = tuple(10.26 * g / 24 for g in grid)
    print("kinetic preconditioner", grid, flush=True)
    h = _handle(P, grid, L)
    N = int(np.prod(grid))
    rng = np.random.default_rng(17)
    nv = 3
    x = rng.standard_normal((nv, N)) + 1j * rng.standard_normal((nv, N))
    sig = np.array([0.25 - 0.0203j, 1.3 - 3.2j, 0.7 + 0.0j])
    y = h.kinetic_precond_apply(torch.from_numpy(x), sig).cpu().numpy()
    pc = O.KineticPreconditioner(grid, L)
    for b in range(nv):
        ref = pc.apply(x[b], sig[b])
        err = np.abs(y[b] - ref).max() / np.abs(ref).max()
        assert err < 1e-12, (b, err)
    h.close()


def test_kinetic_precond_inverts_the_shifted_stencil_and_checks_sigma(P):
    """M^-1 M v = v with M applied by the GPU Hamiltonian on a zero potential."""
    grid = (12, 12, 12)
    L = (10.26,) * 3
    N = int(np.prod(grid))
    psi = np.zeros((1, N))
    psi[0, 0] = 1.0
    h = P.Handle(grid, L, np.zeros(N), psi, np.array([-0.5]))
    v = np.random.default_rng(3).standard_normal((2, N)) + 0j
    sig = np.array([0.25 - 0.5j, 2.0 + 0.1j])
    Mv = h.hamiltonian_apply(-sig, torch.from_numpy(v), precision="fp64")
    back = h.kinetic_precond_apply(Mv, sig).cpu().numpy()
    assert np.abs(back - v).max() < 1e-12 * np.abs(v).max()
    with pytest.raises(P.RPAError) as e:
        h.kinetic_precond_apply(torch.from_numpy(v), np.array([0.25, -0.1 + 0j]))
    assert e.value.status == P.RPA_E_ARG
    h.close()


# --- preconditioned COCG inside the persistent solver (precond=1) --------------------

from bounds import residual_error_bound  # noqa: E402


@pytest.fixture(scope="module")
def pcells():
    long = sc.make_cell("long", cells=(3, 2, 1), n=(36, 24, 12), n_occ=16, seed=9)
    sc.ks_orbitals(long)
    return {"tiny": sc.preset("tiny"), "long": long, "si8": sc.preset("si8")}


def _oracle_solutions(ham, c, u, omega, tol, pc):
    """The oracle's preconditioned COCG (reading R17) per orbital: solutions
    and iteration counts."""
    xs, its = [], []
    for n in range(c.n_occ):
        b = -c.psi[n] * u
        z = c.eps[n] + 1j * omega
        x0 = O.galerkin_guess(c.psi, c.eps, n, b, omega, ham.dV)
        sg = O.kinetic_shift(c.v_loc, c.eps[n], omega)
        x, it, status = O.cocg_precond(lambda v, z=z: ham.apply(v) - z * v,
                                       lambda r, sg=sg: pc.apply(r, sg), b, x0, tol, 20000)
        assert status == "ok"
        xs.append(x)
        its.append(it)
    return np.array(xs), its


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("name,omega", [("tiny", 0.0203), ("tiny", 0.69), ("long", 0.31),
                                        ("si8", 0.0203), ("si8", 3.22)])
def test_preconditioned_solves_match_oracle(P, pcells, precision, name, omega):
    """Grids whose padded tile sizes differ per axis (16; 48 x 32 x 16; 32):
    every GPU solution meets the unpreconditioned stopping rule on its true
    residual, chi0 u matches the oracle's preconditioned route within the
    bound the residuals of both give, and the FP64 solver takes the
    oracle's iteration counts (the same recurrence; rounding may move a stop
    by one iteration)."""
    c = pcells[name]
    tol = 1e-10 if precision == "fp64" else 1e-8
    slack = 1.0 if precision == "fp32_refine" else 2.0
    ham = O.Hamiltonian(c.n, c.L, c.v_loc)
    pc = O.KineticPreconditioner(c.n, c.L)
    h = P.handle_for_cell(c, precision=precision, stern_tol=tol, precond=True, batch=2)
    u = np.random.default_rng(61).standard_normal((2, c.N_d))
    xs, st = h.sternheimer_solve(omega, torch.from_numpy(u))
    y, st2 = h.chi0_apply(omega, torch.from_numpy(u))
    stats = h.last_iteration_stats()[0]
    h.close()
    xs, y = xs.cpu().numpy(), y.cpu().numpy()
    assert st["n_noconv"] == 0 and st2["n_noconv"] == 0
    its_or = []
    for i in range(2):
        r, b, bound = residual_error_bound(ham, c.psi, c.eps, u[i], omega, xs[i])
        assert np.all(r <= slack * tol * b), (i, (r / b).max())
        xo, it = _oracle_solutions(ham, c, u[i], omega, 1e-12, pc)
        ref = 4.0 * np.sum(c.psi * xo.real, axis=0)
        ref_err = residual_error_bound(ham, c.psi, c.eps, u[i], omega, xo)[2]
        err = np.abs(y[i] - ref).max()
        assert err <= bound + ref_err, (i, err, bound, ref_err)
        its_or += _oracle_solutions(ham, c, u[i], omega, tol, pc)[1]
    print(f"{name} omega={omega} {precision}: GPU preconditioned iterations per solve "
          f"{stats['mean']:.2f} (max {stats['max']}), oracle {np.mean(its_or):.2f} (max {max(its_or)})",
          flush=True)
    if precision == "fp64":
        assert abs(stats["mean"] - np.mean(its_or)) <= 1.0 and abs(stats["max"] - max(its_or)) <= 1


def test_preconditioned_lanczos_matches_oracle(P, pcells):
    """Algorithm 1 with preconditioned solves, FP64: within 1e-8 of the
    oracle's preconditioned route, and fewer COCG iterations than plain."""
    c = pcells["tiny"]
    ham, coul = O.Hamiltonian(c.n, c.L, c.v_loc), O.Coulomb(c.n, c.L)
    pc = O.KineticPreconditioner(c.n, c.L)
    om, _ = O.frequency_rule(2)
    pts = O.coarse_index_set(c.n, 6)
    h = P.handle_for_cell(c, stern_tol=1e-10, precond=True)
    d, st = h.lanczos_energy_density(om, pts, 8)
    h.close()
    h0 = P.handle_for_cell(c, stern_tol=1e-10)
    _, st0 = h0.lanczos_energy_density(om, pts, 8)
    h0.close()
    ref = O.energy_density(ham, coul, c.psi, c.eps, om, pts, 8, tol=1e-10, precond=pc, v_loc=c.v_loc)
    assert np.abs(d.cpu().numpy() - ref).max() <= 1e-8
    assert st["cocg_iters_total"] < 0.6 * st0["cocg_iters_total"], (st, st0)


def test_preconditioned_setup_rejects_large_grids(P):
    grid = (9, 24, 72)
    N = int(np.prod(grid))
    psi = np.zeros((1, N))
    psi[0, 0] = 1.0
    with pytest.raises(P.RPAError) as e:
        P.Handle(grid, (5.0, 10.0, 30.0), np.zeros(N), psi, np.array([-0.5]), precond=True)
    assert e.value.status == P.RPA_E_ARG


def test_preconditioner_frequency_window(P, pcells):
    """With a frequency window, solves inside it take the preconditioned
    kernels and the others the plain ones, in the same Lanczos steps: each
    frequency's energy density is bitwise that of the all-plain or
    all-preconditioned handle (per-system results do not depend on the
    launch they ran in), and the per-frequency statistics show which."""
    c = pcells["tiny"]
    om = np.array([0.0203, 0.69, 3.22])
    pts = np.array([0, 333, 1000, 1727])
    runs = {}
    split = {}
    for key, kw in (("plain", {}), ("all", {"precond": True}),
                    ("window", {"precond": True, "precond_window": (0.5, 5.0)})):
        h = P.handle_for_cell(c, stern_tol=1e-10, **kw)
        d, st = h.lanczos_energy_density(om, pts, 6)
        runs[key] = (d, h.last_iteration_stats())
        split[key] = h.last_cocg_split()
        h.close()
    # the launch time is attributed to the kernels that ran
    assert split["plain"]["plain"] > 0 and split["plain"]["precond"] == 0
    assert split["all"]["plain"] == 0 and split["all"]["precond"] > 0
    assert split["window"]["plain"] > 0 and split["window"]["precond"] > 0
    d0, s0 = runs["plain"]
    d1, s1 = runs["all"]
    dw, sw = runs["window"]
    assert torch.equal(dw[0], d0[0]) and torch.equal(dw[1:], d1[1:])
    assert sw[0]["mean"] == s0[0]["mean"] and [s["mean"] for s in sw[1:]] == [s["mean"] for s in s1[1:]]
    assert all(s1[k]["mean"] < s0[k]["mean"] for k in range(3))
    ham, coul = O.Hamiltonian(c.n, c.L, c.v_loc), O.Coulomb(c.n, c.L)
    ref = O.energy_density(ham, coul, c.psi, c.eps, om, pts, 6, tol=1e-10)
    assert np.abs(dw.cpu().numpy() - ref).max() <= 1e-8
