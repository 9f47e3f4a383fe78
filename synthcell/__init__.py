"""Seeded synthetic Si-like cells: the inputs of the RPA hot path.

This module produces the *problem data* that the RPA method consumes -- the
Kohn-Sham eigenpairs (psi_n, eps_n) of a finite-difference Hamiltonian
H = -1/2 Lap_h + V_loc (+ V_nl) on a periodic orthorhombic grid (the paper's
Eq. 3 takes them as given) -- plus seeded point lists.  It holds none of the
RPA method's arithmetic (no Coulomb operator, no Sternheimer solve, no
Lanczos, no quadrature, no interpolation).  Both the CPU oracle and the HIP
path consume exactly the arrays produced here, so parity is a statement about
the RPA path and not about two eigensolvers.

Cell recipe (stand-in for the paper's Si systems, section "Chemical Systems"):
  * diamond sites, 8 per cubic cell of side a = 10.26 bohr, replicated
    (cx, cy, cz) times, each coordinate jittered by U(-0.05, 0.05) bohr
    drawn from numpy's PCG64 with the cell seed, in site order
    (cell-major, basis-minor);
  * V_loc(r) = sum over atoms and all periodic images of
    depth * exp(-|r - R|^2 / (2 sigma^2)), depth = -2.0 Ha, sigma = 1.0 bohr;
  * grid points r = (ix h_x, iy h_y, iz h_z), flat index (ix*ny + iy)*nz + iz;
  * optional separable nonlocal projectors (4 per atom: s, px, py, pz angular
    parts times a Gaussian radial of width 1.0 bohr, truncated at 3 bohr,
    normalised h^3 sum chi^2 = 1, coefficients gamma ~ U(0.5, 2) Ha).

Orbitals come from a Chebyshev-filtered subspace iteration whose kinetic
operator is the 12th-order central-difference Laplacian applied through its
exact Fourier symbol (the FD operator is circulant on a periodic grid).  The
returned orbitals are normalised so that h^3 * sum(psi^2) = 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

A_SI = 10.26          # cubic cell side (bohr)
DEPTH = -2.0          # Gaussian well depth (Ha)
SIGMA = 1.0           # Gaussian well width (bohr), standard deviation
JITTER = 0.05         # uniform jitter amplitude (bohr)
FD_RADIUS = 6         # 12th-order central differences

_DIAMOND_BASIS = np.array([
    [0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25],
])


@dataclass
class Cell:
    """A periodic orthorhombic cell with its grid, potential and orbitals."""
    name: str
    n: tuple            # (nx, ny, nz)
    L: tuple            # (Lx, Ly, Lz) bohr
    atoms: np.ndarray   # (N_atoms, 3) bohr
    v_loc: np.ndarray   # (N_d,) float64, Ha
    n_occ: int
    seed: int
    psi: np.ndarray = None      # (n_occ, N_d) float64, h^3 sum psi^2 = 1
    eps: np.ndarray = None      # (n_occ,) float64 ascending
    eps_buffer: np.ndarray = None  # Ritz values of the buffer states above n_occ
    psi_extra: np.ndarray = None   # converged eigenvectors just above n_occ (ks_orbitals n_extra)
    eps_extra: np.ndarray = None
    gap: float = float("nan")   # eps_{n_occ+1} - eps_{n_occ}
    eig_residual: float = float("nan")
    proj: dict = None           # nonlocal projectors (CSR), optional
    extra: dict = field(default_factory=dict)

    @property
    def N_d(self) -> int:
        return int(np.prod(self.n))

    @property
    def h(self) -> tuple:
        return tuple(self.L[d] / self.n[d] for d in range(3))

    @property
    def dV(self) -> float:
        hx, hy, hz = self.h
        return hx * hy * hz

    @property
    def n_atoms(self) -> int:
        return int(self.atoms.shape[0])


def diamond_atoms(cells=(1, 1, 1), a=A_SI, seed=None, jitter=JITTER) -> np.ndarray:
    """Diamond sites of a (cx, cy, cz) supercell, optionally jittered (seeded)."""
    cx, cy, cz = cells
    pos = []
    for i in range(cx):
        for j in range(cy):
            for k in range(cz):
                for b in _DIAMOND_BASIS:
                    pos.append((np.array([i, j, k], dtype=float) + b) * a)
    pos = np.array(pos)
    if seed is not None and jitter > 0:
        rng = np.random.default_rng(seed)
        pos = pos + rng.uniform(-jitter, jitter, size=pos.shape)
    return pos


def _periodic_gauss_1d(coords: np.ndarray, center: float, length: float, sigma: float) -> np.ndarray:
    """sum_m exp(-(x - X - m L)^2 / (2 sigma^2)) over all images that matter."""
    reach = 10.0 * sigma                 # exp(-50) ~ 2e-22: negligible beyond
    mmax = int(math.ceil((reach + length) / length))
    out = np.zeros_like(coords)
    for m in range(-mmax, mmax + 1):
        d = coords - center - m * length
        out += np.exp(-(d * d) / (2.0 * sigma * sigma))
    return out


def gaussian_vloc(n, L, atoms, depth=DEPTH, sigma=SIGMA) -> np.ndarray:
    """Sum of periodic Gaussian wells sampled on the grid, flat (N_d,)."""
    grids = [np.arange(n[d]) * (L[d] / n[d]) for d in range(3)]
    v = np.zeros(tuple(n))
    for R in atoms:
        gx = _periodic_gauss_1d(grids[0], R[0], L[0], sigma)
        gy = _periodic_gauss_1d(grids[1], R[1], L[1], sigma)
        gz = _periodic_gauss_1d(grids[2], R[2], L[2], sigma)
        v += np.einsum("i,j,k->ijk", gx, gy, gz)
    return (depth * v).reshape(-1)


# ----------------------------------------------------------------------------
# Kinetic operator for the ground-state eigensolve (problem setup only)
# ----------------------------------------------------------------------------

def _central_d2_weights(radius: int) -> list:
    """Central second-derivative weights w_0..w_R on a unit-spacing grid.

    Solved here from the moment conditions of the symmetric stencil (a small
    Vandermonde system in exact rationals), i.e. independently of any closed
    form used elsewhere.
    """
    from fractions import Fraction
    R = radius
    # unknowns w_1..w_R; conditions sum_k w_k * 2 * k^(2j) = (2j)! * [j == 1], j=1..R
    A = [[Fraction(2 * k ** (2 * j)) for k in range(1, R + 1)] for j in range(1, R + 1)]
    rhs = [Fraction(2) if j == 1 else Fraction(0) for j in range(1, R + 1)]
    # Gaussian elimination in rationals
    m = [row[:] + [rhs[i]] for i, row in enumerate(A)]
    for c in range(R):
        piv = next(r for r in range(c, R) if m[r][c] != 0)
        m[c], m[piv] = m[piv], m[c]
        for r in range(R):
            if r != c and m[r][c] != 0:
                f = m[r][c] / m[c][c]
                m[r] = [a - f * b for a, b in zip(m[r], m[c])]
    w = [m[i][R] / m[i][i] for i in range(R)]
    w0 = -2 * sum(w)
    return [w0] + w


def kinetic_symbol(n, L, radius=FD_RADIUS) -> np.ndarray:
    """Eigenvalues of -1/2 Lap_h on the periodic grid, indexed like fftn output."""
    w = [float(x) for x in _central_d2_weights(radius)]
    sym = np.zeros(tuple(n))
    for d in range(3):
        h = L[d] / n[d]
        theta = 2.0 * np.pi * np.arange(n[d]) / n[d]
        lam = w[0] + 2.0 * sum(w[k] * np.cos(k * theta) for k in range(1, radius + 1))
        shape = [1, 1, 1]
        shape[d] = n[d]
        sym = sym + (-0.5 * lam / (h * h)).reshape(shape)
    return sym


def projector_balls(n, L, atoms, seed, n_proj=4, rc=3.0, width=1.0):
    """Separable nonlocal projectors on atom-centred balls (CSR form).

    Returns dict with 'ptr' (n_atoms*n_proj+1,), 'idx' (nnz,) int64 grid
    indices, 'val' (nnz,) float64 projector values (h^3 sum val^2 = 1 per
    projector), 'gamma' (n_atoms*n_proj,) Ha.
    """
    h = [L[d] / n[d] for d in range(3)]
    dV = h[0] * h[1] * h[2]
    rng = np.random.default_rng(seed)
    gamma = rng.uniform(0.5, 2.0, size=atoms.shape[0] * n_proj)
    ptr, idx, val = [0], [], []
    reach = [int(math.ceil(rc / h[d])) for d in range(3)]
    for R in atoms:
        c = [int(round(R[d] / h[d])) for d in range(3)]
        offs = [np.arange(c[d] - reach[d], c[d] + reach[d] + 1) for d in range(3)]
        gx, gy, gz = np.meshgrid(*offs, indexing="ij")
        dx = gx * h[0] - R[0]
        dy = gy * h[1] - R[1]
        dz = gz * h[2] - R[2]
        r2 = dx * dx + dy * dy + dz * dz
        inside = r2 <= rc * rc
        gidx = ((np.mod(gx, n[0]) * n[1] + np.mod(gy, n[1])) * n[2] + np.mod(gz, n[2]))[inside]
        radial = np.exp(-r2[inside] / (2.0 * width * width))
        ang = [np.ones_like(radial), dx[inside], dy[inside], dz[inside]]
        order = np.argsort(gidx)
        gidx = gidx[order]
        for a in ang[:n_proj]:
            chi = (a * radial)[order]
            chi = chi / math.sqrt(dV * float(np.sum(chi * chi)))
            idx.append(gidx.astype(np.int64))
            val.append(chi)
            ptr.append(ptr[-1] + gidx.size)
    return {"ptr": np.array(ptr, dtype=np.int64), "idx": np.concatenate(idx),
            "val": np.concatenate(val), "gamma": gamma, "n_proj": n_proj}


def _make_apply_h(cell: Cell, torch, device):
    """Returns a function X[k, N_d] -> H X[k, N_d] (torch, float64)."""
    n = cell.n
    sym = torch.as_tensor(kinetic_symbol(n, cell.L), device=device)
    v = torch.as_tensor(cell.v_loc, device=device)
    proj = cell.proj
    if proj is not None:
        P = _dense_projector_matrix(cell, torch, device)   # (n_p, N_d) sparse-ish dense by atom
        gamma = torch.as_tensor(proj["gamma"], device=device)
        dV = cell.dV
    else:
        P = None

    def apply_h(X):
        k = X.shape[0]
        Y = torch.fft.ifftn(torch.fft.fftn(X.reshape(k, *n), dim=(1, 2, 3)) * sym,
                            dim=(1, 2, 3)).real.reshape(k, -1)
        Y = Y + v * X
        if P is not None:
            c = (X @ P.T) * (dV * gamma)        # (k, n_p)
            Y = Y + c @ P
        return Y
    return apply_h


def _dense_projector_matrix(cell, torch, device):
    proj = cell.proj
    n_p = proj["ptr"].size - 1
    P = torch.zeros((n_p, cell.N_d), dtype=torch.float64, device=device)
    ptr = proj["ptr"]
    rows = np.repeat(np.arange(n_p), np.diff(ptr))
    P[torch.as_tensor(rows, device=device), torch.as_tensor(proj["idx"], device=device)] = \
        torch.as_tensor(proj["val"], device=device)
    return P


def ks_orbitals(cell: Cell, n_buffer=None, tol=1e-10, degree=24, max_iter=600,
                device=None, seed=0, verbose=False, n_extra=0):
    """Lowest n_occ eigenpairs of H by Chebyshev-filtered subspace iteration.

    Fills cell.psi (h^3-normalised), cell.eps, cell.gap, cell.eig_residual
    (max Euclidean residual ||H x - e x|| of unit-norm x over occupied states).
    With n_extra > 0 the next n_extra eigenpairs are converged too and kept
    as cell.psi_extra / cell.eps_extra (the residual then covers them).
    """
    import torch
    if device is None:
        device = "cpu"
    nocc = cell.n_occ
    if n_buffer is None:
        n_buffer = max(16, int(math.ceil(0.1 * nocc)))
    if n_extra > 0:
        n_buffer = max(n_buffer, n_extra + 16)
    nconv = nocc + n_extra
    k = nocc + n_buffer
    N = cell.N_d
    apply_h = _make_apply_h(cell, torch, device)
    sym_max = float(np.max(kinetic_symbol(cell.n, cell.L)))
    vmax = float(np.max(cell.v_loc))
    nl_max = 0.0
    if cell.proj is not None:
        nl_max = float(np.max(cell.proj["gamma"]))
    upper = sym_max + max(vmax, 0.0) + nl_max + 1e-3

    gen = torch.Generator(device="cpu").manual_seed(seed)
    X = torch.randn((k, N), generator=gen, dtype=torch.float64).to(device)

    def orth(X):
        Q, _ = torch.linalg.qr(X.T)
        return Q.T.contiguous()

    def rayleigh_ritz(X):
        HX = apply_h(X)
        Hs = X @ HX.T
        Hs = 0.5 * (Hs + Hs.T)
        ev, Qs = torch.linalg.eigh(Hs.cpu())
        Qs = Qs.to(device)
        X = Qs.T @ X
        HX = Qs.T @ HX
        return X, HX, ev.to(device)

    X = orth(X)
    X, HX, ev = rayleigh_ritz(X)
    if verbose and verbose >= 2:
        print(f"  chefsi: {k} states on {N} points, initial subspace ready", flush=True)
    res = float("inf")
    for it in range(max_iter):
        a = float(ev[-1])          # filter out everything above the top Ritz value
        a0 = float(ev[0])
        b = upper
        e = 0.5 * (b - a)
        c = 0.5 * (b + a)
        sigma = e / (a0 - c)
        sigma1 = sigma
        Y = (apply_h(X) - c * X) * (sigma1 / e)
        Xp = X
        for _ in range(2, degree + 1):
            sigma2 = 1.0 / (2.0 / sigma1 - sigma)
            Ynew = (apply_h(Y) - c * Y) * (2.0 * sigma2 / e) - (sigma * sigma2) * Xp
            Xp, Y = Y, Ynew
            sigma = sigma2
        X = orth(Y)
        X, HX, ev = rayleigh_ritz(X)
        R = HX[:nconv] - ev[:nconv, None] * X[:nconv]
        res = float(torch.max(torch.linalg.norm(R, dim=1)))
        if verbose and (it % 10 == 0 or verbose >= 2):
            print(f"  chefsi it {it}: max residual {res:.3e}", flush=True)
        if res <= tol:
            break
    ev_np = ev.cpu().numpy()
    psi = (X[:nocc].cpu().numpy()) / math.sqrt(cell.dV)
    # deterministic sign: largest-magnitude entry positive
    for i in range(nocc):
        j = int(np.argmax(np.abs(psi[i])))
        if psi[i, j] < 0:
            psi[i] = -psi[i]
    cell.psi = np.ascontiguousarray(psi)
    cell.eps = ev_np[:nocc].copy()
    if n_extra > 0:
        px = (X[nocc:nconv].cpu().numpy()) / math.sqrt(cell.dV)
        for i in range(n_extra):
            j = int(np.argmax(np.abs(px[i])))
            if px[i, j] < 0:
                px[i] = -px[i]
        cell.psi_extra = np.ascontiguousarray(px)
        cell.eps_extra = ev_np[nocc:nconv].copy()
    cell.eps_buffer = ev_np[nocc:].copy()
    cell.gap = float(ev_np[nocc] - ev_np[nocc - 1])
    cell.eig_residual = res
    return cell


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def make_cell(name: str, cells=(1, 1, 1), n=(12, 12, 12), n_occ=4, seed=101,
              with_projectors=False, proj_seed=None, a=A_SI, jitter=JITTER) -> Cell:
    atoms = diamond_atoms(cells, a=a, seed=seed, jitter=jitter)
    L = tuple(float(cells[d] * a) for d in range(3))
    v = gaussian_vloc(n, L, atoms)
    cell = Cell(name=name, n=tuple(int(x) for x in n), L=L, atoms=atoms, v_loc=v,
                n_occ=int(n_occ), seed=int(seed))
    if with_projectors:
        cell.proj = projector_balls(n, L, atoms, seed=proj_seed)
    return cell


# name -> (supercell, grid, n_occ, cell seed)
PRESETS = {
    "tiny":  dict(cells=(1, 1, 1), n=(12, 12, 12), n_occ=4, seed=101),
    "si8":   dict(cells=(1, 1, 1), n=(24, 24, 24), n_occ=16, seed=102),
    "si64":  dict(cells=(2, 2, 2), n=(48, 48, 48), n_occ=128, seed=103),
    "si16":  dict(cells=(1, 1, 2), n=(24, 24, 48), n_occ=32, seed=411),
    "si216": dict(cells=(3, 3, 3), n=(72, 72, 72), n_occ=432, seed=105,
                  with_projectors=True, proj_seed=205),
}


def preset(name: str, orbitals=True, device=None, verbose=False, n_extra=0, **overrides) -> Cell:
    cfg = dict(PRESETS[name])
    cfg.update(overrides)
    cell = make_cell(name, **cfg)
    if orbitals:
        ks_orbitals(cell, device=device, verbose=verbose, n_extra=n_extra)
    return cell


def coarse_points(n, stride) -> np.ndarray:
    """Flat indices of the origin-aligned stride-g sublattice, x-major order."""
    nx, ny, nz = n
    if nx % stride or ny % stride or nz % stride:
        raise ValueError("stride must divide every grid dimension")
    ix = np.arange(0, nx, stride)
    iy = np.arange(0, ny, stride)
    iz = np.arange(0, nz, stride)
    gx, gy, gz = np.meshgrid(ix, iy, iz, indexing="ij")
    return ((gx * ny + gy) * nz + gz).reshape(-1).astype(np.int64)


def sublattice_points(n, stride, every) -> np.ndarray:
    """Every `every`-th coarse point per axis (a regular subset of the coarse set)."""
    return coarse_points(n, stride * every)


def random_coarse_points(n, stride, count, seed) -> np.ndarray:
    pts = coarse_points(n, stride)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(pts, size=count, replace=False)).astype(np.int64)


def random_field(shape, seed, dtype=np.float64) -> np.ndarray:
    """Seeded standard-normal test field."""
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)
