"""Interpolation-accuracy sweep over the coarse-grid spacing g (section
"Interpolating Diagonal Entries" and the error metrics of the paper).

The reference is the directly computed diagonal on every grid point (g = 1).
For each stride g dividing the grid and each interpolant, the coarse values
(taken from the reference on the origin-aligned stride-g sublattice) are
interpolated and frequency-integrated by the library (rpa_energy_from_coarse),
and compared per atom with the reference:

    dE  = |E_c - E_c^(g)| / N_atoms
    L1  = sum_j |c_j - c_j^(g)| / N_atoms,  c_j = (1/2pi) sum_k w_k d_j(omega_k)
    ECR = dE / L1   (error cancellation ratio, <= 1)

Usage: python -m paper_2609_16408_amd.gsweep [--cell tiny] [--n-lanczos 8]
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

from . import Handle, frequency_rule

KINDS = ("trilinear", "tricubic", "fourier")


def sublattice(n, g) -> np.ndarray:
    """Flat indices (x-major) of the points whose three indices are multiples of g."""
    ix, iy, iz = (np.arange(0, n[d], g) for d in range(3))
    gx, gy, gz = np.meshgrid(ix, iy, iz, indexing="ij")
    return ((gx * n[1] + gy) * n[2] + gz).reshape(-1).astype(np.int64)


def g_sweep(h: Handle, n_atoms: int, dV: float, n_omega=8, n_lanczos=8, strides=(2, 3, 4, 6),
            kinds=KINDS, chunk=2048, log=None):
    """Returns (reference dict, list of row dicts, reference d [n_omega][N] on the host).
    The reference is computed `chunk` points per call; `log` (optional)
    receives a line per finished chunk."""
    import torch
    n = h.n
    omega, weight = frequency_rule(n_omega)
    d_host = np.zeros((n_omega, h.N))
    st = {"cocg_iters_total": 0, "n_systems": 0}
    for p0 in range(0, h.N, chunk):
        pts = np.arange(p0, min(h.N, p0 + chunk), dtype=np.int64)
        d, s = h.lanczos_energy_density(omega, pts, n_lanczos)
        d_host[:, pts] = d.cpu().numpy()
        st["cocg_iters_total"] += s["cocg_iters_total"]
        st["n_systems"] += s["n_systems"]
        if log:
            log(f"reference points {pts[-1] + 1}/{h.N}: {s['seconds']:.1f} s")
    c_direct = weight @ d_host / (2.0 * math.pi)
    e_direct = float(c_direct.sum())
    ref = {"E_c_per_atom": e_direct / n_atoms, "points": int(h.N), "n_omega": n_omega,
           "n_lanczos": n_lanczos, "cocg_iters_per_system": st["cocg_iters_total"] / st["n_systems"]}
    rows = []
    for g in strides:
        if any(n[d] % g for d in range(3)):
            continue
        idx = sublattice(n, g)
        dc = torch.from_numpy(np.ascontiguousarray(d_host[:, idx])).cuda()
        for kind in kinds:
            e_g, e_fine = h.energy_from_coarse(weight, g, kind, dc, want_fine=True)
            c_hat = e_fine.cpu().numpy() * dV
            delta = c_direct - c_hat
            de = abs(e_direct - e_g) / n_atoms
            l1 = float(np.abs(delta).sum()) / n_atoms
            rows.append({"g": g, "kind": kind, "coarse_points": int(idx.size),
                         "E_c_per_atom": e_g / n_atoms, "dE_per_atom": de, "L1_per_atom": l1,
                         "ECR": de / l1 if l1 > 0 else 0.0})
    return ref, rows, d_host


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cell", default="tiny", help="synthetic cell preset")
    ap.add_argument("--n-lanczos", type=int, default=8)
    ap.add_argument("--n-omega", type=int, default=8)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_refine"])
    args = ap.parse_args()
    import synthcell as sc
    c = sc.preset(args.cell, device="cuda")
    h = Handle(c.n, c.L, c.v_loc, c.psi, c.eps, precision=args.precision, stern_tol=args.tol,
               proj=c.proj)
    ref, rows, _ = g_sweep(h, c.n_atoms, c.dV, args.n_omega, args.n_lanczos,
                           log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps({"reference": ref, "cell": args.cell}))
    for r in rows:
        print(json.dumps(r))
    h.close()


if __name__ == "__main__":
    main()
