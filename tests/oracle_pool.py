"""The CPU oracle spread over the host's cores, for the parity tests at full
cell size (test infrastructure; nothing in the product imports it).

One worker process per core (at most 16), each single-threaded, started with
the 'spawn' method so that no worker inherits the parent's HIP state; the
cell's arrays reach the workers as memory-mapped .npy files.  The work is
split the way Algorithm 1 allows: the Sternheimer solves of one chi0
application are independent per occupied orbital, so each worker takes a
slice of the orbitals and the partial accumulations are summed.
"""
from __future__ import annotations

import concurrent.futures as cf
import multiprocessing as mp
import os
import shutil
import sys
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_W = {}


def _init(root, spec):
    if root not in sys.path:
        sys.path.insert(0, root)
    from threadpoolctl import threadpool_limits
    _W["limits"] = threadpool_limits(limits=1)
    import oracle as O
    v = np.load(spec["v"], mmap_mode="r")
    _W["psi"] = np.load(spec["psi"], mmap_mode="r")
    _W["eps"] = np.load(spec["eps"])
    _W["ham"] = O.Hamiltonian(spec["n"], spec["L"], np.asarray(v), proj=spec["proj"])
    _W["O"] = O


def _chi0_part(u, omega, tol, orbitals):
    O = _W["O"]
    st = {}
    r = O.chi0_apply(_W["ham"], _W["psi"], _W["eps"], u, omega, tol=tol, orbitals=orbitals, stats=st)
    return r, st.get("iters", [])


def _check_solves(x_paths, v, u, omega, tol, orbitals):
    """For each orbital n of the slice: the oracle's solution x* (COCG at
    `tol` from the Galerkin guess), its true residual, and for every set of
    GPU solutions X[v, n] given by path its true residual and distance to x*.
    Also the slice's part of chi0 u = 4 sum_n psi_n Re x*_n."""
    O = _W["O"]
    ham, psi, eps = _W["ham"], _W["psi"], _W["eps"]
    Xs = {k: np.load(p, mmap_mode="r") for k, p in x_paths.items()}
    out = {k: [] for k in Xs}
    acc = np.zeros(ham.N)
    for n in orbitals:
        b = -psi[n] * u
        z = eps[n] + 1j * omega
        apply_A = lambda y, z=z: ham.apply(y) - z * y
        x0 = O.galerkin_guess(psi, eps, n, b, omega, ham.dV)
        xo, its, status = O.cocg(apply_A, b, x0, tol, 20000)
        acc += 4.0 * psi[n] * xo.real
        r_or = float(np.linalg.norm(b - apply_A(xo)))
        for k, X in Xs.items():
            xg = np.asarray(X[v, n])
            out[k].append({
                "n": int(n),
                "b": float(np.linalg.norm(b)),
                "r_gpu": float(np.linalg.norm(b - apply_A(xg))),
                "r_oracle": r_or,
                "d2": float(np.linalg.norm(xg - xo)),
                "status": status,
                "iters": int(its),
            })
    return out, acc


class OraclePool:
    """Context manager around a process pool holding one cell."""

    def __init__(self, cell, workers=None):
        self.cell = cell
        self.workers = int(workers or min(16, os.cpu_count() or 1))
        self.dir = None
        self.ex = None

    def __enter__(self):
        c = self.cell
        self.dir = tempfile.mkdtemp(prefix="oracle_pool_")
        spec = {"n": tuple(c.n), "L": tuple(c.L), "proj": c.proj}
        for k, a in (("v", c.v_loc), ("psi", c.psi), ("eps", c.eps)):
            spec[k] = os.path.join(self.dir, k + ".npy")
            np.save(spec[k], np.ascontiguousarray(a, dtype=np.float64))
        saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
        for k in saved:
            os.environ[k] = "1"
        try:
            self.ex = cf.ProcessPoolExecutor(self.workers, mp_context=mp.get_context("spawn"),
                                             initializer=_init, initargs=(ROOT, spec))
            # start every worker now (fail early, and keep later timings honest)
            list(self.ex.map(abs, range(self.workers)))
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        return self

    def __exit__(self, *exc):
        if self.ex is not None:
            self.ex.shutdown(wait=True, cancel_futures=True)
        if self.dir:
            shutil.rmtree(self.dir, ignore_errors=True)

    def _slices(self):
        # orbitals dealt round-robin: neighbouring orbitals cost alike
        n = self.cell.n_occ
        return [list(range(w, n, self.workers)) for w in range(min(self.workers, n))]

    def chi0(self, u, omega, tol):
        """oracle.chi0_apply(u) summed over the orbital slices; also the
        per-solve iteration counts."""
        futs = [self.ex.submit(_chi0_part, np.asarray(u, dtype=np.float64), float(omega), tol, sl)
                for sl in self._slices()]
        r = np.zeros(self.cell.N_d)
        its = []
        for f in futs:
            part, it = f.result()
            r += part
            its += it
        return r, its

    def check_solves(self, xs, u, omega, tol, v=0):
        """Per-orbital residual / distance records of GPU solution sets
        xs = {name: complex [nvec, n_occ, N]} (start vector v) against the
        oracle's COCG at `tol`; returns ({name: records by n}, oracle chi0 u)."""
        paths = {}
        for k, x in xs.items():
            paths[k] = os.path.join(self.dir, f"x_{k}.npy")
            np.save(paths[k], np.ascontiguousarray(x))
        futs = [self.ex.submit(_check_solves, paths, v, np.asarray(u, dtype=np.float64), float(omega),
                               tol, sl) for sl in self._slices()]
        out = {k: [] for k in xs}
        y = np.zeros(self.cell.N_d)
        for f in futs:
            part, acc = f.result()
            for k in part:
                out[k] += part[k]
            y += acc
        for k in out:
            out[k].sort(key=lambda d: d["n"])
        return out, y

    def energy_density(self, coul, point, omega, n_lanczos, tol, breakdown_rel=1e-13):
        """Algorithm 1 for one point and frequency with the oracle's Lanczos
        recurrence (lanczos_tridiag) and quadrature; each chi0 application is
        spread over the pool."""
        import oracle as O
        def apply(q):
            r, _ = self.chi0(coul.half(q), omega, tol)
            return coul.half(r)
        q1 = np.zeros(self.cell.N_d)
        q1[int(point)] = 1.0
        a, b, _ = O.lanczos_tridiag(apply, q1, n_lanczos, breakdown_rel=breakdown_rel)
        return O.tridiag_quadrature(a, b)
