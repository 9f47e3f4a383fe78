"""Write si8_fp64_nl30.txt: the oracle's energy density d_j(omega_k)
(Algorithm 1; Eqs. 6-8) on the Si8-like cell at the settings of its
plain FP64 workload -- N_l = 30 Lanczos steps, Sternheimer tolerance 1e-8 --
for a subset of the stride-2 coarse points at all 8 frequencies of the
mapped Gauss-Legendre rule (Eq. 9).

Calls only the oracle and the seeded cell builder.  The subset: every 6th
coarse point per axis (8 points) plus 8 coarse points drawn with seed 302.
Runs the (point, frequency) pairs over a process pool, one thread each.

Usage: python tests/golden/make_si8_fp64_nl30.py [workers]
"""
import concurrent.futures as cf
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "si8_fp64_nl30.txt")
N_L, TOL = 30, 1e-8

_W = {}


def _init():
    sys.path.insert(0, ROOT)
    from threadpoolctl import threadpool_limits
    _W["lim"] = threadpool_limits(limits=1)
    import oracle as O
    import synthcell as sc
    c = sc.preset("si8")
    _W.update(O=O, c=c, ham=O.Hamiltonian(c.n, c.L, c.v_loc), coul=O.Coulomb(c.n, c.L))


def _one(args):
    p, k, omega = args
    O, c = _W["O"], _W["c"]
    t = time.perf_counter()
    st = {}
    d = O.energy_density(_W["ham"], _W["coul"], c.psi, c.eps, [omega], [p], N_L, tol=TOL, stats=st)
    return p, k, omega, float(d[0, 0]), time.perf_counter() - t, float(sum(st["iters"])) / len(st["iters"])


def points():
    import synthcell as sc
    import numpy as np
    n = (24, 24, 24)
    sub = sc.sublattice_points(n, 2, 6)
    rnd = sc.random_coarse_points(n, 2, 8, seed=302)
    return np.array(sorted(set(sub.tolist()) | set(rnd.tolist())), dtype=np.int64)


def main():
    sys.path.insert(0, ROOT)
    os.environ["OMP_NUM_THREADS"] = "1"
    import oracle as O
    import synthcell as sc
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else max(1, (os.cpu_count() or 2) - 1)
    c = sc.preset("si8")
    om, _ = O.frequency_rule(8)
    pts = points()
    # slowest (smallest omega) first
    jobs = [(int(p), k, float(om[k])) for k in range(len(om)) for p in pts]
    rows = []
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(workers, initializer=_init) as ex:
        for r in ex.map(_one, jobs):
            rows.append(r)
            print(f"point {r[0]} omega {r[2]:.4g}: d = {r[3]:.12e} ({r[4]:.0f} s, "
                  f"{r[5]:.0f} COCG iterations per solve); {len(rows)}/{len(jobs)} "
                  f"after {time.perf_counter() - t0:.0f} s", flush=True)
    with open(OUT, "w") as f:
        f.write("# Oracle energy density d_j(omega_k) (Algorithm 1) on the Si8-like cell\n")
        f.write(f"# cell: synthcell preset si8 (24^3 grid, 16 orbitals, seed {c.seed})\n")
        f.write(f"# settings: N_l {N_L}, Sternheimer tol {TOL:g}, COCG from the Galerkin guess, "
                "breakdown 1e-13\n")
        f.write("# eps: " + " ".join(f"{e:.15e}" for e in c.eps) + "\n")
        f.write("# written by tests/golden/make_si8_fp64_nl30.py\n")
        f.write("# columns: point k omega d\n")
        for p, k, w, d, _, _ in sorted(rows, key=lambda r: (r[1], r[0])):
            f.write(f"{p} {k} {w:.17g} {d:.17e}\n")
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
