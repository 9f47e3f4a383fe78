"""Block Lanczos quadrature on the GPU (lanczos_energy_density_block)
against the oracle's block Gauss rule (oracle.energy_density_block: block
three-term recurrence, full reorthogonalisation, thin QR, diag of
E_1^T f(T) E_1), and block size 1 against the scalar path.

Tiny cell (12^3, 4 orbitals), FP64 at Sternheimer tol 1e-10, 7 points at
the 2-point frequency rule, so block 3 leaves a ragged group of 1 and block
4 one of 3.  Si8-like cell: accuracy per chi0 application of block and
scalar estimates against the stored N_l = 30 oracle values.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
import synthcell as sc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def P():
    import paper_2609_16408_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.lib()
    return P


@pytest.fixture(scope="module")
def tiny():
    return sc.preset("tiny")


@pytest.fixture(scope="module")
def tiny_ops(tiny):
    return O.Hamiltonian(tiny.n, tiny.L, tiny.v_loc), O.Coulomb(tiny.n, tiny.L)


def _pts(c):
    return sc.coarse_points(c.n, 3)[[0, 5, 9, 17, 22, 40, 63]]


@pytest.mark.parametrize("block", [1, 3, 4])
def test_block_lanczos_matches_oracle(P, tiny, tiny_ops, block):
    """GPU block estimates within 1e-8 of the oracle's at identical settings
    (FP64, tol 1e-10, 4 block steps), ragged last group included; every
    estimate <= 0."""
    ham, coul = tiny_ops
    om, _ = O.frequency_rule(2)
    pts = _pts(tiny)
    ref = O.energy_density_block(ham, coul, tiny.psi, tiny.eps, om, pts, 4, block, tol=1e-10)
    h = P.handle_for_cell(tiny, precision="fp64", stern_tol=1e-10, batch=8)
    d, st = h.lanczos_energy_density_block(om, pts, 4, block)
    h.close()
    d = d.cpu().numpy()
    err = np.abs(d - ref).max()
    print(f"block {block}: max |d - d_oracle| = {err:.2e}", flush=True)
    assert st["n_noconv"] == 0
    assert np.all(d <= 0)
    assert err <= 1e-8, err


def test_block_one_equals_scalar_path(P, tiny):
    """Block size 1 is the scalar Lanczos quadrature: same values as
    lanczos_energy_density up to the order of the reductions (their
    rounding can move a COCG stop by an iteration, a change of order
    tol |d| = 2e-12 here)."""
    om, _ = O.frequency_rule(2)
    pts = _pts(tiny)
    h = P.handle_for_cell(tiny, precision="fp64", stern_tol=1e-10, batch=8)
    d1, _ = h.lanczos_energy_density_block(om, pts, 6, 1)
    ds, _ = h.lanczos_energy_density(om, pts, 6)
    h.close()
    err = (d1 - ds).abs().max().item()
    assert err <= 1e-10, err


def test_block_lanczos_batches_and_groups_are_independent(P, tiny):
    """A group's estimates do not depend on which other groups share its
    batch: a batch of 8 columns (two groups of 4, one of 3 per frequency
    split over batches) gives the same values as batches of one group."""
    om, _ = O.frequency_rule(2)
    pts = _pts(tiny)
    out = []
    for batch in (4, 8):
        h = P.handle_for_cell(tiny, precision="fp64", stern_tol=1e-10, batch=batch)
        d, _ = h.lanczos_energy_density_block(om, pts, 4, 4)
        h.close()
        out.append(d.cpu().numpy())
    assert np.abs(out[0] - out[1]).max() <= 1e-13


def test_block_lanczos_rejects_bad_sizes(P, tiny):
    h = P.handle_for_cell(tiny, precision="fp64", stern_tol=1e-10, batch=8)
    om, _ = O.frequency_rule(2)
    with pytest.raises(P.RPAError):
        h.lanczos_energy_density_block(om, _pts(tiny), 4, 9)
    with pytest.raises(P.RPAError):
        h.lanczos_energy_density_block(om, _pts(tiny), 9, 8)
    h.close()


def _read_golden(path):
    meta, rows = {}, []
    for line in open(path):
        line = line.strip()
        if not line:
            continue
        if line.startswith("#"):
            if ":" in line:
                k, v = line[1:].split(":", 1)
                meta[k.strip()] = v.strip()
            continue
        p, k, om, d = line.split()
        rows.append((int(p), int(k), float(om), float(d)))
    return meta, rows


def test_si8_block_accuracy_per_chi0_application(P):
    """Si8-like cell, FP64, tol 1e-8, at the smallest and a mid frequency:
    with m chi0 applications per point (m scalar steps, or m block steps
    for a group of 4), the block estimates are at least as close to the
    converged N_l = 30 oracle values (stored) as the scalar ones on average,
    and both approach them as m grows."""
    meta, rows = _read_golden(os.path.join(GOLDEN, "si8_fp64_nl30.txt"))
    c = sc.preset("si8")
    pts = np.array(sorted({p for p, _, _, _ in rows}), dtype=np.int64)[:8]
    ks = [0, 5]
    om_all = np.array(sorted({(k, o) for _, k, o, _ in rows}))[:, 1]
    om = om_all[ks]
    ref = np.zeros((len(ks), len(pts)))
    col = {int(p): i for i, p in enumerate(pts)}
    for p, k, _, v in rows:
        if k in ks and int(p) in col:
            ref[ks.index(k), col[int(p)]] = v
    h = P.handle_for_cell(c, precision="fp64", stern_tol=1e-8, batch=32)
    errs = {}
    for m in (2, 4):
        ds, _ = h.lanczos_energy_density(om, pts, m)
        db, _ = h.lanczos_energy_density_block(om, pts, m, 4)
        errs[m] = (np.abs(ds.cpu().numpy() - ref).mean(), np.abs(db.cpu().numpy() - ref).mean())
        print(f"si8 m={m}: mean |d - d_30| scalar {errs[m][0]:.3e}, block-4 {errs[m][1]:.3e}",
              flush=True)
    h.close()
    for m in (2, 4):
        assert errs[m][1] <= errs[m][0] * 1.05
    assert errs[4][0] < errs[2][0] and errs[4][1] < errs[2][1]


def _block_ratio_sequences(ham, coul, c, om, pts, block, m):
    """Per (frequency, group): min |diag B_k| / max |A_0..A_k entries| of the
    oracle's untruncated block Lanczos (the quantity its breakdown test
    compares), for k < m - 1."""
    seqs = []
    for w in om:
        A = O.nuhalf_chi0_nuhalf(ham, coul, c.psi, c.eps, w, tol=1e-10)
        ap = lambda X, A=A: np.stack([A(X[:, i]) for i in range(X.shape[1])], axis=1)
        for g0 in range(0, len(pts), block):
            grp = pts[g0:g0 + block]
            Q1 = np.zeros((c.N_d, len(grp)))
            Q1[grp, np.arange(len(grp))] = 1.0
            Ab, Bb, _ = O.block_lanczos(ap, Q1, m, breakdown_rel=0.0)
            amax, r = 0.0, []
            for k, Bk in enumerate(Bb):
                amax = max(amax, float(np.abs(Ab[k]).max()))
                r.append(float(np.abs(np.diag(Bk)).min()) / amax)
            seqs.append(np.array(r))
    return seqs


def test_block_lanczos_breakdown_truncates_like_the_oracle(P, tiny, tiny_ops):
    """Block Lanczos truncation (reading R18) forced from the host: the
    threshold sits at the geometric middle of the widest gap (at least 2x)
    of the oracle's ratio sequences that truncates some groups but not all,
    so both sides stop the same groups at the same step (their ratios agree
    to ~1e-9).  The truncated estimates equal the oracle's, differ from the
    untruncated ones, and the call warns."""
    ham, coul = tiny_ops
    om, m, block = np.array([0.0203, 0.69]), 8, 3
    pts = np.array([0, 100, 777, 1500, 1001, 333])
    seqs = _block_ratio_sequences(ham, coul, tiny, om, pts, block, m)
    allr = np.sort(np.concatenate(seqs))
    best, thr = 0.0, None
    for lo, hi in zip(allr[:-1], allr[1:]):
        t = math.sqrt(lo * hi)
        cut = [bool(np.any(r <= t)) for r in seqs]
        if any(cut) and not all(cut) and hi / lo > best:
            best, thr = hi / lo, t
    assert thr is not None and best > 2.0, (best, seqs)
    n_cut = sum(bool(np.any(r <= thr)) for r in seqs)
    h = P.handle_for_cell(tiny, precision="fp64", stern_tol=1e-10, batch=8, lanczos_breakdown=thr)
    with pytest.warns(P.RPAWarning):
        d, st = h.lanczos_energy_density_block(om, pts, m, block)
    h.close()
    assert st["n_breakdown"] == n_cut
    ref = np.zeros((len(om), len(pts)))
    full = np.zeros_like(ref)
    for k, w in enumerate(om):
        A = O.nuhalf_chi0_nuhalf(ham, coul, tiny.psi, tiny.eps, w, tol=1e-10)
        ap = lambda X, A=A: np.stack([A(X[:, i]) for i in range(X.shape[1])], axis=1)
        for g0 in range(0, len(pts), block):
            grp = pts[g0:g0 + block]
            Q1 = np.zeros((tiny.N_d, len(grp)))
            Q1[grp, np.arange(len(grp))] = 1.0
            Ab, Bb, broke = O.block_lanczos(ap, Q1, m, breakdown_rel=thr)
            ref[k, g0:g0 + len(grp)] = O.block_quadrature(Ab, Bb)
            Ab, Bb, _ = O.block_lanczos(ap, Q1, m, breakdown_rel=0.0)
            full[k, g0:g0 + len(grp)] = O.block_quadrature(Ab, Bb)
    d = d.cpu().numpy()
    err = np.abs(d - ref).max()
    print(f"block breakdown: threshold {thr:.2e} (gap x{best:.1f}), {n_cut} of {len(seqs)} groups "
          f"truncated, max |d - d_oracle| = {err:.2e}", flush=True)
    assert err <= 1e-9, err
    assert np.abs(ref - full).max() > 1e-12
