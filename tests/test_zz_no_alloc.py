"""The allocation-free chi0 entry point (chi0_apply_noalloc) against
chi0_apply on the same handles, two calls in a row with the second on a
smaller input (the shared scratch array keeps the first call's contents),
and its refusal of a problem that does not fit the array."""
import numpy as np
import pytest

import synthcell as sc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2609_16408_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.lib()
    return P


def test_noalloc_chi0_matches_chi0_apply_twice_in_a_row(P):
    big = sc.preset("si8")
    small = sc.preset("tiny")
    h1 = P.handle_for_cell(big, precision="fp32_refine", stern_tol=1e-8)
    h2 = P.handle_for_cell(small, precision="fp64", stern_tol=1e-10)
    x1 = torch.from_numpy(np.random.default_rng(71).standard_normal((3, big.N_d))).cuda()
    x2 = torch.from_numpy(np.random.default_rng(72).standard_normal((2, small.N_d))).cuda()
    # first call: the larger input, symmetrized, FP32 + refinement
    y1, st1 = h1.chi0_apply_noalloc(0.31, x1, symmetrized=True)
    r1, rs1 = h1.chi0_apply(0.31, x1, symmetrized=True)
    # second call: a smaller cell and fewer vectors, FP64, plain chi0
    y2, st2 = h2.chi0_apply_noalloc(0.0203, x2)
    r2, rs2 = h2.chi0_apply(0.0203, x2)
    torch.cuda.synchronize()
    # start-vector batching changes no bit (fixed-order reductions), so the
    # two entry points agree exactly
    assert torch.equal(y1, r1), (y1 - r1).abs().max().item()
    assert torch.equal(y2, r2), (y2 - r2).abs().max().item()
    for st, rs in ((st1, rs1), (st2, rs2)):
        assert st["n_noconv"] == 0 and st["n_systems"] == rs["n_systems"]
        assert st["cocg_iters_total"] == rs["cocg_iters_total"]
    # the handle's own workspaces are untouched: chi0_apply after the
    # allocation-free call on the same handle still gives the same result
    y3, _ = h2.chi0_apply_noalloc(0.0203, x2[:1])
    assert torch.equal(y3[0], r2[0])
    h1.close()
    h2.close()


def test_noalloc_refuses_a_problem_beyond_its_scratch(P):
    n = (48, 48, 48)
    N = int(np.prod(n))
    psi = np.random.default_rng(73).standard_normal((128, N))
    h = P.Handle(n, (20.52,) * 3, np.zeros(N), psi, np.linspace(-1.0, -0.5, 128))
    with pytest.raises(P.RPAError) as e:
        h.chi0_apply_noalloc(0.5, torch.zeros((1, N), dtype=torch.float64))
    assert e.value.status == P.RPA_E_ARG
    assert "too large" in str(e.value)
    h.close()
