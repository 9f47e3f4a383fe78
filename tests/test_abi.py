"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/rpa.h declares, and its host-only entry points work."""
import ctypes

import numpy as np
import pytest

import oracle as O
import paper_2609_16408_amd as P


def test_library_exports_every_declared_symbol():
    L = P.lib()
    names = P.declared_symbols()
    for required in ("rpa_setup", "chi0_apply", "lanczos_energy_density", "interpolate",
                     "correlation_energy", "rpa_destroy", "rpa_last_error"):
        assert required in names
    for name in names:
        assert hasattr(L, name), name


@pytest.mark.parametrize("n", [1, 2, 3, 8, 16])
def test_host_frequency_rule_matches_oracle(n):
    om, w = P.frequency_rule(n)
    om_o, w_o = O.frequency_rule(n)
    assert np.allclose(om, om_o, rtol=1e-13, atol=0)
    assert np.allclose(w, w_o, rtol=1e-12, atol=0)


def test_frequency_rule_rejects_bad_size():
    with pytest.raises(P.RPAError) as e:
        P.frequency_rule(0)
    assert e.value.status == P.RPA_E_ARG


def test_setup_rejects_bad_arguments_without_a_gpu():
    L = P.lib()
    prm = P.SetupParams()
    prm.n[:] = (5, 12, 12)             # n < 7 is rejected before any device call
    prm.L[:] = (1.0, 1.0, 1.0)
    prm.fd_radius = 6
    prm.n_occ = 2
    h = ctypes.c_void_p()
    st = L.rpa_setup(ctypes.byref(prm), None, ctypes.byref(h))
    assert st == P.RPA_E_ARG
    assert b"n[d]" in L.rpa_last_error(None)
    prm.n[:] = (12, 12, 12)
    prm.fd_radius = 4
    assert L.rpa_setup(ctypes.byref(prm), None, ctypes.byref(h)) == P.RPA_E_ARG


def test_null_handle_is_rejected():
    L = P.lib()
    st = L.interpolate(None, 1, 2, 1, None, None, None)
    assert st == P.RPA_E_ARG
    sig = np.array([0.25])
    st = L.rpa_kinetic_precond_apply(None, 1, sig.ctypes.data, sig.ctypes.data, None, None, None)
    assert st == P.RPA_E_ARG


@pytest.mark.parametrize("n,L", [((5, 12, 12), (1.0, 1.0, 1.0)), ((12, 12, 5000), (1.0, 1.0, 1.0)),
                                 ((12, 12, 12), (1.0, 0.0, 1.0)), ((12, 12, 12), (1.0, float("nan"), 1.0))])
def test_kinetic_precond_create_rejects_bad_grids_without_a_gpu(n, L):
    nn = np.ascontiguousarray(n, dtype=np.int32)
    LL = np.ascontiguousarray(L, dtype=np.float64)
    out = ctypes.c_void_p()
    assert P.lib().rpa_kinetic_precond_create(nn.ctypes.data, LL.ctypes.data, None,
                                              ctypes.byref(out)) == P.RPA_E_ARG
    assert not out.value
    assert P.lib().rpa_kinetic_precond_destroy(None) == P.RPA_OK


@pytest.mark.parametrize("case,msg", [
    ("idx", b"proj_idx out of range"), ("ptr", b"non-decreasing"), ("count", b"n_proj"),
    ("null", b"required"), ("gamma", b"proj_gamma must be finite")])
def test_setup_rejects_bad_projectors_without_a_gpu(case, msg):
    """Projector layouts are validated on the host before any device call."""
    L = P.lib()
    N = 12 ** 3
    eps = np.array([-0.5, -0.4])
    dummy = np.zeros(1)
    prm = P._setup_params((12, 12, 12), (10.0, 10.0, 10.0), dummy.ctypes.data,
                          dummy.ctypes.data, eps, "fp64", 1e-8, 100)
    proj = {"ptr": np.array([0, 3, 6]), "idx": np.array([0, 1, 2, 5, 6, N - 1]),
            "val": np.ones(6), "gamma": np.array([1.0, 2.0])}
    if case == "idx":
        proj["idx"][4] = N
    if case == "ptr":
        proj["ptr"] = np.array([0, 4, 3])
    if case == "gamma":
        proj["gamma"][1] = np.nan
    keep = P._set_proj(prm, proj)
    if case == "count":
        prm.n_proj = 5000
    if case == "null":
        prm.proj_val = None
    h = ctypes.c_void_p()
    assert L.rpa_setup(ctypes.byref(prm), None, ctypes.byref(h)) == P.RPA_E_ARG
    assert msg in L.rpa_last_error(None), L.rpa_last_error(None)
    del keep
