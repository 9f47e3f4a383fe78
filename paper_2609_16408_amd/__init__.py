"""Python binding of librpa_mi355x.so (include/rpa.h): argument marshalling only.

Every step of the RPA hot path runs in the HIP library; PyTorch supplies device
memory and the stream.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os
import warnings

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librpa_mi355x.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "rpa.h")

RPA_OK, RPA_E_ARG, RPA_E_OOM, RPA_E_HIP, RPA_E_STATE = 0, 1, 2, 3, 4
RPA_W_NOCONV, RPA_W_BREAKDOWN = 16, 17
PRECISION = {"fp64": 0, "fp32_refine": 1}
INTERP = {"none": 0, "trilinear": 1, "tricubic": 2, "fourier": 3}

_lib = None


class RPAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"rpa status {status}: {msg}")
        self.status = status


class RPAWarning(UserWarning):
    pass


class SetupParams(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3), ("L", ctypes.c_double * 3),
        ("fd_radius", ctypes.c_int32), ("n_occ", ctypes.c_int32),
        ("v_loc", ctypes.c_void_p), ("psi", ctypes.c_void_p), ("eps", ctypes.c_void_p),
        ("n_proj", ctypes.c_int32), ("proj_ptr", ctypes.c_void_p), ("proj_idx", ctypes.c_void_p),
        ("proj_val", ctypes.c_void_p), ("proj_gamma", ctypes.c_void_p),
        ("precision", ctypes.c_int32), ("stern_tol", ctypes.c_double),
        ("stern_maxit", ctypes.c_int32), ("batch", ctypes.c_int32),
        ("hbm_budget", ctypes.c_uint64), ("tile_y", ctypes.c_int32),
        ("slots_per_cu", ctypes.c_int32), ("inner_tol", ctypes.c_double),
        ("use_graph", ctypes.c_int32), ("fp32_maxit", ctypes.c_int32),
        ("lanczos_breakdown", ctypes.c_double), ("precond", ctypes.c_int32),
        ("precond_omega_min", ctypes.c_double), ("precond_omega_max", ctypes.c_double),
        ("progress", ctypes.c_int32),
        ("n_extra", ctypes.c_int32), ("psi_extra", ctypes.c_void_p), ("eps_extra", ctypes.c_void_p),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_systems", ctypes.c_int64), ("cocg_iters_total", ctypes.c_int64),
        ("cocg_iters_max", ctypes.c_int64), ("refine_cycles", ctypes.c_int64),
        ("n_noconv", ctypes.c_int64), ("n_breakdown", ctypes.c_int64),
        ("seconds", ctypes.c_double), ("n_fp64_fallback", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneResult(ctypes.Structure):
    _fields_ = [("tile_y", ctypes.c_int32), ("slots_per_cu", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("n_tried", ctypes.c_int32),
                ("system_iters_per_s", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerParams(ctypes.Structure):
    _fields_ = [("n_workers", ctypes.c_int32), ("hbm_budget", ctypes.c_uint64),
                ("fake_executor_us", ctypes.c_int32)]


class JobInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_finish", ctypes.c_double),
                ("footprint", ctypes.c_int64), ("stats", Stats)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "stats"}
        d["stats"] = self.stats.as_dict()
        d["latency"] = self.t_finish - self.t_submit
        return d


_VP, _I32, _D, _I64P = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
_SIGS = {
    "rpa_setup": [ctypes.POINTER(SetupParams), _VP, ctypes.POINTER(_VP)],
    "rpa_destroy": [_VP],
    "rpa_frequency_rule": [_I32, _VP, _VP],
    "chi0_apply": [_VP, _D, _I32, _VP, _VP, _I32, ctypes.POINTER(Stats), _VP],
    "chi0_apply_noalloc": [_VP, _D, _I32, _VP, _VP, _I32, ctypes.POINTER(Stats), _VP],
    "lanczos_energy_density": [_VP, _I32, _VP, _I32, _VP, _I32, _VP, ctypes.POINTER(Stats), _VP],
    "lanczos_energy_density_block": [_VP, _I32, _VP, _I32, _VP, _I32, _I32, _VP, ctypes.POINTER(Stats),
                                     _VP],
    "interpolate": [_VP, _I32, _I32, _I32, _VP, _VP, _VP],
    "rpa_energy_from_coarse": [_VP, _I32, _VP, _I32, _I32, _VP, _VP, _VP, _VP],
    "correlation_energy": [_VP, _I32, _VP, _VP, _I32, _I32, _I32, _VP, _VP,
                           ctypes.POINTER(Stats), _VP],
    "rpa_hamiltonian_apply": [_VP, _I32, _VP, _VP, _VP, _VP, _I32, _VP],
    "rpa_coulomb_apply": [_VP, _I32, _I32, _VP, _VP, _VP],
    "rpa_kinetic_precond_create": [_VP, _VP, _VP, _VP],
    "rpa_kinetic_precond_apply": [_VP, _I32, _VP, _VP, _VP, _VP, _VP],
    "rpa_kinetic_precond_destroy": [_VP],
    "rpa_last_cocg_timing": [_VP, _VP, _VP, _VP, _VP, _VP],
    "rpa_last_cocg_split": [_VP, _VP, _VP, _VP],
    "rpa_last_iteration_stats": [_VP, _I32, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP],
    "rpa_sternheimer_solve": [_VP, _D, _I32, _VP, _VP, ctypes.POINTER(Stats), _VP],
    "rpa_release_workspace": [_VP],
    "rpa_autotune": [_VP, _I32, _I32, ctypes.POINTER(TuneResult), _VP],
    "rpa_server_create": [_VP, _VP],
    "rpa_server_add_cell": [_VP, ctypes.POINTER(SetupParams), _VP],
    "rpa_server_submit": [_VP, _I32, _D, _I32, _VP, _I32, _VP, _VP],
    "rpa_server_wait": [_VP, ctypes.c_int64, _VP],
    "rpa_server_status": [_VP, _VP, _VP, _VP, _VP],
    "rpa_server_destroy": [_VP],
}


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2609_16408_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.rpa_last_error.argtypes = [_VP]
        L.rpa_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def declared_symbols() -> list:
    """Function names declared in include/rpa.h."""
    import re
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:rpa_status|const char\*)\s+(\w+)\s*\(", txt, re.M)))


def _check(status, what="", last_error=True):
    if status == RPA_OK:
        return status
    msg = lib().rpa_last_error(None).decode() if last_error else f"status {status}"
    if status in (RPA_W_NOCONV, RPA_W_BREAKDOWN):
        warnings.warn(f"{what}: {msg}", RPAWarning, stacklevel=3)
        return status
    raise RPAError(status, f"{what}: {msg}")


def frequency_rule(n_omega: int):
    om = np.zeros(n_omega)
    w = np.zeros(n_omega)
    _check(lib().rpa_frequency_rule(n_omega, om.ctypes.data, w.ctypes.data), "rpa_frequency_rule")
    return om, w


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Handle:
    """A resident problem (grid, potential, occupied orbitals) on the GPU."""

    def __init__(self, n, L, v_loc, psi, eps, precision="fp64", stern_tol=1e-10,
                 stern_maxit=20000, batch=0, tile_y=0, slots_per_cu=0, inner_tol=0.0,
                 hbm_budget=0, use_graph=False, proj=None, fp32_maxit=0, lanczos_breakdown=0.0,
                 precond=False, precond_window=None, progress=False, extra=None, stream=None):
        import torch
        self._torch = torch
        dev = torch.device("cuda")
        self.n = tuple(int(v) for v in n)
        self.N = int(np.prod(self.n))
        self.L = tuple(float(v) for v in L)
        v = torch.as_tensor(np.ascontiguousarray(v_loc, dtype=np.float64)).to(dev) \
            if not torch.is_tensor(v_loc) else v_loc.to(dev, torch.float64).contiguous()
        p = torch.as_tensor(np.ascontiguousarray(psi, dtype=np.float64)).to(dev) \
            if not torch.is_tensor(psi) else psi.to(dev, torch.float64).contiguous()
        self.eps = np.ascontiguousarray(eps, dtype=np.float64)
        self.n_occ = int(self.eps.size)
        assert p.shape == (self.n_occ, self.N) and v.numel() == self.N
        prm = SetupParams()
        prm.n[:] = self.n
        prm.L[:] = self.L
        prm.fd_radius = 6
        prm.n_occ = self.n_occ
        prm.v_loc = v.data_ptr()
        prm.psi = p.data_ptr()
        prm.eps = self.eps.ctypes.data
        keep = _set_proj(prm, proj)   # host arrays, copied by rpa_setup
        prm.precision = PRECISION[precision]
        prm.stern_tol = float(stern_tol)
        prm.stern_maxit = int(stern_maxit)
        prm.batch = int(batch)
        prm.hbm_budget = int(hbm_budget)
        prm.tile_y = int(tile_y)
        prm.slots_per_cu = int(slots_per_cu)
        prm.inner_tol = float(inner_tol)
        prm.use_graph = 1 if use_graph else 0
        prm.fp32_maxit = int(fp32_maxit)
        prm.lanczos_breakdown = float(lanczos_breakdown)
        prm.precond = 1 if precond else 0
        if precond_window is not None:
            prm.precond_omega_min, prm.precond_omega_max = (float(v) for v in precond_window)
        prm.progress = 1 if progress else 0
        if extra is not None:
            # extra eigenpairs (psi_extra [n_x][N], eps_extra [n_x]) widen the Galerkin guess
            px, ex = extra
            px = torch.as_tensor(np.ascontiguousarray(px, dtype=np.float64)).to(dev) \
                if not torch.is_tensor(px) else px.to(dev, torch.float64).contiguous()
            ex = np.ascontiguousarray(ex, dtype=np.float64)
            assert px.shape == (ex.size, self.N)
            prm.n_extra = int(ex.size)
            prm.psi_extra = px.data_ptr()
            prm.eps_extra = ex.ctypes.data
            self._extra_keep = (px, ex)
        h = ctypes.c_void_p()
        _check(lib().rpa_setup(ctypes.byref(prm), _stream(stream), ctypes.byref(h)), "rpa_setup")
        del keep
        self._h = h
        self.precision = precision

    def autotune(self, n_lanczos=8, probe_iters=0, stream=None):
        """Time the candidate launch shapes and keep the fastest (rpa_autotune)."""
        res = TuneResult()
        _check(lib().rpa_autotune(self._h, int(n_lanczos), int(probe_iters), ctypes.byref(res),
                                  _stream(stream)), "rpa_autotune")
        return res.as_dict()

    def release_workspace(self):
        """Free the workspaces (resident cell data stays); captured graphs are dropped."""
        _check(lib().rpa_release_workspace(self._h), "rpa_release_workspace")

    def close(self):
        if getattr(self, "_pc", None):
            lib().rpa_kinetic_precond_destroy(self._pc)
            self._pc = None
        if getattr(self, "_h", None):
            lib().rpa_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f64(self, x):
        return x.to(self._torch.device("cuda"), self._torch.float64).contiguous()

    def chi0_apply(self, omega, x, symmetrized=False, stream=None):
        x = self._f64(x).reshape(-1, self.N)
        y = self._torch.empty_like(x)
        st = Stats()
        _check(lib().chi0_apply(self._h, float(omega), x.shape[0], _ptr(x), _ptr(y),
                                1 if symmetrized else 0, ctypes.byref(st), _stream(stream)),
               "chi0_apply")
        return y, st.as_dict()

    def chi0_apply_noalloc(self, omega, x, y=None, symmetrized=False, stream=None):
        """chi0_apply through the allocation-free entry point; y (FP64
        [nvec, N] on the device) may be supplied by the caller."""
        x = self._f64(x).reshape(-1, self.N)
        if y is None:
            y = self._torch.empty_like(x)
        st = Stats()
        _check(lib().chi0_apply_noalloc(self._h, float(omega), x.shape[0], _ptr(x), _ptr(y),
                                        1 if symmetrized else 0, ctypes.byref(st), _stream(stream)),
               "chi0_apply_noalloc")
        return y, st.as_dict()

    def sternheimer_solve(self, omega, u, stream=None):
        """Solutions x[v, n] of (H - eps_n - i omega) x = -psi_n * u[v]
        (complex128 [nvec, n_occ, N])."""
        u = self._f64(u).reshape(-1, self.N)
        x = self._torch.empty((u.shape[0], self.n_occ, self.N), dtype=self._torch.complex128,
                              device="cuda")
        st = Stats()
        _check(lib().rpa_sternheimer_solve(self._h, float(omega), u.shape[0], _ptr(u), _ptr(x),
                                           ctypes.byref(st), _stream(stream)),
               "rpa_sternheimer_solve")
        return x, st.as_dict()

    def lanczos_energy_density(self, omegas, points, n_lanczos, stream=None):
        om = np.ascontiguousarray(omegas, dtype=np.float64)
        pts = np.ascontiguousarray(points, dtype=np.int64)
        d = self._torch.empty((om.size, pts.size), dtype=self._torch.float64, device="cuda")
        st = Stats()
        _check(lib().lanczos_energy_density(self._h, om.size, om.ctypes.data, pts.size,
                                            pts.ctypes.data, int(n_lanczos), _ptr(d),
                                            ctypes.byref(st), _stream(stream)),
               "lanczos_energy_density")
        return d, st.as_dict()

    def lanczos_energy_density_block(self, omegas, points, n_lanczos, block, stream=None):
        """Block Lanczos quadrature over consecutive groups of `block` points
        per frequency; d[k, p] as lanczos_energy_density."""
        om = np.ascontiguousarray(omegas, dtype=np.float64)
        pts = np.ascontiguousarray(points, dtype=np.int64)
        d = self._torch.empty((om.size, pts.size), dtype=self._torch.float64, device="cuda")
        st = Stats()
        _check(lib().lanczos_energy_density_block(self._h, om.size, om.ctypes.data, pts.size,
                                                  pts.ctypes.data, int(n_lanczos), int(block), _ptr(d),
                                                  ctypes.byref(st), _stream(stream)),
               "lanczos_energy_density_block")
        return d, st.as_dict()

    def interpolate(self, kind, stride, coarse, stream=None):
        c = self._f64(coarse)
        nf = c.shape[0] if c.dim() == 2 else 1
        fine = self._torch.empty((nf, self.N), dtype=self._torch.float64, device="cuda")
        _check(lib().interpolate(self._h, INTERP[kind], int(stride), nf, _ptr(c), _ptr(fine),
                                 _stream(stream)), "interpolate")
        return fine

    def energy_from_coarse(self, weights, stride, kind, d_coarse, want_fine=True, stream=None):
        w = np.ascontiguousarray(weights, dtype=np.float64)
        dc = self._f64(d_coarse)
        e_c = ctypes.c_double()
        e_fine = self._torch.empty(self.N, dtype=self._torch.float64, device="cuda") if want_fine else None
        _check(lib().rpa_energy_from_coarse(self._h, w.size, w.ctypes.data, int(stride), INTERP[kind],
                                            _ptr(dc), ctypes.byref(e_c),
                                            _ptr(e_fine) if want_fine else None, _stream(stream)),
               "rpa_energy_from_coarse")
        return e_c.value, e_fine

    def correlation_energy(self, omegas, weights, stride, kind, n_lanczos, want_fine=True,
                           stream=None):
        om = np.ascontiguousarray(omegas, dtype=np.float64)
        w = np.ascontiguousarray(weights, dtype=np.float64)
        e_c = ctypes.c_double()
        e_fine = self._torch.empty(self.N, dtype=self._torch.float64, device="cuda") if want_fine else None
        st = Stats()
        _check(lib().correlation_energy(self._h, om.size, om.ctypes.data, w.ctypes.data,
                                        int(stride), INTERP[kind], int(n_lanczos),
                                        ctypes.byref(e_c), _ptr(e_fine) if want_fine else None,
                                        ctypes.byref(st), _stream(stream)),
               "correlation_energy")
        return e_c.value, e_fine, st.as_dict()

    def hamiltonian_apply(self, shifts, x, precision="fp64", stream=None):
        """y = (H - shift_v) x_v for complex x [nvec, N] (complex128 for fp64,
        complex64 for the FP32 stencil)."""
        torch = self._torch
        dt = torch.complex128 if precision == "fp64" else torch.complex64
        x = x.to(torch.device("cuda"), dt).contiguous().reshape(-1, self.N)
        y = torch.empty_like(x)
        sh = np.asarray(shifts, dtype=np.complex128).reshape(-1)
        sr = np.ascontiguousarray(sh.real)
        si = np.ascontiguousarray(sh.imag)
        _check(lib().rpa_hamiltonian_apply(self._h, x.shape[0], sr.ctypes.data, si.ctypes.data,
                                           _ptr(x), _ptr(y), PRECISION[precision],
                                           _stream(stream)), "rpa_hamiltonian_apply")
        return y

    def coulomb_apply(self, power, x, stream=None):
        x = self._f64(x).reshape(-1, self.N)
        y = self._torch.empty_like(x)
        _check(lib().rpa_coulomb_apply(self._h, int(power), x.shape[0], _ptr(x), _ptr(y),
                                       _stream(stream)), "rpa_coulomb_apply")
        return y

    def kinetic_precond_apply(self, x, sigma, stream=None):
        """(-1/2 Lap_h + sigma_v)^-1 x[v] for complex x [nvec][N_d]; sigma: nvec complex."""
        t = self._torch
        x = t.as_tensor(x).to(t.device("cuda")).reshape(-1, self.N)
        nvec = x.shape[0]
        sg = np.asarray(sigma, dtype=np.complex128).reshape(-1)
        if sg.size == 1:
            sg = np.full(nvec, sg[0])
        if sg.size != nvec:
            raise ValueError("one sigma per vector")
        xp = t.stack([x.real, x.imag], dim=1).to(t.float64).contiguous() if x.is_complex() \
            else t.stack([x.to(t.float64), t.zeros_like(x, dtype=t.float64)], dim=1).contiguous()
        yp = t.empty_like(xp)
        sr = np.ascontiguousarray(sg.real)
        si = np.ascontiguousarray(sg.imag)
        if getattr(self, "_pc", None) is None:
            n = np.ascontiguousarray(self.n, dtype=np.int32)
            L = np.ascontiguousarray(self.L, dtype=np.float64)
            pc = ctypes.c_void_p()
            _check(lib().rpa_kinetic_precond_create(n.ctypes.data, L.ctypes.data, _stream(stream),
                                                    ctypes.byref(pc)), "rpa_kinetic_precond_create",
                   last_error=False)
            self._pc = pc
        _check(lib().rpa_kinetic_precond_apply(self._pc, nvec, sr.ctypes.data, si.ctypes.data,
                                               _ptr(xp), _ptr(yp), _stream(stream)),
               "rpa_kinetic_precond_apply", last_error=False)
        return t.complex(yp[:, 0], yp[:, 1])

    def last_iteration_stats(self):
        """Per-frequency COCG iteration statistics of the last chi0_apply /
        lanczos_energy_density call: a list of dicts (omega, solves, mean,
        std, min, max), one per frequency argument of that call."""
        n = ctypes.c_int32()
        _check(lib().rpa_last_iteration_stats(self._h, 0, None, None, None, None, None, None, None,
                                              ctypes.byref(n)), "rpa_last_iteration_stats")
        k = n.value
        om, mean, sd = np.zeros(k), np.zeros(k), np.zeros(k)
        cnt, mn, mx, cyc = (np.zeros(k, dtype=np.int64) for _ in range(4))
        _check(lib().rpa_last_iteration_stats(self._h, k, om.ctypes.data, cnt.ctypes.data,
                                              mean.ctypes.data, sd.ctypes.data, mn.ctypes.data,
                                              mx.ctypes.data, cyc.ctypes.data, ctypes.byref(n)),
               "rpa_last_iteration_stats")
        return [{"omega": float(om[i]), "solves": int(cnt[i]), "mean": float(mean[i]),
                 "std": float(sd[i]), "min": int(mn[i]), "max": int(mx[i]),
                 "refine_cycles": int(cyc[i])} for i in range(k)]

    def last_cocg_split(self):
        """Sternheimer launch time of the last call (ms) by kernel: plain,
        preconditioned, FP64 follow-up."""
        v = [ctypes.c_double() for _ in range(3)]
        _check(lib().rpa_last_cocg_split(self._h, *(ctypes.byref(x) for x in v)), "rpa_last_cocg_split")
        return {"plain": v[0].value, "precond": v[1].value, "followup": v[2].value}

    def last_cocg_timing(self):
        ms = ctypes.c_double()
        launches, grid, block, ty = (ctypes.c_int32() for _ in range(4))
        _check(lib().rpa_last_cocg_timing(self._h, ctypes.byref(ms), ctypes.byref(launches),
                                          ctypes.byref(grid), ctypes.byref(block),
                                          ctypes.byref(ty)), "rpa_last_cocg_timing")
        return {"ms": ms.value, "launches": launches.value, "grid": grid.value,
                "block": block.value, "tile_y": ty.value}


def _set_proj(prm, proj):
    """Fill the projector fields of SetupParams from a dict with CSR arrays
    'ptr', 'idx', 'val', 'gamma' (None: no projectors); returns the arrays,
    which must stay alive until the C call that reads them returns."""
    if proj is None:
        prm.n_proj = 0
        return ()
    ptr = np.ascontiguousarray(proj["ptr"], dtype=np.int64)
    idx = np.ascontiguousarray(proj["idx"], dtype=np.int64)
    val = np.ascontiguousarray(proj["val"], dtype=np.float64)
    gam = np.ascontiguousarray(proj["gamma"], dtype=np.float64)
    prm.n_proj = int(ptr.size - 1)
    prm.proj_ptr, prm.proj_idx = ptr.ctypes.data, idx.ctypes.data
    prm.proj_val, prm.proj_gamma = val.ctypes.data, gam.ctypes.data
    return (ptr, idx, val, gam)


def _setup_params(n, L, v_ptr, psi_ptr, eps, precision, stern_tol, stern_maxit, batch=0,
                  tile_y=0, slots_per_cu=0, inner_tol=0.0, hbm_budget=0):
    prm = SetupParams()
    prm.n[:] = tuple(int(x) for x in n)
    prm.L[:] = tuple(float(x) for x in L)
    prm.fd_radius = 6
    prm.n_occ = int(eps.size)
    prm.v_loc = v_ptr
    prm.psi = psi_ptr
    prm.eps = eps.ctypes.data
    prm.n_proj = 0
    prm.precision = PRECISION[precision]
    prm.stern_tol = float(stern_tol)
    prm.stern_maxit = int(stern_maxit)
    prm.batch = int(batch)
    prm.hbm_budget = int(hbm_budget)
    prm.tile_y = int(tile_y)
    prm.slots_per_cu = int(slots_per_cu)
    prm.inner_tol = float(inner_tol)
    return prm


class Server:
    """Energy-density serving loop (rpa_server_* of the C ABI)."""

    def __init__(self, n_workers=3, hbm_budget=0, fake_executor_us=0):
        p = ServerParams(int(n_workers), int(hbm_budget), int(fake_executor_us))
        h = ctypes.c_void_p()
        _check(lib().rpa_server_create(ctypes.byref(p), ctypes.byref(h)), "rpa_server_create")
        self._h = h
        self.fake = fake_executor_us > 0
        self._keep = {}
        self._out = {}

    def add_cell(self, n, L, v_loc, psi, eps, precision="fp32_refine", stern_tol=1e-6,
                 stern_maxit=20000, batch=0, proj=None):
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        if self.fake:
            prm = _setup_params(n, L, None, None, eps, precision, stern_tol, stern_maxit, batch)
        else:
            import torch
            v = torch.as_tensor(np.ascontiguousarray(v_loc, dtype=np.float64)).cuda()
            p = torch.as_tensor(np.ascontiguousarray(psi, dtype=np.float64)).cuda()
            prm = _setup_params(n, L, v.data_ptr(), p.data_ptr(), eps, precision, stern_tol,
                                stern_maxit, batch)
        keep = _set_proj(prm, proj)   # copied by rpa_server_add_cell
        cid = ctypes.c_int32()
        _check(lib().rpa_server_add_cell(self._h, ctypes.byref(prm), ctypes.byref(cid)),
               "rpa_server_add_cell")
        del keep
        self._keep[cid.value] = eps
        return cid.value

    def submit(self, cell_id, omega, points, n_lanczos):
        pts = np.ascontiguousarray(points, dtype=np.int64)
        out = None
        if not self.fake:
            import torch
            out = torch.empty(pts.size, dtype=torch.float64, device="cuda")
        jid = ctypes.c_int64()
        _check(lib().rpa_server_submit(self._h, int(cell_id), float(omega), pts.size,
                                       pts.ctypes.data, int(n_lanczos),
                                       _ptr(out) if out is not None else None, ctypes.byref(jid)),
               "rpa_server_submit")
        self._out[jid.value] = out
        return jid.value

    def wait(self, job_id):
        info = JobInfo()
        _check(lib().rpa_server_wait(self._h, ctypes.c_int64(job_id), ctypes.byref(info)),
               "rpa_server_wait")
        return self._out.pop(job_id, None), info.as_dict()

    def status(self):
        w, r = ctypes.c_int32(), ctypes.c_int32()
        u, hw = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().rpa_server_status(self._h, ctypes.byref(w), ctypes.byref(r), ctypes.byref(u),
                                       ctypes.byref(hw)), "rpa_server_status")
        return {"waiting": w.value, "running": r.value, "in_use": u.value, "high_water": hw.value}

    def close(self):
        if getattr(self, "_h", None):
            lib().rpa_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def handle_for_cell(cell, **kw) -> Handle:
    """Handle for a synthcell.Cell (convenience for tests and the benchmark)."""
    kw.setdefault("proj", cell.proj)
    return Handle(cell.n, cell.L, cell.v_loc, cell.psi, cell.eps, **kw)
