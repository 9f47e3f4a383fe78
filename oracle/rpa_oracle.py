"""FP64 CPU oracle of the matrix-free real-space RPA method (Lanczos quadrature
on coarse grid points, interpolation, frequency integration).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP library.

Every function states the passage of the paper it follows.  Where the paper
is silent or ambiguous the reading taken is stated in the docstring:

  R1 (Background, Eq. 1, the Coulomb operator): nu = 4 pi (-Lap_h)^-1 on
     zero-mean fields; the G = 0 mode is dropped.  With the literal sign
     f(nu chi0) could become complex; only the positive operator keeps
     nu^1/2 chi0 nu^1/2 negative semidefinite.
  R2 (Implementation, Kronecker nu^1/2): Lap_h is the same 12th-order FD
     Laplacian as in H, diagonalised axis by axis.
  R3 (Background, Eqs. 2 and 4; Algorithm 1 accumulation with factor 4):
     orbitals are normalised h^3 sum psi^2 = 1 and the response acts on
     function values with the quadrature weight h^3, so the Sternheimer
     accumulation 4 sum_n psi_n Re dpsi_n equals h^3 * chi0(Eq. 2) u.
  R4 (Trace Approximations, Eq. 8 and Algorithm 1): the per-point quantity
     is e_j^T f(nu^1/2 chi0 nu^1/2) e_j.
  R5 (Eq. 9 vs Algorithm 1): the 1/(2 pi) prefactor of Eq. 9 is kept.
  R6 (Eq. 9): Gauss-Legendre nodes x_k mapped by omega = (1+x)/(1-x), with
     weights W_k * 2/(1-x_k)^2.  The mapping reproduces the omega column of
     the COCG iteration tables.
  R7 (Algorithm 1 Lanczos loop): full reorthogonalisation (two classical
     Gram-Schmidt passes against every stored q) after the three-term
     update; T is N_l x N_l; breakdown when beta_k <= 1e-13 max|alpha|,
     which truncates T.
  R8 (Implementation, COCG): stop when ||b - A x||_2 <= tol ||b||_2 using the
     recursively updated residual; b is the right-hand side of Eq. 4.
  R9 (Implementation, Galerkin initial guess): exact solve inside the
     occupied span, x0 = sum_m psi_m (h^3 psi_m^T b) / (eps_m - eps_n - i w).
  R10 (Interpolating Diagonal Entries, coarse set C_g): points whose three
     indices are all multiples of g.
  R11 (tricubic): separable 4-point Lagrange interpolation, periodic.
  R12 (Fourier): per-axis spectrum zero-padding, the even-length Nyquist
     coefficient split evenly between +k and -k.
  R17 (Conclusions and Future Work, preconditioned Sternheimer solves):
     preconditioned COCG (z = M^-1 r, rho = r^T z) with the shifted kinetic operator
     M_n = -1/2 Lap_h + sigma_n, sigma_n = max(mean V_loc - eps_n, 1/4 Ha) - i w,
     inverted exactly in the per-axis eigenbasis of Lap_h; the stopping rule
     R8 is unchanged, so the solution tolerance is that of the plain solve.
  R19 (block COCG, not in the paper, which uses plain COCG): block
     conjugate gradient over right-hand sides that share (orbital, frequency),
     with unconjugated transposes; block size 1 is COCG.  In the oracle only,
     to measure whether it would cut the solves' cost.
  R18 (Conclusions and Future Work, block Lanczos quadrature): block Gauss
     quadrature from Q_1 = [e_j for a group of points]; block three-term
     recurrence with thin QR, full reorthogonalisation as in R7, breakdown when
     a diagonal entry of B_k falls to 1e-13 max|A_k|; d_j is the j-th diagonal
     entry of E_1^T f(T) E_1 for the block tridiagonal T.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

FOUR_PI = 4.0 * math.pi

__all__ = [
    "fd_weights", "d2_periodic_1d", "laplacian", "Hamiltonian", "Coulomb",
    "chi0_sos", "galerkin_guess", "cocg", "chi0_apply", "nuhalf_chi0_nuhalf",
    "lanczos_tridiag", "tridiag_quadrature", "f_rpa", "exact_diag_f",
    "frequency_rule", "interpolation_matrix_1d", "interpolate",
    "correlation_energy_from_coarse", "energy_density", "interp_metrics",
    "coarse_index_set", "KineticPreconditioner", "kinetic_shift", "cocg_precond",
    "block_lanczos", "block_tridiag", "block_quadrature", "energy_density_block",
    "galerkin_space", "block_cocg",
]


# -----------------------------------------------------------------------------
# Finite differences (the discretised Hamiltonian of Eq. 3; 12th order)
# -----------------------------------------------------------------------------

def fd_weights(radius: int = 6) -> list:
    """Central second-derivative weights w_0..w_R for unit spacing.

    Fornberg's closed form for the symmetric stencil of order 2R:
    w_k = 2 (-1)^(k+1) (R!)^2 / (k^2 (R-k)! (R+k)!), w_0 = -2 sum_k w_k.
    """
    R = radius
    w = [Fraction(2 * (-1) ** (k + 1) * math.factorial(R) ** 2,
                  k * k * math.factorial(R - k) * math.factorial(R + k)) for k in range(1, R + 1)]
    return [-2 * sum(w)] + w


def d2_periodic_1d(n: int, h: float, radius: int = 6) -> np.ndarray:
    """Dense periodic 1D second-derivative matrix (circulant)."""
    w = [float(x) for x in fd_weights(radius)]
    D = np.zeros((n, n))
    for i in range(n):
        D[i, i] += w[0]
        for k in range(1, radius + 1):
            D[i, (i + k) % n] += w[k]
            D[i, (i - k) % n] += w[k]
    return D / (h * h)


def laplacian(n, L, radius: int = 6) -> sp.csr_matrix:
    """Lap_h = D2_x (x) I (x) I + I (x) D2_y (x) I + I (x) I (x) D2_z (z fastest)."""
    D = [sp.csr_matrix(d2_periodic_1d(n[d], L[d] / n[d], radius)) for d in range(3)]
    I = [sp.identity(n[d], format="csr") for d in range(3)]
    lap = sp.kron(sp.kron(D[0], I[1]), I[2]) + sp.kron(sp.kron(I[0], D[1]), I[2]) \
        + sp.kron(sp.kron(I[0], I[1]), D[2])
    return lap.tocsr()


class Hamiltonian:
    """H = -1/2 Lap_h + diag(V_loc) + V_nl (Background, Eq. 3, FD form).

    V_nl = h^3 sum_p gamma_p chi_p chi_p^T for separable projectors given in
    CSR form (ptr, idx, val, gamma).
    """

    def __init__(self, n, L, v_loc, proj=None, radius: int = 6):
        self.n = tuple(n)
        self.L = tuple(L)
        self.N = int(np.prod(n))
        self.dV = float(np.prod([L[d] / n[d] for d in range(3)]))
        self.H = (-0.5 * laplacian(n, L, radius) + sp.diags(np.asarray(v_loc, dtype=np.float64))).tocsr()
        self.P = None
        if proj is not None:
            ptr = np.asarray(proj["ptr"])
            rows = np.repeat(np.arange(ptr.size - 1), np.diff(ptr))
            self.P = sp.csr_matrix((proj["val"], (rows, proj["idx"])), shape=(ptr.size - 1, self.N))
            self.gamma = np.asarray(proj["gamma"], dtype=np.float64)

    def apply(self, x):
        y = self.H @ x
        if self.P is not None:
            c = self.P @ x
            c = (self.gamma * self.dV)[:, None] * c if c.ndim == 2 else self.gamma * self.dV * c
            y = y + self.P.T @ c
        return y

    def dense(self) -> np.ndarray:
        Hd = self.H.toarray()
        if self.P is not None:
            Pd = self.P.toarray()
            Hd = Hd + self.dV * (Pd.T * self.gamma) @ Pd
        return Hd

    def shifted_sparse(self, z: complex) -> sp.csc_matrix:
        """H - z I as a sparse matrix (for the direct-solve 'exact' mode)."""
        A = self.H.astype(np.complex128) - z * sp.identity(self.N, dtype=np.complex128, format="csr")
        if self.P is not None:
            A = A + self.dV * (self.P.T @ sp.diags(self.gamma) @ self.P)
        return A.tocsc()


# -----------------------------------------------------------------------------
# Coulomb operator nu and nu^1/2 (Background Eq. 1; Implementation: Kronecker)
# -----------------------------------------------------------------------------

class Coulomb:
    """nu^s = 4 pi^s (-Lap_h)^-s through the per-axis eigendecomposition.

    Each periodic 1D D2 = V diag(lam) V^T (numpy eigh); the 3D eigenvalues of
    -Lap_h are mu = -(lam_x + lam_y + lam_z) >= 0 and the single mu = 0 mode
    (the constant) is dropped (reading R1).  Application is the Kronecker form
    (V_x (x) V_y (x) V_z) diag(s) (V_x (x) V_y (x) V_z)^T.
    """

    def __init__(self, n, L, radius: int = 6):
        self.n = tuple(n)
        self.V = []
        lams = []
        for d in range(3):
            lam, V = np.linalg.eigh(d2_periodic_1d(n[d], L[d] / n[d], radius))
            self.V.append(V)
            lams.append(lam)
        mu = -(lams[0][:, None, None] + lams[1][None, :, None] + lams[2][None, None, :])
        zero = mu <= 1e-10 * mu.max()
        if int(zero.sum()) != 1:
            raise RuntimeError("expected exactly one zero mode of -Lap_h")
        self.mu = np.where(zero, 1.0, mu)
        self.zero = zero
        self.s_half = np.where(zero, 0.0, np.sqrt(FOUR_PI / self.mu))
        self.s_full = np.where(zero, 0.0, FOUR_PI / self.mu)

    def _kron(self, q, s):
        Q = np.asarray(q, dtype=np.float64).reshape(self.n)
        Vx, Vy, Vz = self.V
        C = np.einsum("ia,jb,kc,ijk->abc", Vx, Vy, Vz, Q, optimize=True)
        C = C * s
        return np.einsum("ia,jb,kc,abc->ijk", Vx, Vy, Vz, C, optimize=True).reshape(-1)

    def half(self, q):
        return self._kron(q, self.s_half)

    def full(self, q):
        return self._kron(q, self.s_full)

    def dense_half(self) -> np.ndarray:
        N = int(np.prod(self.n))
        return np.stack([self.half(e) for e in np.eye(N)], axis=1)


# -----------------------------------------------------------------------------
# chi0: explicit sum over states (Eq. 2) and Sternheimer form (Eq. 4)
# -----------------------------------------------------------------------------

def chi0_sos(psi_all: np.ndarray, eps_all: np.ndarray, n_occ: int, omega: float, dV: float) -> np.ndarray:
    """Dense chi0(i omega) of Eq. 2 acting on function values (weight h^3).

    psi_all holds *all* eigenvectors of the discrete H (rows, h^3-normalised),
    occupations are 1 for the n_occ lowest states and 0 otherwise, the factor 2
    of Eq. 2 is the spin sum.  Only pairs with f_j != f_k contribute; the pair
    (j,k) and its mirror (k,j) are summed with their complex denominators and
    the (vanishing) imaginary part is discarded after a check.
    """
    N_states, N = psi_all.shape
    chi = np.zeros((N, N))
    occ = np.arange(n_occ)
    unocc = np.arange(n_occ, N_states)
    for j in occ:
        P = psi_all[j][None, :] * psi_all[unocc]            # psi_j psi_k, k unoccupied
        # (f_j - f_k) = +1 for (j occ, k unocc) and -1 for the mirrored pair
        c = 1.0 / (eps_all[j] - eps_all[unocc] - 1j * omega) \
            - 1.0 / (eps_all[unocc] - eps_all[j] - 1j * omega)
        if np.max(np.abs(c.imag)) > 1e-12 * max(1.0, np.max(np.abs(c.real))):
            raise AssertionError("Eq. 2 pair sum should be real")
        chi += 2.0 * dV * (P.T * c.real) @ P
    return chi


def galerkin_guess(psi: np.ndarray, eps: np.ndarray, n: int, b: np.ndarray, omega: float, dV: float):
    """Initial guess by Galerkin projection onto the occupied orbitals (R9)."""
    c = dV * (psi @ b)                                   # h^3 psi_m^T b
    return (c / (eps - eps[n] - 1j * omega)) @ psi


def galerkin_space(psi: np.ndarray, eps: np.ndarray, psi_extra=None, eps_extra=None):
    """Eigenpairs spanned by the Galerkin guess: the occupied ones, then any
    further eigenpairs of H given (an extension of R9, not in the paper)."""
    if (psi_extra is None) != (eps_extra is None):
        raise ValueError("psi_extra and eps_extra go together")
    if psi_extra is None:
        return psi, eps
    return np.vstack([psi, psi_extra]), np.concatenate([eps, eps_extra])


def cocg(apply_A, b: np.ndarray, x0: np.ndarray, tol: float, maxit: int):
    """Conjugate Orthogonal CG for complex symmetric A (unconjugated u^T v).

    Returns (x, iterations, status) with status 'ok', 'noconv' or 'breakdown'.
    Stopping rule R8.
    """
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b, dtype=np.complex128), 0, "ok"
    x = np.array(x0, dtype=np.complex128)
    r = b - apply_A(x)
    if np.linalg.norm(r) <= tol * bnorm:
        return x, 0, "ok"
    p = r.copy()
    rho = r @ r
    for it in range(1, maxit + 1):
        q = apply_A(p)
        mu = p @ q
        if abs(mu) < 1e-300:
            return x, it, "breakdown"
        alpha = rho / mu
        x = x + alpha * p
        r = r - alpha * q
        if np.linalg.norm(r) <= tol * bnorm:
            return x, it, "ok"
        rho_new = r @ r
        p = r + (rho_new / rho) * p
        rho = rho_new
    return x, maxit, "noconv"


def chi0_apply(ham: Hamiltonian, psi: np.ndarray, eps: np.ndarray, u: np.ndarray, omega: float,
               tol: float = 1e-10, maxit: int = 20000, exact: bool = False, stats: dict | None = None,
               precond: "KineticPreconditioner | None" = None, v_loc: np.ndarray | None = None,
               psi_extra: np.ndarray | None = None, eps_extra: np.ndarray | None = None,
               orbitals=None):
    """r = chi0(i omega) u by the Sternheimer route (Eq. 4; Algorithm 1 inner loop).

    For each occupied n: solve (H - eps_n - i omega) dpsi_n = -psi_n (.) u by
    COCG from the Galerkin guess (or by a sparse direct solve when exact=True),
    then accumulate r += 4 psi_n (.) Re dpsi_n.  With `precond` (and the
    local potential `v_loc` for its shift) the solves are preconditioned
    COCG with the shifted kinetic operator (reading R17).  With `psi_extra`,
    `eps_extra` (further eigenpairs of H above the occupied ones) the
    Galerkin guess spans them too; the accumulation stays over the occupied
    orbitals only.  With `orbitals` (indices n) only those solves are done and
    accumulated: the sum over n of Algorithm 1 split into parts, which sum to
    the full result (the Galerkin guess still spans every occupied orbital).
    """
    if precond is not None and v_loc is None:
        raise ValueError("the preconditioner shift needs v_loc")
    psi_g, eps_g = galerkin_space(psi, eps, psi_extra, eps_extra)
    r = np.zeros(ham.N)
    for n in (range(psi.shape[0]) if orbitals is None else orbitals):
        b = -psi[n] * u
        z = eps[n] + 1j * omega
        if exact:
            x = spla.spsolve(ham.shifted_sparse(z), b.astype(np.complex128))
            its, status = 0, "ok"
        else:
            x0 = galerkin_guess(psi_g, eps_g, n, b, omega, ham.dV)
            if precond is None:
                x, its, status = cocg(lambda v, z=z: ham.apply(v) - z * v, b, x0, tol, maxit)
            else:
                sigma = kinetic_shift(v_loc, eps[n], omega)
                x, its, status = cocg_precond(lambda v, z=z: ham.apply(v) - z * v,
                                              lambda r, sg=sigma: precond.apply(r, sg), b, x0, tol, maxit)
        if stats is not None:
            stats.setdefault("iters", []).append(its)
            if status != "ok":
                stats.setdefault("flags", []).append(status)
        r += 4.0 * psi[n] * x.real
    return r


def nuhalf_chi0_nuhalf(ham, coul, psi, eps, omega, tol=1e-10, maxit=20000, exact=False, stats=None,
                       precond=None, v_loc=None):
    """Matrix-free A~ = nu^1/2 chi0 nu^1/2 (Trace Approximations, Eq. 8);
    with `precond` (and v_loc) the solves are preconditioned (reading R17)."""
    def apply(q):
        u = coul.half(q)
        r = chi0_apply(ham, psi, eps, u, omega, tol=tol, maxit=maxit, exact=exact, stats=stats,
                       precond=precond, v_loc=v_loc)
        return coul.half(r)
    return apply


# -----------------------------------------------------------------------------
# Lanczos quadrature (Eqs. 6-7, Algorithm 1)
# -----------------------------------------------------------------------------

def f_rpa(lam):
    """f(x) = log(1 - x) + x (Trace Approximations)."""
    lam = np.asarray(lam, dtype=np.float64)
    return np.log1p(-lam) + lam


def lanczos_tridiag(apply_A, q1: np.ndarray, m: int, breakdown_rel: float = 1e-13):
    """m Lanczos steps on symmetric A from unit q1; returns (alpha, beta, broke).

    Three-term recurrence of Algorithm 1 followed by full reorthogonalisation
    (reading R7).  beta has length len(alpha) - 1.
    """
    Q = [np.array(q1, dtype=np.float64)]
    alpha, beta = [], []
    q_prev = np.zeros_like(Q[0])
    beta_prev = 0.0
    broke = False
    for k in range(m):
        v = apply_A(Q[k])
        a = float(Q[k] @ v)
        v = v - a * Q[k] - beta_prev * q_prev
        Qm = np.array(Q)
        for _ in range(2):
            v = v - Qm.T @ (Qm @ v)
        alpha.append(a)
        if k < m - 1:
            bk = float(np.linalg.norm(v))
            if bk <= breakdown_rel * max(abs(x) for x in alpha):
                broke = True
                break
            beta.append(bk)
            q_prev = Q[k]
            beta_prev = bk
            Q.append(v / bk)
    return np.array(alpha), np.array(beta), broke


def tridiag_quadrature(alpha: np.ndarray, beta: np.ndarray) -> float:
    """[f(T)]_11 = sum_i Q_1i^2 f(lambda_i) for T = tridiag(beta, alpha, beta)."""
    if len(alpha) == 1:
        return float(f_rpa(alpha[0]))
    lam, Q = sla.eigh_tridiagonal(np.asarray(alpha), np.asarray(beta))
    return float(np.sum(Q[0, :] ** 2 * f_rpa(lam)))


def exact_diag_f(A: np.ndarray) -> np.ndarray:
    """diag f(A) of a dense symmetric A from its eigendecomposition."""
    lam, U = np.linalg.eigh(0.5 * (A + A.T))
    return (U * U) @ f_rpa(lam)


# -----------------------------------------------------------------------------
# Frequency quadrature (Eq. 9)
# -----------------------------------------------------------------------------

def frequency_rule(n_omega: int):
    """Gauss-Legendre on [-1, 1] mapped to [0, inf) by omega = (1+x)/(1-x) (R6)."""
    x, W = np.polynomial.legendre.leggauss(n_omega)
    omega = (1.0 + x) / (1.0 - x)
    weight = W * 2.0 / (1.0 - x) ** 2
    return omega, weight


# -----------------------------------------------------------------------------
# Coarse grid and interpolation (section "Interpolating Diagonal Entries")
# -----------------------------------------------------------------------------

def coarse_index_set(n, g: int) -> np.ndarray:
    """C_g: flat indices whose three grid indices are multiples of g (R10)."""
    idx = []
    for i in range(0, n[0], g):
        for j in range(0, n[1], g):
            for k in range(0, n[2], g):
                idx.append((i * n[1] + j) * n[2] + k)
    return np.array(idx, dtype=np.int64)


def interpolation_matrix_1d(n_fine: int, g: int, kind: str) -> np.ndarray:
    """(n_fine x n_coarse) periodic 1D interpolation matrix for one axis."""
    nc = n_fine // g
    M = np.zeros((n_fine, nc))
    if kind == "none" or g == 1:
        if g != 1:
            raise ValueError("no interpolation requires g = 1")
        return np.eye(n_fine)
    for i in range(n_fine):
        c, t = divmod(i, g)
        t = t / g
        if kind == "trilinear":
            M[i, c % nc] += 1.0 - t
            M[i, (c + 1) % nc] += t
        elif kind == "tricubic":
            # Lagrange basis on the nodes -1, 0, 1, 2 (R11)
            nodes = (-1.0, 0.0, 1.0, 2.0)
            for a, xa in enumerate(nodes):
                la = 1.0
                for b, xb in enumerate(nodes):
                    if b != a:
                        la *= (t - xb) / (xa - xb)
                M[i, (c - 1 + a) % nc] += la
        elif kind == "fourier":
            pass
        else:
            raise ValueError(kind)
    if kind == "fourier":
        for c in range(nc):
            e = np.zeros(nc)
            e[c] = 1.0
            M[:, c] = _fourier_upsample_1d(e, n_fine)
    return M


def _fourier_upsample_1d(v: np.ndarray, n_fine: int) -> np.ndarray:
    """FFT, zero-pad the spectrum to n_fine, inverse FFT (R12)."""
    nc = v.size
    C = np.fft.fft(v)
    F = np.zeros(n_fine, dtype=np.complex128)
    half = nc // 2
    if nc % 2 == 1:
        F[: half + 1] = C[: half + 1]
        F[n_fine - half:] = C[half + 1:]
    else:
        F[:half] = C[:half]
        F[n_fine - half + 1:] = C[half + 1:]
        F[half] = 0.5 * C[half]
        F[n_fine - half] = 0.5 * C[half]
    return np.fft.ifft(F).real * (n_fine / nc)


def interpolate(coarse: np.ndarray, n, g: int, kind: str) -> np.ndarray:
    """d_hat = I_g(d_Cg): tensor-product of the three 1D interpolants."""
    nc = tuple(n[d] // g for d in range(3))
    C = np.asarray(coarse, dtype=np.float64).reshape(nc)
    if g == 1:
        return C.reshape(-1).copy()
    Mx, My, Mz = (interpolation_matrix_1d(n[d], g, kind) for d in range(3))
    return np.einsum("ia,jb,kc,abc->ijk", Mx, My, Mz, C, optimize=True).reshape(-1)


def correlation_energy_from_coarse(d_coarse: np.ndarray, weight: np.ndarray, n, g: int, kind: str, dV: float):
    """E_c^(g) = 1/(2 pi) sum_k w_k sum_j d_hat_j(omega_k) and
    e(r) = 1/(2 pi) sum_k w_k d_hat(omega_k)(r) / h^3."""
    e_c = 0.0
    e_fine = np.zeros(int(np.prod(n)))
    for k in range(d_coarse.shape[0]):
        dh = interpolate(d_coarse[k], n, g, kind)
        e_c += weight[k] * float(np.sum(dh))
        e_fine += weight[k] * dh
    return e_c / (2.0 * math.pi), e_fine / (2.0 * math.pi * dV)


def interp_metrics(d_direct: np.ndarray, d_interp: np.ndarray, n_atoms: int = 1):
    """|Delta E|, L1 and ECR of the section "Error Metrics" (per atom)."""
    delta = np.asarray(d_direct) - np.asarray(d_interp)
    dE = abs(float(np.sum(delta))) / n_atoms
    l1 = float(np.sum(np.abs(delta))) / n_atoms
    return dE, l1, (dE / l1 if l1 > 0 else 0.0)


# -----------------------------------------------------------------------------
# Algorithm 1 over a set of points and frequencies
# -----------------------------------------------------------------------------

def energy_density(ham: Hamiltonian, coul: Coulomb, psi, eps, omegas, points, n_lanczos: int,
                   tol: float = 1e-10, maxit: int = 20000, exact: bool = False, stats: dict | None = None,
                   breakdown_rel: float = 1e-13, precond=None, v_loc=None):
    """d[k, p] = [f(T_m)]_11 from q_1 = e_{points[p]} at omega_k (Algorithm 1);
    breakdown_rel is the truncation threshold of reading R7; `precond` (with
    v_loc) preconditions the Sternheimer solves (reading R17)."""
    d = np.zeros((len(omegas), len(points)))
    for k, w in enumerate(omegas):
        A = nuhalf_chi0_nuhalf(ham, coul, psi, eps, w, tol=tol, maxit=maxit, exact=exact, stats=stats,
                               precond=precond, v_loc=v_loc)
        for p, j in enumerate(points):
            q1 = np.zeros(ham.N)
            q1[j] = 1.0
            a, b, broke = lanczos_tridiag(A, q1, n_lanczos, breakdown_rel=breakdown_rel)
            if stats is not None:
                stats.setdefault("lanczos_len", []).append(len(a))
                if broke:
                    stats.setdefault("breakdowns", []).append((k, p))
            d[k, p] = tridiag_quadrature(a, b)
    return d


# -----------------------------------------------------------------------------
# Next steps named in Conclusions and Future Work: preconditioned Sternheimer
# solves and block Lanczos quadrature.  The paper names both without details;
# the readings taken are R17 and R18 in the module docstring.
# -----------------------------------------------------------------------------

class KineticPreconditioner:
    """M^-1 for the shifted kinetic operator M = -1/2 Lap_h + sigma (R17).

    Lap_h is the FD Laplacian of H, diagonalised axis by axis (numpy eigh of
    each periodic 1D D2, as for the Coulomb operator), so
    M^-1 = (V_x (x) V_y (x) V_z) diag(1 / (kin + sigma)) (V_x (x) V_y (x) V_z)^T
    with kin = -1/2 (lam_x + lam_y + lam_z) >= 0.  For complex sigma with a
    positive real part it is complex symmetric and nonsingular, which COCG
    needs.
    """

    def __init__(self, n, L, radius: int = 6):
        self.n = tuple(n)
        self.V = []
        lams = []
        for d in range(3):
            lam, V = np.linalg.eigh(d2_periodic_1d(n[d], L[d] / n[d], radius))
            self.V.append(V)
            lams.append(lam)
        self.kin = -0.5 * (lams[0][:, None, None] + lams[1][None, :, None] + lams[2][None, None, :])

    def apply(self, r, sigma):
        if not complex(sigma).real > 0.0:
            raise ValueError("the kinetic preconditioner needs Re(sigma) > 0")
        R = np.asarray(r).reshape(self.n)
        Vx, Vy, Vz = self.V
        C = np.einsum("ia,jb,kc,ijk->abc", Vx, Vy, Vz, R, optimize=True)
        C = C / (self.kin + sigma)
        return np.einsum("ia,jb,kc,abc->ijk", Vx, Vy, Vz, C, optimize=True).reshape(-1)


def kinetic_shift(v_loc: np.ndarray, eps_n: float, omega: float, floor: float = 0.25) -> complex:
    """sigma_n of the kinetic preconditioner (R17): max(mean(V_loc) - eps_n, floor) - i omega.

    M then equals H - eps_n - i omega with the potential replaced by its mean;
    the real part is clipped from below so that M stays well away from
    singular for orbitals above the mean potential.
    """
    return complex(max(float(np.mean(v_loc)) - float(eps_n), float(floor)), -float(omega))


def cocg_precond(apply_A, apply_Minv, b: np.ndarray, x0: np.ndarray, tol: float, maxit: int):
    """COCG with a complex symmetric preconditioner M (R17).

    z = M^-1 r, rho = r^T z, p = z + (rho'/rho) p; the stopping rule R8 stays
    on the unpreconditioned residual.  With M = I every iterate equals that of
    cocg.  Returns (x, iterations, status).
    """
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b, dtype=np.complex128), 0, "ok"
    x = np.array(x0, dtype=np.complex128)
    r = b - apply_A(x)
    if np.linalg.norm(r) <= tol * bnorm:
        return x, 0, "ok"
    z = apply_Minv(r)
    p = z.copy()
    rho = r @ z
    for it in range(1, maxit + 1):
        q = apply_A(p)
        mu = p @ q
        if abs(mu) < 1e-300:
            return x, it, "breakdown"
        alpha = rho / mu
        x = x + alpha * p
        r = r - alpha * q
        if np.linalg.norm(r) <= tol * bnorm:
            return x, it, "ok"
        z = apply_Minv(r)
        rho_new = r @ z
        if abs(rho_new) < 1e-300:
            return x, it, "breakdown"
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, maxit, "noconv"


def block_cocg(apply_A, B: np.ndarray, X0: np.ndarray, tol: float, maxit: int):
    """Block COCG for s right-hand sides of one complex symmetric A (an
    extension for comparison, not in the paper; reading R19).

    O'Leary's block conjugate gradient with unconjugated transposes:
    R = B - A X, P = R; per iteration Q = A P, alpha = (P^T Q)^-1 (R^T R),
    X += P alpha, R -= Q alpha, beta = (R^T R)^-1 (R'^T R'), P = R' + P beta.
    Columns are N-vectors; stops when every column meets the stopping rule
    R8, ||b_j - A x_j|| <= tol ||b_j|| on the recursive residual.  With s = 1
    every iterate equals that of cocg.  Returns (X, iterations, status).
    """
    Bm = np.asarray(B, dtype=np.complex128)
    bn = np.linalg.norm(Bm, axis=0)
    X = np.array(X0, dtype=np.complex128)
    R = Bm - np.stack([apply_A(X[:, j]) for j in range(X.shape[1])], axis=1)
    if np.all(np.linalg.norm(R, axis=0) <= tol * bn):
        return X, 0, "ok"
    P = R.copy()
    rho = R.T @ R
    for it in range(1, maxit + 1):
        Q = np.stack([apply_A(P[:, j]) for j in range(P.shape[1])], axis=1)
        mu = P.T @ Q
        try:
            alpha = np.linalg.solve(mu, rho)
        except np.linalg.LinAlgError:
            return X, it, "breakdown"
        X = X + P @ alpha
        R = R - Q @ alpha
        if np.all(np.linalg.norm(R, axis=0) <= tol * bn):
            return X, it, "ok"
        rho_new = R.T @ R
        try:
            beta = np.linalg.solve(rho, rho_new)
        except np.linalg.LinAlgError:
            return X, it, "breakdown"
        if not np.all(np.isfinite(beta)):
            return X, it, "breakdown"
        P = R + P @ beta
        rho = rho_new
    return X, maxit, "noconv"


def block_lanczos(apply_A, Q1: np.ndarray, m: int, breakdown_rel: float = 1e-13):
    """m block Lanczos steps on symmetric A from orthonormal columns Q1 (R18).

    Block three-term recurrence A Q_k = Q_{k-1} B_{k-1}^T + Q_k A_k + Q_{k+1} B_k
    with A_k = Q_k^T A Q_k (symmetrised) and Q_{k+1} B_k the thin QR of the
    remainder, after two classical Gram-Schmidt passes against every stored
    block.  Stops early (broke = True) when a diagonal entry of B_k is at most
    breakdown_rel times the largest |A_k| entry.  apply_A maps N x b to N x b.
    Returns (list of A_k, list of B_k, broke); len(B) = len(A) - 1.
    """
    Q = [np.array(Q1, dtype=np.float64)]
    b = Q[0].shape[1]
    A_blocks, B_blocks = [], []
    Q_prev = np.zeros_like(Q[0])
    B_prev = np.zeros((b, b))
    broke = False
    for k in range(m):
        W = apply_A(Q[k])
        Ak = Q[k].T @ W
        Ak = 0.5 * (Ak + Ak.T)
        W = W - Q[k] @ Ak - Q_prev @ B_prev.T
        Qall = np.hstack(Q)
        for _ in range(2):
            W = W - Qall @ (Qall.T @ W)
        A_blocks.append(Ak)
        if k < m - 1:
            Qn, R = np.linalg.qr(W)
            scale = max(float(np.abs(a).max()) for a in A_blocks)
            if float(np.abs(np.diag(R)).min()) <= breakdown_rel * scale:
                broke = True
                break
            B_blocks.append(R)
            Q_prev, B_prev = Q[k], R
            Q.append(Qn)
    return A_blocks, B_blocks, broke


def block_tridiag(A_blocks, B_blocks) -> np.ndarray:
    """Dense block tridiagonal T: diagonal A_k, below B_k, above B_k^T."""
    b = A_blocks[0].shape[0]
    k = len(A_blocks)
    T = np.zeros((k * b, k * b))
    for i, Ai in enumerate(A_blocks):
        T[i * b:(i + 1) * b, i * b:(i + 1) * b] = Ai
    for i, Bi in enumerate(B_blocks):
        T[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = Bi
        T[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = Bi.T
    return T


def block_quadrature(A_blocks, B_blocks) -> np.ndarray:
    """diag(E_1^T f(T) E_1): the block Gauss estimate of e_j^T f(A) e_j (R18)."""
    b = A_blocks[0].shape[0]
    lam, U = np.linalg.eigh(block_tridiag(A_blocks, B_blocks))
    return (U[:b, :] ** 2) @ f_rpa(lam)


def energy_density_block(ham: Hamiltonian, coul: Coulomb, psi, eps, omegas, points, n_lanczos: int,
                         block: int, tol: float = 1e-10, maxit: int = 20000, exact: bool = False,
                         stats: dict | None = None):
    """d[k, p] by block Lanczos quadrature over consecutive groups of `block` points (R18).

    The start block of a group is [e_j for j in the group]; the last group may
    be smaller.  block = 1 is the scalar quadrature of energy_density.
    """
    if block < 1:
        raise ValueError("block must be >= 1")
    points = list(points)
    d = np.zeros((len(omegas), len(points)))
    for k, w in enumerate(omegas):
        A = nuhalf_chi0_nuhalf(ham, coul, psi, eps, w, tol=tol, maxit=maxit, exact=exact, stats=stats)
        apply_block = lambda X, A=A: np.stack([A(X[:, c]) for c in range(X.shape[1])], axis=1)
        for g0 in range(0, len(points), block):
            grp = points[g0:g0 + block]
            Q1 = np.zeros((ham.N, len(grp)))
            Q1[grp, np.arange(len(grp))] = 1.0
            Ab, Bb, broke = block_lanczos(apply_block, Q1, n_lanczos)
            if stats is not None and broke:
                stats.setdefault("breakdowns", []).append((k, g0))
            d[k, g0:g0 + len(grp)] = block_quadrature(Ab, Bb)
    return d
