"""Error bounds that turn measured residuals of Sternheimer solutions into
bounds on their errors (test infrastructure)."""
import numpy as np


def residual_error_bound(ham, psi, eps, u, omega, x):
    """True residuals of the solutions x[n] of (H - eps_n - i omega) x = -psi_n u,
    and the bound they give on the error of chi0 u = 4 sum_n psi_n Re x_n.

    H is real symmetric, so A_n = H - eps_n - i omega is normal with
    eigenvalues lambda - eps_n - i omega, all of modulus >= omega: hence
    ||x_n - x_n*||_2 <= ||r_n||_2 / omega, and elementwise
    |d(chi0 u)| <= 4 sum_n ||psi_n||_inf ||x_n - x_n*||_2."""
    r, b = [], []
    for n in range(psi.shape[0]):
        bn = -psi[n] * u
        z = eps[n] + 1j * omega
        r.append(np.linalg.norm(bn - (ham.apply(x[n]) - z * x[n])))
        b.append(np.linalg.norm(bn))
    r, b = np.array(r), np.array(b)
    bound = 4.0 * float(np.sum(np.abs(psi).max(axis=1) * r)) / omega
    return r, b, bound
