"""Fermi-Dirac states (eq. W_FermiDirac) and their closed-form moments
(eq. momentsFermiDirac), for omega(v) = |v|^2 / 2 in two velocity
dimensions.
"""
import numpy as np
from scipy.special import spence


def fd_matrix(vx, vy, inv_kT, mu_up, mu_down, U=None, v0=(0.0, 0.0)):
    """W_FD(v) = U diag(f_up, f_down) U^H with f_s = 1/(exp((omega - mu_s)/kT) + 1),
    omega = |v - v0|^2 / 2; U holds the spin basis as columns (Table 1).
    vx, vy broadcast; returns [..., 2, 2] complex."""
    U = np.eye(2, dtype=np.complex128) if U is None else np.asarray(U, np.complex128)
    om = 0.5 * ((vx - v0[0]) ** 2 + (vy - v0[1]) ** 2)
    f_up = 1.0 / (np.exp((om - mu_up) * inv_kT) + 1.0)
    f_dn = 1.0 / (np.exp((om - mu_down) * inv_kT) + 1.0)
    D = np.zeros(np.shape(om) + (2, 2), dtype=np.complex128)
    D[..., 0, 0] = f_up
    D[..., 1, 1] = f_dn
    return U @ D @ U.conj().T


def fd_density(inv_kT, mus):
    """tr rho_FD = 2 pi kT sum_s log(1 + e^{mu_s/kT}) (eq. momentsFermiDirac)."""
    kT = 1.0 / inv_kT
    return 2.0 * np.pi * kT * sum(np.log1p(np.exp(m / kT)) for m in mus)


def polylog2(z):
    """Li_2(z) for real z <= 1 via Spence's function: Li_2(z) = spence(1 - z)."""
    return spence(1.0 - z)


def fd_energy(inv_kT, mus):
    """epsilon_FD = kT (-sum_s Li_2(-e^{mu_s/kT})) / sum_s log(1 + e^{mu_s/kT})
    (eq. momentsFermiDirac); tr(rho) epsilon is the energy density."""
    kT = 1.0 / inv_kT
    num = -sum(polylog2(-np.exp(m / kT)) for m in mus)
    den = sum(np.log1p(np.exp(m / kT)) for m in mus)
    return kT * num / den
