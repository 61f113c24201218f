"""Diagnostics of a Wigner state (Sec. 2 and Sec. 5): local entropy
(eq. entropy_def), the entropy production density of the H-theorem, the
quantum relative entropy to a Fermi-Dirac state (eq. relentropy_hom, per
cell; eq. relentropy_inhom and relentropy_local are their x-integrals),
the eigenvalue range, and the local Fermi-Dirac fit (temperature and
chemical potentials matched to the eigenvalues of the spin density and to
the internal energy through eq. momentsFermiDirac, velocity shift from
eq. velocity, spin basis = eigenbasis of the spin density).

Written with 2x2 matrix functions from numpy's Hermitian eigensolver and
scipy's root finder, point by point.

Reading: matrix logarithms are taken with every eigenvalue clamped into
[0, 1] and log(x) read as log(max(x, 1e-300)), so that 0 log 0 = 0 and a
state with an eigenvalue at 0 or 1 still gives finite values.
"""
import numpy as np
from scipy.optimize import brentq

from .fermi_dirac import fd_matrix, polylog2
from .pauli import SIGMA, to_pauli
from .step import moments

TINY = 1e-300


def _log(x):
    return np.log(np.maximum(x, TINY))


def _eig(W):
    lam, V = np.linalg.eigh(np.asarray(W, np.complex128))
    return np.clip(lam, 0.0, 1.0), V


def _fn(W, f):
    """f(W) for Hermitian W[..., 2, 2] through its eigendecomposition."""
    lam, V = _eig(W)
    return np.einsum("...ij,...j,...kj->...ik", V, f(lam), V.conj())


def _tr(A, B):
    return np.einsum("...ij,...ji->...", A, B).real


def _velocity(N, L):
    h = 2.0 * L / N
    v = h * (np.arange(N) - N // 2)
    return h, np.meshgrid(v, v, indexing="ij")


def entropy(W, L):
    """S[W](x) = -h^2 sum_v tr[W log W + (1 - W) log(1 - W)]
    (eq. entropy_def) for W[Nx, N, N, 2, 2]; returns [Nx]."""
    h, _ = _velocity(W.shape[1], L)
    lam, _ = _eig(W)
    s = lam * _log(lam) + (1.0 - lam) * _log(1.0 - lam)
    return -h * h * s.sum(axis=(1, 2, 3))


def entropy_production(W, C, L):
    """sigma(x) = -h^2 sum_v tr[(log W - log(1 - W)) C[W]] (the H-theorem's
    integrand over v); its x-integral is d/dt of the total entropy."""
    h, _ = _velocity(W.shape[1], L)
    G = _fn(W, lambda l: _log(l) - _log(1.0 - l))
    return -h * h * _tr(G, np.asarray(C, np.complex128)).sum(axis=(1, 2))


def relative_entropy(W, F, L):
    """S(W || F)(x) = h^2 sum_v tr[W (log W - log F) + W~ (log W~ - log F~)]
    with W~ = 1 - W (eq. relentropy_hom) for states W, F[Nx, N, N, 2, 2]."""
    h, _ = _velocity(W.shape[1], L)
    I = np.eye(2)
    Wt = I - W
    Ft = I - F
    a = _tr(W, _fn(W, _log) - _fn(F, _log))
    b = _tr(Wt, _fn(Wt, _log) - _fn(Ft, _log))
    return h * h * (a + b).sum(axis=(1, 2))


def eigen_range(W):
    """Smallest and largest eigenvalue of W(v) per cell (Sec. 5), unclamped."""
    lam = np.linalg.eigvalsh(np.asarray(W, np.complex128))
    return lam.min(axis=(1, 2, 3)), lam.max(axis=(1, 2, 3))


def _fd_eps(kT, rho_s):
    """Internal energy per particle of the Fermi-Dirac state whose per-spin
    densities are rho_s at temperature kT (eq. momentsFermiDirac, with the
    chemical potentials from inverting its density formula)."""
    z = np.expm1(np.asarray(rho_s) / (2.0 * np.pi * kT))  # e^{mu_s/kT}
    mus = kT * np.log(z)
    num = -sum(polylog2(-zz) for zz in z)
    den = sum(np.log1p(zz) for zz in z)
    return kT * num / den, mus


def fit_local_fd(W, L):
    """Per cell: the Fermi-Dirac state with the same spin density matrix,
    momentum and energy as W (Sec. 5).  Returns a dict of arrays [Nx]:
    kT, mu_up, mu_down, ux, uy, and U[Nx, 2, 2] (columns: spin up, down =
    eigenvectors of rho for its larger and smaller eigenvalue).  kT and the
    mu are NaN where no such state is found: an eigenvalue of rho <= 0, or
    a temperature below rho_up / (1200 pi) (where e^{rho_s / (2 pi kT)}
    leaves the float64 range; this includes energies at or below the
    zero-temperature limit).

    The temperature solves eps_FD(kT) = eps; eps_FD(kT) >= kT for fermions
    (the classical value kT is a lower bound), so the root lies in
    [rho_up / (1200 pi), eps]."""
    mom = moments(to_pauli(W), L)
    Nx = W.shape[0]
    out = {k: np.full(Nx, np.nan) for k in ("kT", "mu_up", "mu_down")}
    n = 2.0 * mom[:, 0]
    out["ux"] = mom[:, 4] / n
    out["uy"] = mom[:, 5] / n
    out["U"] = np.zeros((Nx, 2, 2), np.complex128)
    for c in range(Nx):
        rho = np.einsum("m,mab->ab", mom[c, :4].astype(np.complex128), SIGMA)
        lam, V = np.linalg.eigh(rho)
        out["U"][c] = V[:, ::-1]
        rs = lam[::-1]  # (up, down) = (larger, smaller)
        eps = mom[c, 6] / n[c] - 0.5 * (out["ux"][c] ** 2 + out["uy"][c] ** 2)
        if rs[1] <= 0.0 or not eps > 0.0:
            continue
        g = lambda lt: _fd_eps(np.exp(lt), rs)[0] - eps
        lo, hi = np.log(rs[0] / (1200.0 * np.pi)), np.log(eps)
        if not (lo < hi and g(lo) < 0.0):
            continue
        if g(hi) <= 0.0:
            lt = hi
        else:
            lt = brentq(g, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
        kT = np.exp(lt)
        _, mus = _fd_eps(kT, rs)
        out["kT"][c], out["mu_up"][c], out["mu_down"][c] = kT, mus[0], mus[1]
    return out


def fd_field(N, L, kT, mu_up, mu_down, U, ux, uy):
    """W_FD(v - u) on the velocity grid for each cell (eq. W_FermiDirac with
    the velocity shift of Sec. 5); NaN parameters give a NaN field."""
    _, (vx, vy) = _velocity(N, L)
    return np.stack([fd_matrix(vx, vy, 1.0 / kT[c], mu_up[c], mu_down[c], U[c], (ux[c], uy[c]))
                     for c in range(len(kT))])


NFIELDS = 11


def diagnostics(W, L, C=None, fd=None):
    """All diagnostics per cell, float64 [Nx, 11]:
    0 entropy, 1 entropy production density (0 without C), 2 relative
    entropy to the global Fermi-Dirac state fd = (inv_kT, mu_up, mu_down, U)
    at zero velocity (0 without fd), 3 relative entropy to the local fit,
    4 smallest and 5 largest eigenvalue, 6 kT, 7 mu_up, 8 mu_down, 9 u_x,
    10 u_y of the local fit."""
    W = np.asarray(W, np.complex128)
    Nx, N = W.shape[0], W.shape[1]
    out = np.zeros((Nx, NFIELDS))
    out[:, 0] = entropy(W, L)
    if C is not None:
        out[:, 1] = entropy_production(W, C, L)
    _, (vx, vy) = _velocity(N, L)
    if fd is not None:
        inv_kT, mu_up, mu_down, U = fd
        F = np.broadcast_to(fd_matrix(vx, vy, inv_kT, mu_up, mu_down, U), W.shape)
        out[:, 2] = relative_entropy(W, F, L)
    fit = fit_local_fd(W, L)
    ok = np.isfinite(fit["kT"])
    out[:, 3] = np.nan
    if ok.any():
        G = fd_field(N, L, fit["kT"][ok], fit["mu_up"][ok], fit["mu_down"][ok], fit["U"][ok],
                     fit["ux"][ok], fit["uy"][ok])
        out[ok, 3] = relative_entropy(W[ok], G, L)
    out[:, 4], out[:, 5] = eigen_range(W)
    out[:, 6], out[:, 7], out[:, 8] = fit["kT"], fit["mu_up"], fit["mu_down"]
    out[:, 9], out[:, 10] = fit["ux"], fit["uy"]
    return out
