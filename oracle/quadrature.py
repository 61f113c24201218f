"""Kernel quadratures of the fast spectral method (Sec. 3.2).

* theta_j = exp(i (j-1) pi / J), theta'_j = exp(i (j-1/2) pi / J),
  j = 1..J (eq. theta_grid), returned as unit vectors in R^2.
* phi_R(x) = int_0^R sin(pi x r / L) dr  (the radial factor of G).
  Reading: the paper prints the antiderivative with the sign flipped;
  integrating directly gives +(2L / (pi x)) sin^2(pi R x / (2L)).  G holds
  phi_R twice, so the sign does not change G.  phi_R(0) = 0 (limit).
* psi_R(x) = int_{-R}^{R} exp(i pi x r / L) dr = (2L / (pi x)) sin(pi R x / L)
  (eq. approxH-J), with the limit psi_R(0) = 2R.  Reading: the paper's psi'
  shows xi in the denominator and in the sine; psi'_j(chi) is
  psi_R(chi . R_{pi/2} theta_j), i.e. the same function of the rotated
  projection.
* omega_{G,j,j'} = -(2 pi / J)^2 / (theta_j . theta'_j') (eq. approxG).
* omega_{H,j} = pi / J (eq. approxH-J).
* (rho_{R,m}, w_{R,m}): Gauss-Legendre nodes and weights on [-R, R]
  (eq. approxH-JM).
"""
import numpy as np


def theta(J):
    """Unit vectors theta_j, j = 1..J, at angles (j-1) pi / J; shape [J, 2]."""
    a = np.arange(J) * np.pi / J
    return np.stack([np.cos(a), np.sin(a)], axis=-1)


def theta_prime(J):
    """Unit vectors theta'_j at angles (j-1/2) pi / J; shape [J, 2]."""
    a = (np.arange(J) + 0.5) * np.pi / J
    return np.stack([np.cos(a), np.sin(a)], axis=-1)


def rot90(t):
    """R_{pi/2} applied to unit vectors t[..., 2]."""
    return np.stack([-t[..., 1], t[..., 0]], axis=-1)


def phi_R(x, L, R):
    """int_0^R sin(pi x r / L) dr, elementwise; 0 at x = 0."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0.0
    xs = x[nz]
    out[nz] = (2.0 * L / (np.pi * xs)) * np.sin(np.pi * R * xs / (2.0 * L)) ** 2
    return out


def psi_R(x, L, R):
    """int_{-R}^{R} exp(i pi x r / L) dr, elementwise; 2R at x = 0."""
    x = np.asarray(x, dtype=np.float64)
    out = np.full_like(x, 2.0 * R)
    nz = x != 0.0
    xs = x[nz]
    out[nz] = (2.0 * L / (np.pi * xs)) * np.sin(np.pi * R * xs / L)
    return out


def omega_G(J):
    """omega_{G,j,j'} = -(2 pi / J)^2 / (theta_j . theta'_j'), shape [J, J].

    Requires even J: for odd J some theta_j is orthogonal to some theta'_j'.
    """
    if J % 2:
        raise ValueError("J must be even")
    dots = theta(J) @ theta_prime(J).T
    return -((2.0 * np.pi / J) ** 2) / dots


def omega_H(J):
    """omega_{H,j} = pi / J."""
    return np.full(J, np.pi / J)


def gauss_legendre(M, R):
    """Gauss-Legendre nodes rho_m and weights w_m on [-R, R] (M points)."""
    x, w = np.polynomial.legendre.leggauss(M)
    return R * x, R * w
