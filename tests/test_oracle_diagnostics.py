"""Pins of the oracle's diagnostics (oracle/diagnostics.py) against things
other than its own code: scipy's matrix logarithm, Klein's inequality,
the closed-form entropy of a Fermi-Dirac state, recovery of known
Fermi-Dirac parameters, the entropy-production density as the time
derivative of the entropy under dW/dt = C[W] (mathematics: the derivative
of tr[W log W + W~ log W~] is log W - log W~), the chain rule of relative
entropy quoted in Sec. 5, and unitary invariance."""
import numpy as np
import pytest
from scipy.linalg import logm

import workloads as wl
from oracle import collision as oc
from oracle import diagnostics as dg
from oracle import pauli
from oracle.fermi_dirac import fd_matrix, polylog2

L = 12.0


def _grid(N):
    h = 2 * L / N
    v = h * (np.arange(N) - N // 2)
    return h, np.meshgrid(v, v, indexing="ij")


def _haar(rng):
    Z = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    Q, R = np.linalg.qr(Z)
    return Q * (np.diag(R) / np.abs(np.diag(R)))


def _random_states(rng, shape, lo=0.05, hi=0.95):
    out = np.zeros(shape + (2, 2), np.complex128)
    for idx in np.ndindex(*shape):
        U = _haar(rng)
        out[idx] = U @ np.diag(rng.uniform(lo, hi, 2)) @ U.conj().T
    return out


def test_entropy_and_relative_entropy_match_scipy_logm():
    rng = np.random.default_rng(0)
    N = 4
    h, _ = _grid(N)
    W = _random_states(rng, (2, N, N))
    F = _random_states(rng, (2, N, N))
    I = np.eye(2)
    S = np.zeros(2)
    R = np.zeros(2)
    for c in range(2):
        for i in range(N):
            for j in range(N):
                w, f = W[c, i, j], F[c, i, j]
                S[c] -= np.trace(w @ logm(w) + (I - w) @ logm(I - w)).real
                R[c] += np.trace(w @ (logm(w) - logm(f)) + (I - w) @ (logm(I - w) - logm(I - f))).real
    assert np.allclose(dg.entropy(W, L), h * h * S, rtol=1e-12, atol=0)
    assert np.allclose(dg.relative_entropy(W, F, L), h * h * R, rtol=1e-10, atol=0)


def test_relative_entropy_klein_inequality_and_zero():
    rng = np.random.default_rng(1)
    W = _random_states(rng, (3, 8, 8), 0.01, 0.99)
    F = _random_states(rng, (3, 8, 8), 0.01, 0.99)
    assert (dg.relative_entropy(W, F, L) > 0).all()
    assert np.abs(dg.relative_entropy(W, W, L)).max() < 1e-12


def test_entropy_is_basis_invariant():
    rng = np.random.default_rng(2)
    W = _random_states(rng, (2, 8, 8))
    F = _random_states(rng, (2, 8, 8))
    U = _haar(rng)
    Wr = U @ W @ U.conj().T
    Fr = U @ F @ U.conj().T
    assert np.allclose(dg.entropy(Wr, L), dg.entropy(W, L), rtol=1e-13)
    assert np.allclose(dg.relative_entropy(Wr, Fr, L), dg.relative_entropy(W, F, L), rtol=1e-11)


def test_entropy_of_fermi_dirac_state_matches_closed_form():
    """Per spin, the 2D Fermi-Dirac entropy with omega = |v|^2/2 is
    (2 E_s - mu_s N_s) / kT with N_s = 2 pi kT log(1 + z_s) and
    E_s = 2 pi kT^2 (-Li_2(-z_s)), z_s = e^{mu_s/kT} (grand potential
    -E_s in two dimensions); the grid sum is a trapezoid rule, exact to
    discretisation accuracy."""
    kT, mus = 1.0, (0.5, -0.5)
    N = 64
    _, (vx, vy) = _grid(N)
    W = fd_matrix(vx, vy, 1.0 / kT, mus[0], mus[1])[None]
    ref = 0.0
    for m in mus:
        z = np.exp(m / kT)
        Ns = 2 * np.pi * kT * np.log1p(z)
        Es = 2 * np.pi * kT**2 * (-polylog2(-z))
        ref += (2 * Es - m * Ns) / kT
    assert abs(dg.entropy(W, L)[0] - ref) < 1e-7 * ref


@pytest.mark.parametrize("N", [32, 64])
def test_fit_recovers_fermi_dirac_parameters(N):
    rng = np.random.default_rng(3)
    U = _haar(rng)
    kT, mu_up, mu_down, u = 1.25, 1.5, -1.5, (0.3, -0.2)
    _, (vx, vy) = _grid(N)
    W = fd_matrix(vx, vy, 1.0 / kT, mu_up, mu_down, U, u)[None]
    fit = dg.fit_local_fd(W, L)
    tol = 1e-5 if N == 32 else 1e-9
    assert abs(fit["kT"][0] - kT) < tol
    assert abs(fit["mu_up"][0] - mu_up) < 4 * tol and abs(fit["mu_down"][0] - mu_down) < 4 * tol
    assert abs(fit["ux"][0] - u[0]) < tol and abs(fit["uy"][0] - u[1]) < tol
    overlap = np.abs(fit["U"][0].conj().T @ U)
    assert np.allclose(overlap, np.eye(2), atol=1e-9)
    d = dg.diagnostics(W, L)
    assert -1e-13 <= d[0, 3] < 1e-3 * tol


def test_fit_without_solution_gives_nan():
    N = 16
    W = np.zeros((2, N, N, 2, 2), np.complex128)
    W[0, ..., 0, 0] = 0.5  # spin-down density zero: no Fermi-Dirac state
    W[1] = 0.5 * np.eye(2)  # uniform on the box: a hot, solvable state
    fit = dg.fit_local_fd(W, L)
    assert np.isnan(fit["kT"][0]) and np.isnan(fit["mu_up"][0])
    assert np.isfinite(fit["kT"][1])


def test_entropy_production_is_the_entropy_rate():
    """sigma(x) = d/dtau S[W + tau C](x) at tau = 0 (Richardson central
    differences), C = C[W] from the oracle collision."""
    N, J, M = 8, 4, 4
    w = wl.config(1, Nx=2, N=N)
    W = w.W0
    t = oc.Tables(N, w.L, w.R, J, M)
    C = np.stack([oc.collision(W[c], w.L, w.R, J, M, t) for c in range(2)])
    sig = dg.entropy_production(W, C, w.L)
    D = lambda s: (dg.entropy(W + s * C, w.L) - dg.entropy(W - s * C, w.L)) / (2 * s)
    s0 = 1e-4 / np.abs(C).max()  # keeps every eigenvalue of W +- s C inside (0, 1)
    rate = (4 * D(s0 / 2) - D(s0)) / 3
    assert np.allclose(sig, rate, rtol=1e-7, atol=0)
    assert (np.abs(sig) > 0).all()


def test_relative_entropy_chain_rule_through_local_fit():
    """S(W || F) = S(W || G) + S(G || F) for G the local Fermi-Dirac fit
    (Sec. 5); on the grid it holds to the accuracy with which the fit
    matches the discrete moments."""
    w = wl.config(2, Nx=3)
    W = w.W0
    U = np.eye(2)
    F = np.broadcast_to(fd_matrix(*_grid(w.N)[1], 1.0, 0.0, 0.0, U), W.shape)
    fit = dg.fit_local_fd(W, w.L)
    G = dg.fd_field(w.N, w.L, fit["kT"], fit["mu_up"], fit["mu_down"], fit["U"], fit["ux"], fit["uy"])
    lhs = dg.relative_entropy(W, F, w.L)
    rhs = dg.relative_entropy(W, G, w.L) + dg.relative_entropy(G, F, w.L)
    assert np.allclose(lhs, rhs, rtol=1e-4, atol=0)


def test_diagnostics_fields_of_configuration_states():
    """Eigenvalues inside [0, 1] for the generated states, and the field
    layout of diagnostics()."""
    w = wl.config(1, Nx=2)
    d = dg.diagnostics(w.W0, w.L)
    assert d.shape == (2, dg.NFIELDS)
    assert (d[:, 4] >= 0.05 - 1e-12).all() and (d[:, 5] <= 0.95 + 1e-12).all()
    lam = np.linalg.eigvalsh(w.W0)
    assert np.allclose(d[:, 4], lam.min(axis=(1, 2, 3))) and np.allclose(d[:, 5], lam.max(axis=(1, 2, 3)))
    assert (d[:, 0] > 0).all() and (d[:, 3] > 0).all()
    assert np.all(d[:, 1] == 0) and np.all(d[:, 2] == 0)
    wp = pauli.to_pauli(w.W0)
    n = 2 * (2 * w.L / w.N) ** 2 * wp[..., 0].sum(axis=(1, 2))
    assert np.all(n > 0)
