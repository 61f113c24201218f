"""Pins of the oracle's reverse-mode derivatives (oracle/adjoint.py) by
properties that do not involve the adjoint code itself:

* C[W] is a polynomial of degree three in the Pauli components (three
  factors of W, 1 - W or f0 per term, Sec. 3.2), so the central difference
  quotient D(h) = (C(w + h d) - C(w - h d)) / 2h equals C'(w)d + h^2 K and
  (4 D(1/2) - D(1)) / 3 is the exact directional derivative.  The adjoint
  must satisfy <lam, C'(w) d> = <C'(w)^T lam, d> to rounding.
* The transport step (eq. slopeLimiterStep with the minmod limiter) is
  linear on each branch of the limiter, so a small central difference is
  exact away from branch switches.
* The splitting step and the trajectory are smooth on a fixed limiter
  branch: Richardson-extrapolated central differences.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import adjoint as ad
from oracle import collision as oc
from oracle import pauli
from oracle import step as ostep
from oracle import transport as tp
from oracle.fermi_dirac import fd_matrix

L, R = 12.0, 7.5


def _fd_state(N, inv_kT, mu_up, mu_down):
    v = (2 * L / N) * (np.arange(N) - N // 2)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    return pauli.to_pauli(fd_matrix(vx, vy, inv_kT, mu_up, mu_down, np.eye(2)))


def _bcs(kind, N):
    if kind == "periodic":
        return {"kind": "periodic"}, {"kind": "periodic"}
    left = {"kind": "dirichlet", "state": _fd_state(N, 0.8, 1.5, -1.5), "alpha": 0.0}
    if kind == "dirichlet":
        return left, {"kind": "dirichlet", "state": _fd_state(N, 2.0, 0.0, 0.0), "alpha": 0.0}
    return left, {"kind": "maxwell", "state": _fd_state(N, 2.0, 0.0, 0.0), "alpha": 0.5}


def _rel(a, b):
    return abs(a - b) / max(abs(a), abs(b))


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("N,J,M", [(8, 4, 4), (8, 6, 3)])
def test_collision_vjp_exact_against_polynomial_jvp(seed, N, J, M):
    rng = np.random.default_rng(seed)
    t = oc.Tables(N, L, R, J, M)
    w = pauli.to_pauli(wl.config(1, Nx=1, N=N).W0)[0] + 0.05 * rng.standard_normal((N, N, 4))
    lam = rng.standard_normal(w.shape)
    d = 0.1 * rng.standard_normal(w.shape)
    C = lambda x: oc.collision_pauli(x, L, R, J, M, t)
    D = lambda h: (C(w + h * d) - C(w - h * d)) / (2 * h)
    jvp = (4 * D(0.5) - D(1.0)) / 3
    g = ad.collision_pauli_vjp(w, lam, L, R, J, M, t)
    assert _rel(np.sum(lam * jvp), np.sum(g * d)) < 1e-12


def test_collision_vjp_sees_every_component():
    """Each Pauli component of the cotangent reaches the gradient: the
    pairing holds for cotangents supported on one component at a time."""
    rng = np.random.default_rng(5)
    N, J, M = 8, 4, 4
    t = oc.Tables(N, L, R, J, M)
    w = pauli.to_pauli(wl.config(1, Nx=1, N=N).W0)[0]
    d = 0.1 * rng.standard_normal(w.shape)
    C = lambda x: oc.collision_pauli(x, L, R, J, M, t)
    D = lambda h: (C(w + h * d) - C(w - h * d)) / (2 * h)
    jvp = (4 * D(0.5) - D(1.0)) / 3
    for mu in range(4):
        lam = np.zeros(w.shape)
        lam[..., mu] = rng.standard_normal((N, N))
        g = ad.collision_pauli_vjp(w, lam, L, R, J, M, t)
        a = np.sum(lam * jvp)
        assert abs(a) > 1e-6
        assert _rel(a, np.sum(g * d)) < 1e-12


@pytest.mark.parametrize("kind", ["periodic", "dirichlet", "maxwell"])
def test_transport_vjp_matches_branchwise_difference(kind):
    rng = np.random.default_rng(3)
    Nx, N = 6, 8
    w = pauli.to_pauli(wl.config(3, Nx=Nx, N=N).W0) + 0.01 * rng.standard_normal((Nx, N, N, 4))
    bl, br = _bcs(kind, N)
    dt = 0.7 / (L * Nx)
    lam = rng.standard_normal(w.shape)
    d = rng.standard_normal(w.shape)
    h = 1e-6
    T = lambda x: tp.transport_step(x, dt, bl, br, L)
    fd = (T(w + h * d) - T(w - h * d)) / (2 * h)
    g = ad.transport_step_vjp(w, lam, dt, bl, br, L)
    assert _rel(np.sum(lam * fd), np.sum(g * d)) < 1e-9


def test_magnetic_vjp():
    rng = np.random.default_rng(4)
    w = rng.standard_normal((3, 4, 4, 4))
    B = rng.standard_normal((3, 3))
    lam = rng.standard_normal(w.shape)
    d, dB = rng.standard_normal(w.shape), rng.standard_normal(B.shape)
    gw, gB = ad.magnetic_vjp(w, B, lam)
    # bilinear in (B, w): exact derivatives
    assert _rel(np.sum(lam * ostep.magnetic(d, B)), np.sum(gw * d)) < 1e-13
    assert _rel(np.sum(lam * ostep.magnetic(w, dB)), np.sum(gB * dB)) < 1e-13


def _richardson(f, h):
    D = lambda s: (f(s) - f(-s)) / (2 * s)
    return (4 * D(h / 2) - D(h)) / 3


@pytest.mark.parametrize("kind", ["periodic", "maxwell"])
def test_step_vjp_state_and_field(kind):
    rng = np.random.default_rng(6)
    Nx, N, J, M = 4, 8, 4, 4
    t = oc.Tables(N, L, R, J, M)
    # O(0.1) noise keeps the limiter's differences far from zero, so the
    # difference quotients stay on one branch
    w = pauli.to_pauli(wl.config(2, Nx=Nx, N=N).W0) + 0.1 * rng.standard_normal((Nx, N, N, 4))
    B = rng.standard_normal((Nx, 3))
    bl, br = _bcs(kind, N)
    dt = 0.5 / (L * Nx)
    lam = rng.standard_normal(w.shape)
    d, dB = rng.standard_normal(w.shape), rng.standard_normal(B.shape)
    S = lambda x, b: ostep.step(x, b, dt, L, R, J, M, bl, br, t)
    gw, gB = ad.step_vjp(w, B, dt, lam, L, R, J, M, bl, br, t)
    jw = _richardson(lambda s: np.sum(lam * S(w + s * d, B)), 1e-5)
    jB = _richardson(lambda s: np.sum(lam * S(w, B + s * dB)), 1e-3)
    assert _rel(jw, np.sum(gw * d)) < 1e-8
    assert _rel(jB, np.sum(gB * dB)) < 1e-8


def test_trajectory_gradient_of_observable():
    """Gradient of dx h^2 sum g(x_j) tr(sigma_z W(T)) over 3 steps, in the
    initial state and the field, against differences of the forward run."""
    rng = np.random.default_rng(7)
    Nx, N, J, M, steps = 3, 8, 4, 4, 3
    t = oc.Tables(N, L, R, J, M)
    w0 = pauli.to_pauli(wl.config(2, Nx=Nx, N=N).W0) + 0.1 * rng.standard_normal((Nx, N, N, 4))
    B = np.tile([0.0, 0.0, 0.5], (Nx, 1)) + 0.1 * rng.standard_normal((Nx, 3))
    per = {"kind": "periodic"}
    dt = 1e-3
    g = wl.adjoint_loss_weight(Nx)
    lamT = ad.observable_weights(g, N, L)

    def loss(x, b):
        for _ in range(steps):
            x = ostep.step(x, b, dt, L, R, J, M, per, per, t)
        return np.sum(lamT * x)

    wT, gw, gB = ad.trajectory_gradient(w0, B, dt, steps, lamT, L, R, J, M, per, per, t)
    # the observable itself: dx h^2 sum g tr(sigma_z W) with tr(sigma_z W) = 2 w3
    h2 = (2 * L / N) ** 2
    assert np.isclose(np.sum(lamT * wT), h2 / Nx * np.sum(g[:, None, None] * 2 * wT[..., 3]))
    d, dB = rng.standard_normal(w0.shape), rng.standard_normal(B.shape)
    jw = _richardson(lambda s: loss(w0 + s * d, B), 1e-5)
    jB = _richardson(lambda s: loss(w0, B + s * dB), 1e-3)
    assert _rel(jw, np.sum(gw * d)) < 1e-8
    assert _rel(jB, np.sum(gB * dB)) < 1e-8
