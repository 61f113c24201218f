"""Pins of the initial states of the paper's simulations (Sec. 5.2, 5.3),
built in `workloads.physics_run`, against properties that do not use the
generator's own steps: unitary conjugation keeps the Fermi-Dirac
eigenvalues (eq. W0homogeneous), the rotation is the matrix exponential
of X(v) (checked against scipy's expm), U0 is unitary, the x-profile of
the periodic run carries no total momentum by symmetry, and the wall
states of Tables 1 and 2 have the tabulated occupations in the tabulated
spin basis."""
import numpy as np
import pytest
import scipy.linalg

import workloads as wl


def _fd(e, kT, mu):
    return 1.0 / (np.exp((e - mu) / kT) + 1.0)


def test_homogeneous_state_keeps_the_fermi_dirac_eigenvalues():
    N, kT, mu, v0 = 32, 1.25, (1.0, 1.5), (0.4, -0.1)
    W = wl.rotated_fd_state(N, kT, *mu, v0)
    assert np.abs(W - np.conj(np.swapaxes(W, -1, -2))).max() < 1e-15
    v = wl.velocity_axis(N)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    e = 0.5 * ((vx - v0[0]) ** 2 + (vy - v0[1]) ** 2)
    want = np.sort(np.stack([_fd(e, kT, mu[0]), _fd(e, kT, mu[1])], -1), -1)
    got = np.linalg.eigvalsh(W)
    assert np.allclose(got, want, rtol=0, atol=1e-14)


def test_rotation_is_the_matrix_exponential():
    rng = np.random.default_rng(3)
    U0 = wl.HOMOGENEOUS_U0
    assert np.allclose(U0 @ np.conj(U0.T), np.eye(2), atol=1e-15)
    for _ in range(5):
        vx, vy = rng.uniform(-12, 12, 2)
        X = wl.rotation_generator(np.array(vx), np.array(vy))
        comp = [np.sin(vy**2), vx - 1.0, 2.0 / (vx**2 + abs(vy) + 1.0), np.cos(vx + 0.5 * vy)]
        assert np.allclose([0.5 * np.trace(X @ wl.SIGMA[m]).real for m in range(4)], comp, atol=1e-15)
        assert np.allclose(wl._expm_herm(X, -1j), scipy.linalg.expm(-1j * X), atol=1e-13)


def test_periodic_profile_has_no_total_momentum():
    w = wl.physics_run("E3")
    assert (w.Nx, w.N, w.dt, w.steps) == (10, 32, 0.008, 250)
    v = wl.velocity_axis(w.N)
    tr = np.trace(w.W0, axis1=-2, axis2=-1).real
    px = (tr * v[None, :, None]).sum()
    py = (tr * v[None, None, :]).sum()
    assert abs(px) < 1e-12 * np.abs(tr * v[None, :, None]).sum()
    assert abs(py) < 1e-12 * np.abs(tr * v[None, None, :]).sum()
    # the cell-wise momenta do not vanish: the profile moves
    assert np.abs((tr * v[None, :, None]).sum(axis=(1, 2))).max() > 1e-2
    B = wl.physics_run("E4").B
    x = wl.cell_centres(10)
    assert np.allclose(B, np.stack([0 * x, np.cos(2 * np.pi * x), np.sin(2 * np.pi * x)], 1))


@pytest.mark.parametrize("name,left,right", [
    ("E5", (0.8, 1.5, -1.5, False), (1.2, 1.5, -1.5, True)),
    ("E6i", (0.6, -0.4, 1.8, False), (1.1, 1.3, -0.9, False)),
    ("E6ii", (1.0, 1.5, -1.5, False), (1.0, 1.5, -1.5, True)),
])
def test_wall_states_follow_the_tables(name, left, right):
    w = wl.physics_run(name)
    assert (w.Nx, w.dt, w.steps) == (40, 0.002, 2000)
    v = wl.velocity_axis(w.N)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    for bc, (ib, mu_u, mu_d, rot) in ((w.left, left), (w.right, right)):
        assert bc.kind == ("dirichlet" if name == "E5" else "maxwell")
        assert (bc.inv_kT, bc.mu_up, bc.mu_down) == (ib, mu_u, mu_d)
        assert bc.alpha == (0.0 if name == "E5" else 0.4)
        S = wl.fd_wall_state(w.N, bc.inv_kT, bc.mu_up, bc.mu_down, bc.U)
        e = 0.5 * (vx**2 + vy**2)
        up = np.asarray(bc.U)[:, 0]
        # the first column of U is the spin-up eigenvector with occupation f(mu_up)
        assert np.allclose(S @ up, _fd(e, 1 / ib, mu_u)[..., None] * up, atol=1e-14)
        c = 1 / np.sqrt(2)
        assert np.allclose(up, [c, c] if rot else [1, 0])
