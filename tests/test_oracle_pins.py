"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test names the passage it checks.  None of them retypes an oracle
formula: they compare against brute force in matrix form (no Pauli algebra,
no FFT), a direct quadrature of the continuum integrals eq. Cc / eq. Cd,
closed forms (eq. momentsFermiDirac, Bessel integrals), library routines the
oracle does not use (numpy.fft, scipy quadrature and Bessel functions), and
invariants (conservation, symmetries, structural zeros).
"""
import numpy as np
import pytest
from scipy import integrate, special

import brute
import continuum as ct
from oracle import collision as oc
from oracle import fermi_dirac as fd
from oracle import pauli, quadrature as qd, spectral as sp
from oracle import step as ostep
from oracle import transport as tp

L, R = 12.0, 7.5


def herm(rng, shape=()):
    A = rng.standard_normal(shape + (2, 2)) + 1j * rng.standard_normal(shape + (2, 2))
    return 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))


# ---------------------------------------------------------------- Fourier grid
def test_dft_matches_numpy_fft():
    """Mean-value coefficients on Xi (Sec. 3.2) vs numpy.fft with shifted axes."""
    rng = np.random.default_rng(0)
    for N in (4, 8, 16):
        f = rng.standard_normal((N, N))
        ref = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(f))) / N**2
        assert np.allclose(sp.dft_N(f), ref, atol=1e-14)
        assert np.allclose(sp.idft_N(sp.dft_N(f)).real, f, atol=1e-13)
        P = 2 * N
        g = rng.standard_normal((P, P))
        refP = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(g))) / P**2
        assert np.allclose(sp.dft_P(g), refP, atol=1e-14)


def test_padded_product_is_linear_convolution():
    """Double zero padding (Sec. 3.2): the product on the 2N grid equals the
    direct linear convolution of Nyquist-free coefficient arrays."""
    rng = np.random.default_rng(1)
    N = 6
    a = sp.zero_nyquist(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    b = sp.zero_nyquist(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    k = sp.freqs(N)
    direct = np.zeros((2 * N, 2 * N), complex)
    for i1, k1 in enumerate(k):
        for j1, l1 in enumerate(k):
            for i2, k2 in enumerate(k):
                for j2, l2 in enumerate(k):
                    direct[k1 + k2 + N, l1 + l2 + N] += a[i1, j1] * b[i2, j2]
    assert np.allclose(sp.conv(sp.pad(a), sp.pad(b)), direct, atol=1e-14)


# ---------------------------------------------------------------- P1, P2
def test_pauli_identities():
    """Sec. 3.1: gain and loss in Pauli form, anticommutator, H_eff
    integrand and commutator, each under v3 <-> v4 symmetrization, against
    2x2 complex matrix products."""
    rng = np.random.default_rng(2)
    I = np.eye(2)
    eta = np.array([1.0, -1.0, -1.0, -1.0])
    for _ in range(20):
        W1, W2, W3, W4 = (herm(rng) for _ in range(4))
        w1, w2, w3, w4 = (pauli.to_pauli(W) for W in (W1, W2, W3, W4))
        Wt2, Wt4 = I - W2, I - W4
        sym = lambda F: 0.5 * (F(W3, W4) + F(W4, W3))
        gain = sym(lambda a, b: -b @ Wt2 @ a + b * np.trace(Wt2 @ a)
                   + (-b @ Wt2 @ a + b * np.trace(Wt2 @ a)).conj().T)
        e2 = pauli.from_pauli(eta * w2)
        assert np.allclose(gain, 2 * pauli.eta_inner(w3, w4) * (I - e2), atol=1e-14)

        def loss(a, b):
            bt = I - b
            X = bt @ a - bt @ W2 - Wt2 @ a + bt * np.trace(W2) - bt * np.trace(a) + np.trace(a @ Wt2) * I
            return -X @ W1 + (-X @ W1).conj().T
        ref = -(pauli.eta_inner(w3, w4) * I - (w3[0] + w4[0] - 1) * e2) @ W1
        assert np.allclose(sym(loss), ref + ref.conj().T, atol=1e-14)

        anti = W1 @ W2 + W2 @ W1
        ref = 2 * (pauli.from_pauli(w1[0] * w2 + w2[0] * w1) - pauli.eta_inner(w1, w2) * I)
        assert np.allclose(anti, ref, atol=1e-14)

        heff = sym(lambda a, b: a @ b - W2 @ a - a @ W2 - np.trace(b) * a + np.trace(W2) * a + W2)
        ref = (pauli.eta_inner(w2, w2) - pauli.eta_inner(w3 - w2, w4 - w2)) * I - (w3[0] + w4[0] - 1) * W2
        assert np.allclose(heff, ref, atol=1e-14)

        comm = -1j * (W2 @ W1 - W1 @ W2)
        ref = pauli.from_pauli(np.concatenate([[0.0], 2 * np.cross(w2[1:], w1[1:])]))
        assert np.allclose(comm, ref, atol=1e-14)


def test_carleman_kinematics():
    """Sec. 3.2: v2 = v + u + u' and underline-omega = u . u' for omega = |v|^2/2."""
    rng = np.random.default_rng(3)
    om = lambda x: 0.5 * np.sum(x * x, -1)
    v, u, up = rng.standard_normal((3, 100, 2))
    v1, v3, v4 = v, v + u, v + up
    v2 = v3 + v4 - v1
    assert np.allclose(v2, v + u + up)
    assert np.allclose(om(v1) + om(v2) - om(v3) - om(v4), np.sum(u * up, -1), atol=1e-12)


# ---------------------------------------------------------------- P3 kernels
def _HJ(xi, chi, J):
    th = qd.theta(J)
    return np.sum(qd.omega_H(J) * qd.psi_R(th @ xi, L, R) * qd.psi_R(qd.rot90(th) @ chi, L, R))


def test_H_at_origin_and_symmetry():
    """eq. approxH-J: H_J(0, 0) = 4 pi R^2 (the exact value of
    int int_{B_R^2} delta(u.u')) and H_J(a, b) = H_J(b, a) for even J."""
    for J in (4, 8, 32):
        assert abs(_HJ(np.zeros(2), np.zeros(2), J) - 4 * np.pi * R**2) < 1e-12 * R**2
    rng = np.random.default_rng(4)
    for _ in range(10):
        a, b = rng.integers(-10, 10, (2, 2)).astype(float)
        assert abs(_HJ(a, b, 32) - _HJ(b, a, 32)) < 1e-10


def test_H_against_bessel_integral():
    """H(xi, 0) = 4 pi R int_0^R J_0(pi r |xi| / L) dr (polar form of the
    delta-kernel); the J = 32 trapezoid of eq. approxH-J reaches it."""
    for xi in ([1.0, 0.0], [3.0, 4.0], [7.0, -2.0], [12.0, 5.0]):
        xi = np.array(xi)
        k = np.pi * np.linalg.norm(xi) / L
        exact = 4 * np.pi * R * integrate.quad(lambda r: special.j0(k * r), 0, R, limit=200)[0]
        assert abs(_HJ(xi, np.zeros(2), 32) - exact) < 1e-9 * abs(4 * np.pi * R * R)


def test_G_against_principal_value_quadrature():
    """eq. approxG against -int int P(1/(theta.theta')) phi_R(xi.theta)
    phi_R(chi.theta') computed independently: the inner principal value by
    folding around the poles b = a + pi/2, a + 3pi/2 (regular integrand,
    Gauss-Legendre), the outer angle by a fine trapezoid rule."""
    J = 32
    th, thp = qd.theta(J), qd.theta_prime(J)

    def GJ(xi, chi):
        return np.sum(qd.omega_G(J) * np.outer(qd.phi_R(th @ xi, L, R), qd.phi_R(thp @ chi, L, R)))

    def G_pv(xi, chi, na=512, ns=96):
        a = 2 * np.pi * np.arange(na) / na
        x, ws = np.polynomial.legendre.leggauss(ns)
        s, ws = np.pi / 4 * (x + 1), np.pi / 4 * ws
        g = lambda b: qd.phi_R(chi[0] * np.cos(b) + chi[1] * np.sin(b), L, R)
        inner = np.zeros(na)
        for p, sgn in ((np.pi / 2, -1.0), (3 * np.pi / 2, 1.0)):
            # 1/cos(a - b) = sgn / sin(s) at b = a + p + s
            bp = a[:, None] + p + s[None, :]
            bm = a[:, None] + p - s[None, :]
            inner += sgn * ((g(bp) - g(bm)) / np.sin(s)[None, :]) @ ws
        f = qd.phi_R(xi[0] * np.cos(a) + xi[1] * np.sin(a), L, R)
        return -(2 * np.pi / na) * np.sum(f * inner)

    for xi, chi in (([1.0, 0.0], [0.0, 1.0]), ([2.0, -1.0], [1.0, 3.0]), ([5.0, 2.0], [-3.0, 4.0])):
        xi, chi = np.array(xi), np.array(chi)
        ref = G_pv(xi, chi)
        assert abs(GJ(xi, chi) - ref) < 1e-8 * max(1.0, abs(ref)), (GJ(xi, chi), ref)
    assert GJ(np.zeros(2), np.array([3.0, 1.0])) == 0.0
    assert GJ(np.array([3.0, 1.0]), np.zeros(2)) == 0.0


def test_gauss_legendre_reproduces_psi():
    """eq. approxH-JM: sum_m w_m exp(i pi rho_m x / L) -> psi_R(x)."""
    for M, xmax, tol in ((32, 10.0, 1e-10), (48, 20.0, 1e-11)):
        rho, w = qd.gauss_legendre(M, R)
        x = np.linspace(-xmax, xmax, 81)
        s = np.exp(1j * np.pi * np.outer(x, rho) / L) @ w
        assert np.abs(s - qd.psi_R(x, L, R)).max() < tol


# ---------------------------------------------------------------- P4 brute force
@pytest.mark.parametrize("N,J,M", [(4, 4, 4), (6, 4, 3)])
def test_oracle_matches_matrix_brute_force(N, J, M):
    """Sec. 3.2 scheme vs direct Fourier-triple sums of the matrix
    integrands (eq. CcPauliCarleman; A + A* of eq. Cd), tiny grids."""
    rng = np.random.default_rng(10 + N)
    Lb, Rb = 3.0, 2.0
    W = 0.3 * herm(rng, (N, N)) + 0.5 * np.eye(2)
    Cb = brute.collision_hat(W, Lb, Rb, J, M)
    cb = sp.zero_nyquist(0.5 * np.einsum("mab,xyba->mxy", brute.SIG, Cb))
    co = sp.zero_nyquist(oc.collision_hat(oc.pauli_hat(W), oc.Tables(N, Lb, Rb, J, M)))
    assert np.abs(cb - co).max() < 1e-12 * np.abs(co).max()


# ---------------------------------------------------------------- continuum
def test_oracle_converges_to_continuum_integrals():
    """eq. validationW: the scheme at N = 16, 32 against a direct quadrature
    of eq. Cc / eq. Heff and eq. Cd in matrix form at one grid point; the
    error is small at N = 32 and falls with N (spectral accuracy, Fig. 1)."""
    Wp = ct.periodized(ct.validation_W, L)
    errs = []
    for N in (16, 32):
        v = sp.velocity_axis(N, L)
        V = np.stack(np.meshgrid(v, v, indexing="ij"), -1)
        w = pauli.to_pauli(ct.validation_W(V))
        t = oc.Tables(N, L, R, 32, N)
        parts = oc.collision_hat(sp.zero_nyquist(sp.dft_N(np.moveaxis(w, -1, 0))), t, parts=True)
        real = lambda ch: pauli.from_pauli(np.moveaxis(sp.idft_N(sp.zero_nyquist(ch)).real, 0, -1))
        i, k = N // 2 + N // 16, N // 2 - N // 16
        Cc = real(parts["Cc"])[i, k]
        Cd = real(parts["A"] + parts["B"] + parts["C"])[i, k]
        if N == 16:
            cc_ref = ct.Cc_at(Wp, V[i, k], R, n_r=32, n_a=48, n_s=32)
            cd_ref = ct.Cd_at(Wp, V[i, k], R, n_r=40, n_a=64, n_t=48)
        errs.append((np.abs(Cc - cc_ref).max() / np.abs(cc_ref).max(),
                     np.abs(Cd - cd_ref).max() / np.abs(cd_ref).max()))
    # both grids put the same velocity (1.5, -1.5) at (i, k)
    assert errs[1][0] < 3e-3 and errs[1][1] < 1e-2, errs
    assert errs[1][0] < errs[0][0] / 10 and errs[1][1] < errs[0][1] / 5, errs


# ---------------------------------------------------------------- P5, P6
def test_structural_zeros():
    """C_c vanishes when all W(v) commute; W proportional to 1 gives a
    collision term proportional to 1 (Sec. 2, scalar case)."""
    N, J, M = 8, 8, 8
    rng = np.random.default_rng(5)
    t = oc.Tables(N, L, R, J, M)
    v = sp.velocity_axis(N, L)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    Wc = fd.fd_matrix(vx, vy, 1.0, 1.0, -0.5, U=np.array([[1, 1j], [1j, 1]]) / np.sqrt(2))
    parts = oc.collision_hat(oc.pauli_hat(Wc), t, parts=True)
    assert np.abs(parts["Cc"]).max() < 1e-14
    f = rng.uniform(0.1, 0.9, (N, N))
    c = oc.collision_pauli(np.stack([f, 0 * f, 0 * f, 0 * f], -1), L, R, J, M, t)
    assert np.abs(c[..., 1:]).max() < 1e-14 * np.abs(c[..., 0]).max()


def test_scalar_reduction_matches_uehling_uhlenbeck():
    """W = f 1 reduces C to the scalar Uehling-Uhlenbeck operator
    2 pi int delta(u.u') [f_a f_b (1-f)(1-f_c) - f f_c (1-f_a)(1-f_b)]
    (Sec. 2; a = v+u, b = v+u', c = v+u+u'), evaluated here by the brute
    force with a scalar integrand."""
    N, J, M, Lb, Rb = 4, 4, 4, 3.0, 2.0
    rng = np.random.default_rng(6)
    f = rng.uniform(0.2, 0.8, (N, N))
    W = f[..., None, None] * np.eye(2)
    orig_c, orig_d = brute.Fc, brute.Fd
    try:
        def uu(W1, W2, W3, W4):
            s = lambda X: X[..., 0, 0][..., None, None] * np.eye(2)   # scalar part
            f1, f2, f3, f4 = s(W1), s(W2), s(W3), s(W4)
            one = np.eye(2)
            return 2 * (f3 * f4 * (one - f1) * (one - f2) - f1 * f2 * (one - f3) * (one - f4))
        brute.Fc = lambda *a: 0 * a[0]
        brute.Fd = lambda W1, W2, W3, W4: 0.5 * (uu(W1, W2, W3, W4) + uu(W1, W2, W4, W3))
        ref = brute.collision_hat(W, Lb, Rb, J, M)[..., 0, 0]
    finally:
        brute.Fc, brute.Fd = orig_c, orig_d
    co = oc.collision_hat(oc.pauli_hat(W), oc.Tables(N, Lb, Rb, J, M))
    assert np.abs(sp.zero_nyquist(co[0] - ref)).max() < 1e-12 * np.abs(ref).max()


# ---------------------------------------------------------------- P7, P8, P9
def test_fermi_dirac_residual_falls_with_N():
    """W_FD (eq. W_FermiDirac) is a stationary state of C; the discrete
    residual falls as the grid is refined (Sec. 2, Fig. 4c)."""
    res = []
    for N in (16, 24):
        v = sp.velocity_axis(N, L)
        vx, vy = np.meshgrid(v, v, indexing="ij")
        U = np.array([[np.cos(0.3), -np.sin(0.3)], [np.sin(0.3), np.cos(0.3)]])
        W = fd.fd_matrix(vx, vy, 1.0, 1.0, 0.5, U=U)
        parts = oc.collision_hat(oc.pauli_hat(W), oc.Tables(N, L, R, 32, N), parts=True)
        c = sp.idft_N(sp.zero_nyquist(sum(parts.values()))).real
        res.append(np.abs(c).max() / np.abs(parts["A"]).max())
    assert res[1] < res[0] / 4, res


def test_collision_conserves_density():
    """int C dv = 0 (Sec. 2) holds for the scheme up to quadrature error."""
    import workloads as wl
    N = 24
    W = wl.perturbed_fd(np.random.default_rng(7), 1, N, 1.0, lambda x: 0.5 + 0 * x)[0]
    c = oc.collision_pauli(pauli.to_pauli(W), L, R, 32, N)
    tot = np.abs(c).sum(axis=(0, 1))
    assert np.all(np.abs(c.sum(axis=(0, 1))) < 1e-8 * tot)


def test_collision_momentum_and_energy_conservation_improves_with_N():
    """int v tr C dv and int |v|^2/2 tr C dv vanish for the continuum operator
    (Sec. 2); the discrete scheme conserves them to discretisation accuracy
    only, so relative to the gross fluxes the errors must fall with N
    (measured: momentum 2e-2 -> 1e-2, energy 5e-3 -> 1e-3 from N = 16 to 32)."""
    import workloads as wl
    errs = []
    for N in (16, 32):
        W = wl.perturbed_fd(np.random.default_rng(7), 1, N, 1.0, lambda x: 0.5 + 0 * x)[0]
        c = oc.collision_pauli(pauli.to_pauli(W), L, R, 32, N)
        v = sp.velocity_axis(N, L)
        vx, vy = np.meshgrid(v, v, indexing="ij")
        tr = 2 * c[..., 0]
        p = max(abs((vx * tr).sum()), abs((vy * tr).sum())) / np.abs(vx * tr).sum()
        e = abs((0.5 * (vx**2 + vy**2) * tr).sum()) / np.abs(0.5 * (vx**2 + vy**2) * tr).sum()
        errs.append((p, e))
    (p16, e16), (p32, e32) = errs
    assert p32 < p16 and e32 < e16
    assert p32 < 2e-2 and e32 < 2e-3


def test_fermi_dirac_moments_closed_form():
    """eq. momentsFermiDirac: discrete density and energy of W_FD on the
    velocity grid equal the log / Li_2 closed forms (trapezoid rule on a
    smooth decaying integrand)."""
    N = 64
    v = sp.velocity_axis(N, L)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    for inv_kT, mus in ((1.0, (1.0, 1.5)), (0.8, (1.5, -1.5)), (2.0, (0.0, 0.0))):
        W = fd.fd_matrix(vx, vy, inv_kT, *mus)
        w = pauli.to_pauli(W)[None]
        m = ostep.moments(w, L)[0]
        dens = 2 * m[0]
        # trapezoid error ~ exp(-2 pi d / h), d = distance of the integrand's
        # poles (|v|^2 = 2 (mu +- i pi kT)) from the real axis
        assert abs(dens - fd.fd_density(inv_kT, mus)) < 1e-7 * dens
        assert abs(m[6] / dens - fd.fd_energy(inv_kT, mus)) < 1e-7
        assert abs(m[4]) < 1e-12 and abs(m[5]) < 1e-12


# ---------------------------------------------------------------- P10, P11
def _transport_state(Nx, N, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-0.2, 0.2, (Nx, N, N, 4)) + np.array([0.5, 0, 0, 0])


def test_transport_periodic_invariants():
    """eq. slopeLimiterStep: constants are preserved; the sum over cells is
    conserved with periodic BCs; at nu = 1 the step is an exact one-cell
    shift; minmod keeps each component total-variation diminishing."""
    per = {"kind": "periodic"}
    Nx, N = 12, 8
    w = _transport_state(Nx, N, 8)
    const = np.ones_like(w) * np.array([0.4, 0.1, -0.2, 0.05])
    assert np.allclose(tp.transport_step(const, 1e-3, per, per, L), const, atol=1e-15)
    dt = 0.5 * (1.0 / Nx) / L
    w1 = tp.transport_step(w, dt, per, per, L)
    assert np.allclose(w1.sum(0), w.sum(0), atol=1e-13)
    tv = lambda a: np.abs(np.roll(a, -1, 0) - a).sum(0)
    assert np.all(tv(w1) <= tv(w) + 1e-13)
    # nu = 1 for v_x = 2L/N * k: choose dt so that the row i = N/2 + 1 moves one cell
    vx1 = 2 * L / N
    w2 = tp.transport_step(w, (1.0 / Nx) / vx1, per, per, L)
    assert np.allclose(w2[:, N // 2 + 1], np.roll(w[:, N // 2 + 1], 1, axis=0), atol=1e-14)
    assert np.allclose(w2[:, N // 2 - 1], np.roll(w[:, N // 2 - 1], -1, axis=0), atol=1e-14)
    assert np.allclose(w2[:, N // 2], w[:, N // 2], atol=0)


def test_maxwell_inflow_balances_flux():
    """Maxwell reflection (Sec. 2): the inflow number flux equals the
    outflow flux of the adjacent cell (specular and diffusive parts), the
    unmirrored row v_x = -L excluded."""
    N = 16
    v = sp.velocity_axis(N, L)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    hv2 = (2 * L / N) ** 2
    wb = pauli.to_pauli(fd.fd_matrix(vx, vy, 1.3, 0.7, -0.2, v0=(0.6, 0.1)))
    wfd = pauli.to_pauli(fd.fd_matrix(vx, vy, 2.0, 0.0, 0.0))
    for side in ("left", "right"):
        for alpha in (0.0, 0.5, 1.0):
            state, inflow = tp.maxwell_inflow(wb, wfd, alpha, side, v, hv2)
            outflow = v < 0 if side == "left" else v > 0
            fin = hv2 * np.sum(2 * state[inflow][..., 0] * np.abs(v[inflow])[:, None])
            fout = hv2 * np.sum(2 * wb[outflow][..., 0] * np.abs(v[outflow])[:, None])
            assert abs(fin - fout) < 1e-13 * fout


# ---------------------------------------------------------------- P12, P13
def test_magnetic_term_rotates_spin():
    """-i[B.sigma, W] (eq. boltzmann) leaves tr W unchanged and is
    orthogonal to the Bloch vector, so |w_vec| is kept to O(dt^3) by Heun."""
    rng = np.random.default_rng(9)
    w = rng.uniform(-0.3, 0.3, (3, 2, 2, 4))
    B = rng.standard_normal((3, 3))
    m = ostep.magnetic(w, B)
    assert np.abs(m[..., 0]).max() == 0.0
    assert np.abs(np.sum(m[..., 1:] * w[..., 1:], -1)).max() < 1e-15
    W = pauli.from_pauli(w[0, 0, 0])
    Bs = pauli.from_pauli(np.concatenate([[0.0], B[0]]))
    assert np.allclose(pauli.from_pauli(m[0, 0, 0]), -1j * (Bs @ W - W @ Bs), atol=1e-15)


def test_step_reductions():
    """Sec. 4 splitting: with one periodic cell transport is the identity and
    the step is one Heun step of C + field; with C and B switched off the
    step is two transport half-steps."""
    N, J, M = 8, 4, 4
    rng = np.random.default_rng(11)
    per = {"kind": "periodic"}
    w = _transport_state(1, N, 12)
    B = rng.standard_normal((1, 3))
    t = oc.Tables(N, L, R, J, M)
    s = ostep.step(w, B, 1e-3, L, R, J, M, per, per, t)
    h = ostep.heun(w, B, 1e-3, L, t)
    assert np.allclose(s, h, atol=1e-15)
    w = _transport_state(6, N, 13)
    zero_t = oc.Tables(N, L, 0.0, J, M)     # R = 0 switches the collision off
    s = ostep.step(w, np.zeros((6, 3)), 2e-3, L, 0.0, J, M, per, per, zero_t)
    ref = tp.transport_step(tp.transport_step(w, 1e-3, per, per, L), 1e-3, per, per, L)
    assert np.allclose(s, ref, atol=1e-15)


# ---------------------------------------------------------------- wall ghost cells
# Sec. 2 boundary conditions inside eq. slopeLimiterStep (Sec. 4), read as
# two ghost cells per wall that hold the inflow state at entering v_x and a
# copy of the adjacent cell otherwise.  The expected values below are closed
# forms of one step, written from the grid alone (explicit loops over rows,
# no call of the oracle's ghost or inflow helpers).

def _rows(N):
    """(i, v_x) for every row of the velocity grid v_x = (2L/N)(i - N/2)."""
    h = 2 * L / N
    return [(i, h * (i - N // 2)) for i in range(N)]


def _const_field(N, c):
    return np.broadcast_to(np.asarray(c, float), (N, N, 4)).copy()


@pytest.mark.parametrize("side", ["left", "right"])
def test_dirichlet_wall_into_empty_slab(side):
    """Zero interior, Dirichlet state Phi on one wall (the other wall a
    zero Dirichlet state): every one-sided difference next to the wall has
    the inflow jump on one side and zero on the other, so every limited
    slope vanishes and the step is first-order upwind.  The wall cell then
    holds (dt/dx) |v_x| Phi on the rows entering through that wall and 0 on
    every other row; every other cell stays 0."""
    Nx, N = 7, 8
    rng = np.random.default_rng(21)
    phi = rng.uniform(0.05, 0.4, (N, N, 4))
    zero = np.zeros((N, N, 4))
    bc_phi = {"kind": "dirichlet", "state": phi}
    bc_zero = {"kind": "dirichlet", "state": zero}
    bl, br = (bc_phi, bc_zero) if side == "left" else (bc_zero, bc_phi)
    dx = 1.0 / Nx
    dt = 0.8 * dx / L                       # CFL number 0.8 on the fastest row
    w1 = tp.transport_step(np.zeros((Nx, N, N, 4)), dt, bl, br, L)
    wall = 0 if side == "left" else Nx - 1
    expect = np.zeros((Nx, N, N, 4))
    for i, vx in _rows(N):
        entering = vx > 0 if side == "left" else vx < 0
        if entering:
            expect[wall, i] = (dt / dx) * abs(vx) * phi[i]
    assert np.array_equal(np.delete(w1, wall, axis=0), np.delete(expect, wall, axis=0))
    assert np.allclose(w1[wall], expect[wall], rtol=1e-14, atol=0)
    assert np.any(expect[wall] != 0)


def test_dirichlet_walls_uniform_interior():
    """Interior state U equal in every cell and velocity, Dirichlet states
    Phi_l, Phi_r: every limited slope vanishes (all interior differences are
    zero and the wall differences meet a zero on their other side), so the
    wall cells relax toward the wall states at the upwind rate,
    U + (dt/dx) |v_x| (Phi - U), on the entering rows, and everything else
    keeps U."""
    Nx, N = 6, 8
    rng = np.random.default_rng(22)
    U = np.array([0.45, 0.05, -0.1, 0.02])
    phl = rng.uniform(0.05, 0.4, (N, N, 4))
    phr = rng.uniform(0.05, 0.4, (N, N, 4))
    dx = 1.0 / Nx
    dt = 0.6 * dx / L
    w = np.broadcast_to(U, (Nx, N, N, 4)).copy()
    w1 = tp.transport_step(w, dt, {"kind": "dirichlet", "state": phl},
                           {"kind": "dirichlet", "state": phr}, L)
    expect = w.copy()
    for i, vx in _rows(N):
        if vx > 0:
            expect[0, i] = U + (dt / dx) * vx * (phl[i] - U)
        if vx < 0:
            expect[Nx - 1, i] = U + (dt / dx) * (-vx) * (phr[i] - U)
    assert np.allclose(w1, expect, rtol=0, atol=1e-15)


def test_maxwell_walls_closed_form():
    """Maxwell walls (Sec. 2) on a slab whose every cell holds the same
    state U(v_x), which varies with v_x only (so that the mirror row
    matters), and a wall state G constant in v.  The inflow state at an
    entering row i is (1 - alpha) U(row N - i) + alpha G Fbar / Z with the
    outgoing number flux Fbar = h^2 sum_out 2 u_0 |v_x| and the incoming
    flux of G, Z = h^2 sum_in 2 g_0 |v_x|, both sums written out below over
    the rows (the row v_x = -L has no mirror: it enters at neither wall's
    sums on the right and keeps U).  Every limited slope vanishes as in the
    Dirichlet case, so the wall cells take U + (dt/dx) |v_x| (state - U) on
    the entering rows."""
    Nx, N = 5, 8
    h = 2 * L / N
    rng = np.random.default_rng(23)
    Urow = np.column_stack([rng.uniform(0.3, 0.6, N), rng.uniform(-0.1, 0.1, (N, 3))])
    U = np.broadcast_to(Urow[:, None, :], (N, N, 4))
    G = np.array([0.35, 0.0, 0.04, -0.03])
    dx = 1.0 / Nx
    dt = 0.7 * dx / L
    for al, ar in ((0.0, 1.0), (0.4, 0.5), (1.0, 0.0)):
        w = np.broadcast_to(U, (Nx, N, N, 4)).copy()
        bl = {"kind": "maxwell", "state": _const_field(N, G), "alpha": al}
        br = {"kind": "maxwell", "state": _const_field(N, G), "alpha": ar}
        w1 = tp.transport_step(w, dt, bl, br, L)
        expect = w.copy()
        for side, alpha, cell in (("left", al, 0), ("right", ar, Nx - 1)):
            if side == "left":
                enter = [i for i, vx in _rows(N) if vx > 0]
                leave = [i for i, vx in _rows(N) if vx < 0]
            else:
                enter = [i for i, vx in _rows(N) if vx < 0 and i > 0]
                leave = [i for i, vx in _rows(N) if vx > 0]
            vabs = {i: abs(vx) for i, vx in _rows(N)}
            Fbar = h * h * sum(N * 2 * Urow[i, 0] * vabs[i] for i in leave)
            Z = h * h * sum(N * 2 * G[0] * vabs[i] for i in enter)
            for i in enter:
                state = (1 - alpha) * Urow[N - i] + alpha * G * Fbar / Z
                expect[cell, i] = Urow[i] + (dt / dx) * vabs[i] * (state - Urow[i])
        assert np.allclose(w1, expect, rtol=0, atol=1e-14), (al, ar)
