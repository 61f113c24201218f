"""Reverse-mode derivatives (vector-Jacobian products) of the oracle's
collision operator, transport step and splitting step, and the gradient of
a final-time observable along a trajectory.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every function here runs the corresponding forward function of this package
backwards, one linear step at a time, and applies the transpose of that
step.  Conventions:

* Real arrays (Pauli components on the velocity grid, the field B) carry
  ordinary gradients:  dl = sum grad * dx.
* Complex coefficient arrays carry "bilinear" cotangents lam with
  dl = Re sum lam * dx (no conjugation).  With this pairing the transpose of
  a dense DFT matrix is the matrix itself (the matrices of ``spectral`` are
  symmetric), a pointwise product transposes to the same product, zero
  padding transposes to truncation and back, and taking a real part
  transposes to embedding a real cotangent.

Nothing here is tuned: the loops are the forward loops, in the same order.
"""
import numpy as np

from . import spectral as sp
from . import transport as tp
from .collision import LEVI_CIVITA, Tables
from .pauli import ETA
from .step import magnetic


# ----------------------------------------------------------------- convolution
def conv_vjp(ahat, bhat, lam, sum_a=None, sum_b=None):
    """Cotangents of a and b for y = conv(a, b) given the cotangent lam of y.
    sum_a / sum_b: axes of the broadcast product to sum out for a / b."""
    ly = sp.dft_P(lam)                      # transpose of the outer dft_P
    ra, rb = sp.idft_P(ahat), sp.idft_P(bhat)
    la = ly * rb
    lb = ly * ra
    if sum_a is not None:
        la = la.sum(axis=sum_a)
    if sum_b is not None:
        lb = lb.sum(axis=sum_b)
    return sp.idft_P(la), sp.idft_P(lb)


# ----------------------------------------------------------------- the four forms
def form_I1_vjp(t, fh, gh, hh, lam):
    """Transpose of collision.form_I1: lam[A, B, N, N] -> (lf, lg[A], lh[B])."""
    F, G, H = sp.pad(fh), sp.pad(gh), sp.pad(hh)
    h_real = sp.idft_P(H)
    lF = np.zeros_like(F)
    lG = np.zeros_like(G)
    lh_real = np.zeros_like(h_real)
    for jp in range(t.J):
        pG = t.phip[jp][None] * G
        inner = sp.conv(F[None], pG)
        for j in range(t.J):
            x = sp.idft_P(t.phi[j][None] * inner)                   # [A, P, P]
            lprod = sp.dft_P(sp.pad(t.omega_G[j, jp] * lam))        # [A, B, P, P]
            lx = (lprod * h_real[None]).sum(axis=1)
            lh_real += (lprod * x[:, None]).sum(axis=0)
            linner = t.phi[j][None] * sp.idft_P(lx)
            la, lb = conv_vjp(F[None], pG, linner, sum_a=0)
            lF += la
            lG += t.phip[jp][None] * lb
    lH = sp.idft_P(lh_real)
    return sp.truncate(lF), sp.truncate(lG), sp.truncate(lH)


def form_I2_vjp(t, fh, gh, hh, lam):
    """Transpose of collision.form_I2: lam[A, B, N, N] -> (lf[A], lg[A], lh[B])."""
    F, G, H = sp.pad(fh), sp.pad(gh), sp.pad(hh)
    lF = np.zeros_like(F)
    lG = np.zeros_like(G)
    lH = np.zeros_like(H)
    for j in range(t.J):
        pF, pG = t.psi[j][None] * F, t.psip[j][None] * G
        a = sp.conv(pF, pG)                                          # [A, P, P]
        lo = sp.pad(t.omega_H[j] * lam)                              # [A, B, P, P]
        la, lh = conv_vjp(a[:, None], H[None], lo, sum_a=1, sum_b=0)
        lH += lh
        lpF, lpG = conv_vjp(pF, pG, la)
        lF += t.psi[j][None] * lpF
        lG += t.psip[j][None] * lpG
    return sp.truncate(lF), sp.truncate(lG), sp.truncate(lH)


def form_I4_vjp(t, fh, gh, hh, lam):
    """Transpose of collision.form_I4: lam[A, B, N, N] -> (lf, lg[A], lh[B])."""
    F, G, H = sp.pad(fh), sp.pad(gh), sp.pad(hh)
    h_real = sp.idft_P(H)
    lF = np.zeros_like(F)
    lG = np.zeros_like(G)
    lh_real = np.zeros_like(h_real)
    for j in range(t.J):
        pG = t.psip[j][None] * G
        inner = sp.conv(F[None], pG)
        x = sp.idft_P(t.psi[j][None] * inner)
        lprod = sp.dft_P(sp.pad(t.omega_H[j] * lam))
        lx = (lprod * h_real[None]).sum(axis=1)
        lh_real += (lprod * x[:, None]).sum(axis=0)
        linner = t.psi[j][None] * sp.idft_P(lx)
        la, lb = conv_vjp(F[None], pG, linner, sum_a=0)
        lF += la
        lG += t.psip[j][None] * lb
    lH = sp.idft_P(lh_real)
    return sp.truncate(lF), sp.truncate(lG), sp.truncate(lH)


def form_I3_vjp(t, fh, gh, hh, lam, m_chunk=8):
    """Transpose of collision.form_I3: lam[A, B, N, N] -> (lf[A], lg[A], lh[B])."""
    F, G, H = sp.pad(fh), sp.pad(gh), sp.pad(hh)
    lF = np.zeros_like(F)
    lG = np.zeros_like(G)
    lH = np.zeros_like(H)
    rG = sp.idft_P(G)                                                # [A, P, P]
    for j in range(t.J):
        for m0 in range(0, t.M, m_chunk):
            ms = np.arange(m0, min(m0 + m_chunk, t.M))
            E = t.modulation(j, ms)                                  # [m, P, P]
            EF = E[:, None] * F[None]                                # [m, A, P, P]
            EH = E[:, None] * H[None]                                # [m, B, P, P]
            inner = sp.conv(G[None, :, None], EH[:, None, :])        # [m, A, B, P, P]
            inner2 = t.psip[j] * inner
            wts = t.omega_H[j] * t.wgl[ms]
            lo = sp.pad(wts[:, None, None, None, None] * lam[None])  # [m, A, B, P, P]
            ly = sp.dft_P(lo)
            rEF = sp.idft_P(EF)[:, :, None]
            rI = sp.idft_P(inner2)
            lEF = sp.idft_P((ly * rI).sum(axis=2))                   # [m, A, P, P]
            linner = t.psip[j] * sp.idft_P(ly * rEF)                 # [m, A, B, P, P]
            ly2 = sp.dft_P(linner)
            rEH = sp.idft_P(EH)[:, None, :]
            lG += sp.idft_P((ly2 * rEH).sum(axis=(0, 2)))
            lEH = sp.idft_P((ly2 * rG[None, :, None]).sum(axis=1))   # [m, B, P, P]
            lF += (E[:, None] * lEF).sum(axis=0)
            lH += (E[:, None] * lEH).sum(axis=0)
    return sp.truncate(lF), sp.truncate(lG), sp.truncate(lH)


# ----------------------------------------------------------------- C[W]
def collision_hat_vjp(what, lamC, t):
    """Transpose of collision.collision_hat at w_hat[4, N, N]: the bilinear
    cotangent of w_hat from the cotangent lamC[4, N, N] of C_hat."""
    N = what.shape[-1]
    one = sp.delta_hat(N)
    w = what
    f0 = 2.0 * w[0] - one
    lw = np.zeros_like(w)
    pi = np.pi

    # C_c,k = -2 eps_klm T1[l, m]
    lT1 = -2.0 * np.einsum("klm,kxy->lmxy", LEVI_CIVITA, lamC[1:4])
    lf, lg, lh = form_I1_vjp(t, f0, w[1:4], w[1:4], lT1)
    lw[0] += 2.0 * lf
    lw[1:4] += lg + lh

    # A: pi * (2 S2[0], -2 S2[1:]),  S2[h] = sum_mu eta_mu T2[mu, h]
    lS2 = np.concatenate([2.0 * pi * lamC[:1], -2.0 * pi * lamC[1:]])
    lT2 = ETA[:, None, None, None] * lS2[None]
    hA = np.stack([one - w[0], w[1], w[2], w[3]])
    lf, lg, lh = form_I2_vjp(t, w, w, hA, lT2)
    lw += lf + lg
    lw[0] -= lh[0]
    lw[1:4] += lh[1:4]

    # B: pi * (-2 S3[0], 2 S3[1:]),  S3[nu] = sum_mu eta_mu T3[mu, nu]
    lS3 = np.concatenate([-2.0 * pi * lamC[:1], 2.0 * pi * lamC[1:]])
    lT3 = ETA[:, None, None, None] * lS3[None]
    lf, lg, lh = form_I3_vjp(t, w, w, w, lT3)
    lw += lf + lg + lh

    # Cq: pi * 2 (T4[0,0] - sum_k T4[k,k]) and pi * 2 (T4[0,k] - T4[k,0])
    lT4 = np.zeros((4, 4) + lamC.shape[1:], dtype=np.complex128)
    lT4[0, 0] = 2.0 * pi * lamC[0]
    for k in range(1, 4):
        lT4[k, k] = -2.0 * pi * lamC[0]
        lT4[0, k] = 2.0 * pi * lamC[k]
        lT4[k, 0] = -2.0 * pi * lamC[k]
    lf, lg, lh = form_I4_vjp(t, f0, w, w, lT4)
    lw[0] += 2.0 * lf
    lw += lg + lh
    return lw


def collision_pauli_vjp(w, lam, L, R, J, M, tables=None):
    """grad_w <lam, C[w]> for one cell: w[N, N, 4], lam[N, N, 4] -> [N, N, 4]."""
    N = w.shape[0]
    t = tables if tables is not None else Tables(N, L, R, J, M)
    what = sp.zero_nyquist(sp.dft_N(np.moveaxis(np.asarray(w, np.float64), -1, 0)))
    # c = Re idft_N(Z(C_hat)):  cotangent of C_hat = Z(idft_N(lam))
    lamC = sp.zero_nyquist(sp.idft_N(np.moveaxis(np.asarray(lam, np.float64), -1, 0)))
    lw = collision_hat_vjp(what, lamC, t)
    # w_hat = Z(dft_N(w)) with w real
    return np.moveaxis(sp.dft_N(sp.zero_nyquist(lw)).real, 0, -1)


# ----------------------------------------------------------------- transport
def ghosts_vjp(w, lwe, bc_left, bc_right, vx, hv2):
    """Transpose of transport.ghosts at w[Nx, ...]: cotangent of w from the
    cotangent lwe[Nx + 4, ...] of the extended array."""
    Nx = w.shape[0]
    lw = np.zeros_like(w)
    if bc_left["kind"] == "periodic":
        np.add.at(lw, np.arange(-2, Nx + 2) % Nx, lwe)
        return lw
    lw += lwe[2:-2]
    for side, bc, cell, gidx in (
        ("left", bc_left, 0, (0, 1)),
        ("right", bc_right, Nx - 1, (Nx + 2, Nx + 3)),
    ):
        if bc["kind"] == "dirichlet":
            inflow = vx > 0 if side == "left" else vx < 0
        else:
            _, inflow = tp.maxwell_inflow(w[cell], bc["state"], bc["alpha"], side, vx, hv2)
        lstate = np.zeros_like(w[cell])
        for g in gidx:
            lw[cell][~inflow] += lwe[g][~inflow]
            lstate[inflow] += lwe[g][inflow]
        if bc["kind"] == "maxwell":
            # state[rows] = (1 - alpha) wb[mir[rows]] + alpha w_fd[rows] Fbar / Z
            N = w.shape[1]
            mir = tp.mirror_rows(N)
            alpha, w_fd = bc["alpha"], bc["state"]
            rows = np.nonzero(inflow)[0]
            lw[cell][mir[rows]] += (1.0 - alpha) * lstate[rows]
            outflow = vx < 0 if side == "left" else vx > 0
            Z = hv2 * np.sum(2.0 * w_fd[..., 0][inflow] * np.abs(vx[inflow])[:, None])
            lF = alpha / Z * np.sum(lstate[rows] * w_fd[rows])
            # Fbar = hv2 sum_out 2 w0 |v_x|
            lw[cell][outflow, :, 0] += lF * hv2 * 2.0 * np.abs(vx[outflow])[:, None]
    return lw


def transport_step_vjp(w, lam, dt, bc_left, bc_right, L):
    """Transpose of transport.transport_step at w[Nx, N, N, 4] (the limiter's
    branches taken at w) applied to lam[Nx, N, N, 4]."""
    Nx, N = w.shape[0], w.shape[1]
    dx = 1.0 / Nx
    vx = (2.0 * L / N) * (np.arange(N) - N // 2)
    hv2 = (2.0 * L / N) ** 2
    we = tp.ghosts(w, bc_left, bc_right, vx, hv2)
    d = we[1:] - we[:-1]
    a, b = d[1:], d[:-1]
    v = vx[None, :, None, None]
    av = np.abs(v)
    nu = dt * v / dx
    lim = 0.5 * (np.sign(nu) - nu)
    c = dt / (2.0 * dx)
    lwe = np.zeros_like(we)
    lS = np.zeros_like(we)
    # out = W0 + c (-v (Wp - Wm) + av (Wp - 2 W0 + Wm)
    #               + lim (-v (Sp - Sm) + av (Sp - 2 S0 + Sm)))
    lwe[2:-2] += lam * (1.0 - 2.0 * c * av)
    lwe[3:-1] += c * (-v + av) * lam
    lwe[1:-3] += c * (v + av) * lam
    lS[3:-1] += c * lim * (-v + av) * lam
    lS[1:-3] += c * lim * (v + av) * lam
    lS[2:-2] += -2.0 * c * lim * av * lam
    # S[1:-1] = minmod(a, b), a = d[1:], b = d[:-1]
    pos = a * b > 0.0
    pick_a = pos & (np.abs(a) <= np.abs(b))
    pick_b = pos & ~(np.abs(a) <= np.abs(b))
    ld = np.zeros_like(d)
    ld[1:] += np.where(pick_a, lS[1:-1], 0.0)
    ld[:-1] += np.where(pick_b, lS[1:-1], 0.0)
    # d = we[1:] - we[:-1]
    lwe[1:] += ld
    lwe[:-1] -= ld
    return ghosts_vjp(w, lwe, bc_left, bc_right, vx, hv2)


# ----------------------------------------------------------------- one step
def magnetic_vjp(w, B, lam):
    """(grad_w, grad_B) of <lam, 2 (B x w_vec) . sigma>."""
    lw = magnetic(lam, -np.asarray(B, np.float64))          # 2 (lam_vec x B)
    lB = 2.0 * np.cross(w[..., 1:4], lam[..., 1:4]).sum(axis=(1, 2))
    return lw, lB


def rhs_vjp(w, B, lam, L, tables):
    t = tables
    lw = np.stack([collision_pauli_vjp(w[i], lam[i], L, t.R, t.J, t.M, t) for i in range(w.shape[0])])
    mw, mB = magnetic_vjp(w, B, lam)
    return lw + mw, mB


def step_vjp(w, B, dt, lam, L, R, J, M, bc_left, bc_right, tables=None):
    """Transpose of step.step at w[Nx, N, N, 4] applied to lam: returns
    (grad of w, grad of B[Nx, 3])."""
    from .step import rhs
    N = w.shape[1]
    t = tables if tables is not None else Tables(N, L, R, J, M)
    wa = tp.transport_step(w, 0.5 * dt, bc_left, bc_right, L)
    w1 = wa + dt * rhs(wa, B, L, t)
    wb = 0.5 * (wa + w1 + dt * rhs(w1, B, L, t))
    lb = transport_step_vjp(wb, lam, 0.5 * dt, bc_left, bc_right, L)
    # wb = (wa + w1 + dt F(w1)) / 2;  w1 = wa + dt F(wa)
    g1, gB1 = rhs_vjp(w1, B, lb, L, t)
    l1 = 0.5 * lb + 0.5 * dt * g1
    ga, gBa = rhs_vjp(wa, B, l1, L, t)
    la = 0.5 * lb + l1 + dt * ga
    gB = 0.5 * dt * gB1 + dt * gBa
    return transport_step_vjp(w, la, 0.5 * dt, bc_left, bc_right, L), gB


# ----------------------------------------------------------------- trajectories
def observable_weights(g, N, L):
    """Gradient, with respect to the Pauli state, of the final-time observable
    l = dx h^2 sum_j g(x_j) sum_v tr(sigma_z W(x_j, v)) = dx h^2 sum g 2 w3."""
    Nx = g.shape[0]
    h2 = (2.0 * L / N) ** 2
    lam = np.zeros((Nx, N, N, 4))
    lam[..., 3] = 2.0 * h2 / Nx * np.asarray(g)[:, None, None]
    return lam


def trajectory_gradient(w0, B, dt, steps, lam_final, L, R, J, M, bc_left, bc_right, tables=None):
    """Gradient of <lam_final, w(T)> with respect to w0 and B over `steps`
    splitting steps (every state kept; no checkpointing in the oracle)."""
    from .step import step
    N = w0.shape[1]
    t = tables if tables is not None else Tables(N, L, R, J, M)
    states = [w0]
    for _ in range(steps):
        states.append(step(states[-1], B, dt, L, R, J, M, bc_left, bc_right, t))
    lam = lam_final
    gB = np.zeros_like(np.asarray(B, np.float64))
    for n in range(steps - 1, -1, -1):
        lam, g = step_vjp(states[n], B, dt, lam, L, R, J, M, bc_left, bc_right, t)
        gB += g
    return states[-1], lam, gB
