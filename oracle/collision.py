"""Collision operator C[W] = C_c[W] + C_d[W] by the fast spectral method of
Sec. 3.2, evaluated literally: naive DFTs, direct sums over the quadrature
indices, one convolution at a time, in the order the paper gives.

Carleman variables (Sec. 3.2): v_1 = v, v_3 = v + u, v_4 = v + u',
v_2 = v + u + u', and omega(v) = |v|^2 / 2 gives underline-omega = u . u'.

Integral types (Sec. 3.2), for functions f, g, h of v:
  I_1 = int P(1/(u.u')) f(v+u) g(v+u+u') h(v)     kernel G(chi+eta, eta)
  I_2 = int delta(u.u') f(v+u) g(v+u')   h(v)     kernel H(chi, eta)
  I_3 = int delta(u.u') f(v+u) g(v+u')   h(v+u+u') kernel H(chi+zeta, eta+zeta)
  I_4 = int delta(u.u') f(v+u) g(v+u+u') h(v)     kernel H(chi+eta, eta)
with G approximated by eq. approxG (J x J angles), H by eq. approxH-J (J
angles) for I_2 and I_4, and by eq. approxH-JM (J angles, M Gauss-Legendre
radii) for I_3.  In Fourier variables each I_k is a sum over
chi + eta + zeta = xi of f_hat(chi) g_hat(eta) h_hat(zeta) times its kernel;
the result is kept on xi in Xi.

Pauli assembly (eq. CcPauli, eq. CdPauli and their Carleman forms, with the
identities of Sec. 3.1: -i[W_2, W_1] = 2 (w_2 x w_1) . sigma and the
anticommutator formula), with f0 = 2 w0 - 1, eps the Levi-Civita symbol and
eta = diag(1, -1, -1, -1):
  C_c,0 = 0,   C_c,k = -2 sum_{l,m} eps_klm I_1[f0, w_l, w_m]
  C_d = pi (A + B + Cq) where
    A_0  =  2 sum_mu eta_mu I_2[w_mu, w_mu, 1 - w0]
    A_k  = -2 sum_mu eta_mu I_2[w_mu, w_mu, w_k]
    B_0  = -2 sum_mu eta_mu I_3[w_mu, w_mu, w0]
    B_k  =  2 sum_mu eta_mu I_3[w_mu, w_mu, w_k]
    Cq_0 =  2 (I_4[f0, w0, w0] - sum_k I_4[f0, w_k, w_k])
    Cq_k =  2 (I_4[f0, w0, w_k] - I_4[f0, w_k, w0])
(A: the term 2<w_3, w_4>_eta (1 - W_1); B: -2<w_3, w_4>_eta (eta w_2).sigma;
Cq: (2 w0(v+u) - 1) {W_1, (eta w_2).sigma}.)
"""
import numpy as np

from . import quadrature as qd
from . import spectral as sp
from .pauli import ETA, from_pauli, to_pauli

LEVI_CIVITA = np.zeros((3, 3, 3))
LEVI_CIVITA[0, 1, 2] = LEVI_CIVITA[1, 2, 0] = LEVI_CIVITA[2, 0, 1] = 1.0
LEVI_CIVITA[0, 2, 1] = LEVI_CIVITA[2, 1, 0] = LEVI_CIVITA[1, 0, 2] = -1.0


class Tables:
    """The 1D quadrature functions evaluated on the padded frequency grid
    b in [-N, N-1]^2 (phi_{R,j}, phi'_{R,j}, psi_{R,j}, psi'_{R,j}) and the
    weights of eq. approxG, approxH-J, approxH-JM."""

    def __init__(self, N, L, R, J, M):
        self.N, self.L, self.R, self.J, self.M = N, L, R, J, M
        b = sp.pfreqs(N).astype(np.float64)
        bx, by = np.meshgrid(b, b, indexing="ij")
        th, thp = qd.theta(J), qd.theta_prime(J)
        thr = qd.rot90(th)
        proj = lambda t: bx[None] * t[:, 0, None, None] + by[None] * t[:, 1, None, None]
        self.phi = qd.phi_R(proj(th), L, R)        # phi_{R,j}(b)
        self.phip = qd.phi_R(proj(thp), L, R)      # phi'_{R,j}(b)
        self.psi = qd.psi_R(proj(th), L, R)        # psi_{R,j}(b)
        self.psip = qd.psi_R(proj(thr), L, R)      # psi'_{R,j}(b)
        self.omega_G = qd.omega_G(J)
        self.omega_H = qd.omega_H(J)
        self.rho, self.wgl = qd.gauss_legendre(M, R)
        self.theta = th
        self._bx, self._by = bx, by

    def modulation(self, j, m):
        """exp(i alpha_{j,m} . b), alpha_{j,m} = pi rho_m theta_j / L, on the
        padded grid; m may be an index array (leading axis)."""
        a = np.pi * np.atleast_1d(self.rho[m]) / self.L
        ax = a[:, None, None] * self.theta[j, 0]
        ay = a[:, None, None] * self.theta[j, 1]
        return np.exp(1j * (ax * self._bx[None] + ay * self._by[None]))


def form_I1(t, fh, gh, hh):
    """I_1[f, g_a, h_b] on Xi for f_hat[N,N], g_hat[A,N,N], h_hat[B,N,N];
    returns [A, B, N, N].  Follows the last display of the G scheme: for each
    (j, j'), the inner convolution f_hat * (phi'_{j'} g_hat), times phi_j,
    then the outer convolution with h_hat, weighted by omega_{G,j,j'}."""
    F, G, H = sp.pad(fh), sp.pad(gh), sp.pad(hh)
    A, B = G.shape[0], H.shape[0]
    out = np.zeros((A, B) + fh.shape, dtype=np.complex128)
    h_real = sp.idft_P(H)                                           # [B, P, P]
    for jp in range(t.J):
        inner = sp.conv(F[None], t.phip[jp][None] * G)              # [A, P, P]
        for j in range(t.J):
            x = sp.idft_P(t.phi[j][None] * inner)                   # [A, P, P]
            outer = sp.truncate(sp.dft_P(x[:, None] * h_real[None]))  # [A, B, N, N]
            out += t.omega_G[j, jp] * outer
    return out


def form_I2(t, fh, gh, hh):
    """I_2[f_a, g_a, h_b] for paired f_hat[A,N,N], g_hat[A,N,N] and
    h_hat[B,N,N]; returns [A, B, N, N].  For each j: the products
    psi_j f_hat and psi'_j g_hat, their convolution, then the convolution
    with h_hat (the double convolution of the I_2 scheme), weight pi/J."""
    F, G, H = sp.pad(fh), sp.pad(gh), sp.pad(hh)
    out = np.zeros((F.shape[0], H.shape[0]) + fh.shape[1:], dtype=np.complex128)
    for j in range(t.J):
        a = sp.conv(t.psi[j][None] * F, t.psip[j][None] * G)       # [A, P, P]
        out += t.omega_H[j] * sp.truncate(sp.conv(a[:, None], H[None]))
    return out


def form_I4(t, fh, gh, hh):
    """I_4[f, g_a, h_b] for f_hat[N,N], g_hat[A,N,N], h_hat[B,N,N]; returns
    [A, B, N, N].  Same scheme as I_1 with H_J(chi+eta, eta) =
    sum_j (pi/J) psi_j(chi+eta) psi'_j(eta): inner convolution
    f_hat * (psi'_j g_hat), times psi_j, outer convolution with h_hat."""
    F, G, H = sp.pad(fh), sp.pad(gh), sp.pad(hh)
    out = np.zeros((G.shape[0], H.shape[0]) + fh.shape, dtype=np.complex128)
    h_real = sp.idft_P(H)                                           # [B, P, P]
    for j in range(t.J):
        inner = sp.conv(F[None], t.psip[j][None] * G)               # [A, P, P]
        x = sp.idft_P(t.psi[j][None] * inner)                       # [A, P, P]
        out += t.omega_H[j] * sp.truncate(sp.dft_P(x[:, None] * h_real[None]))
    return out


def form_I3(t, fh, gh, hh, m_chunk=8):
    """I_3[f_a, g_a, h_b] for paired f_hat[A,N,N], g_hat[A,N,N] and
    h_hat[B,N,N]; returns [A, B, N, N].  Scheme of eq. approxH-JM: for each
    (j, m), the modulated arrays exp(i alpha_jm . chi) f_hat and
    exp(i alpha_jm . zeta) h_hat, the inner convolution g_hat * (mod h_hat),
    times psi'_j, the outer convolution with (mod f_hat), weight
    (pi/J) w_{R,m}."""
    F, G, H = sp.pad(fh), sp.pad(gh), sp.pad(hh)
    A, B = F.shape[0], H.shape[0]
    out = np.zeros((A, B) + fh.shape[1:], dtype=np.complex128)
    for j in range(t.J):
        for m0 in range(0, t.M, m_chunk):
            ms = np.arange(m0, min(m0 + m_chunk, t.M))
            E = t.modulation(j, ms)                                  # [m, P, P]
            EF = E[:, None] * F[None]                           # [m, A, P, P]
            EH = E[:, None] * H[None]                           # [m, B, P, P]
            inner = sp.conv(G[None, :, None], EH[:, None, :])        # [m, A, B, P, P]
            inner = t.psip[j] * inner
            outer = sp.truncate(sp.conv(EF[:, :, None], inner))      # [m, A, B, N, N]
            wts = t.omega_H[j] * t.wgl[ms]
            out += np.tensordot(wts, outer, axes=(0, 0))
    return out


def pauli_hat(W):
    """w_hat_mu on Xi for W[N, N, 2, 2], Nyquist rows/columns zeroed."""
    w = to_pauli(W)                                  # [N, N, 4]
    return sp.zero_nyquist(sp.dft_N(np.moveaxis(w, -1, 0)))


def collision_hat(what, t, parts=False):
    """C_hat on Xi ([4, N, N], Pauli components) from w_hat[4, N, N]."""
    N = what.shape[-1]
    one = sp.delta_hat(N)
    f0 = 2.0 * what[0] - one
    w = what
    C = np.zeros((4, N, N), dtype=np.complex128)

    # conservative part: C_c,k = -2 sum eps_klm I_1[f0, w_l, w_m]
    T1 = form_I1(t, f0, w[1:4], w[1:4])                   # [l, m]
    Cc = np.zeros_like(C)
    Cc[1:4] = -2.0 * np.einsum("klm,lmxy->kxy", LEVI_CIVITA, T1)

    # term A: 2 <w(v+u), w(v+u')>_eta (1 - W(v))
    hA = np.stack([one - w[0], w[1], w[2], w[3]])
    T2 = form_I2(t, w, w, hA)                             # [mu, h]
    S2 = np.einsum("m,mhxy->hxy", ETA, T2)
    Aq = np.concatenate([2.0 * S2[:1], -2.0 * S2[1:]])

    # term B: -2 <w(v+u), w(v+u')>_eta (eta w(v+u+u')) . sigma
    T3 = form_I3(t, w, w, w)                              # [mu, nu]
    S3 = np.einsum("m,mnxy->nxy", ETA, T3)
    Bq = np.concatenate([-2.0 * S3[:1], 2.0 * S3[1:]])

    # term C: (2 w0(v+u) - 1) {W(v), (eta w(v+u+u')) . sigma}
    T4 = form_I4(t, f0, w, w)                             # [g, h]
    Cq = np.zeros_like(C)
    Cq[0] = 2.0 * (T4[0, 0] - T4[1, 1] - T4[2, 2] - T4[3, 3])
    for k in range(1, 4):
        Cq[k] = 2.0 * (T4[0, k] - T4[k, 0])

    Cd = np.pi * (Aq + Bq + Cq)
    if parts:
        return {"Cc": Cc, "A": np.pi * Aq, "B": np.pi * Bq, "C": np.pi * Cq}
    return Cc + Cd


def collision_pauli(w, L, R, J, M, tables=None):
    """C[W] in Pauli components on the velocity grid: w[N, N, 4] -> c[N, N, 4]."""
    N = w.shape[0]
    t = tables if tables is not None else Tables(N, L, R, J, M)
    what = sp.zero_nyquist(sp.dft_N(np.moveaxis(np.asarray(w, np.float64), -1, 0)))
    Ch = sp.zero_nyquist(collision_hat(what, t))
    return np.moveaxis(sp.idft_N(Ch).real, 0, -1)


def collision(W, L, R, J, M, tables=None):
    """C[W] for one spatial cell: W[N, N, 2, 2] complex -> C[N, N, 2, 2]."""
    return from_pauli(collision_pauli(to_pauli(W), L, R, J, M, tables))
