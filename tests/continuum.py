"""Direct quadrature of the continuum collision integrals of Sec. 2, used to
pin the oracle.  Shares nothing with the oracle: it evaluates the matrix
integrands of eq. Cc / eq. Heff and eq. Cd (the A[W]_{1234} form) with 2x2
complex matrix products, at single velocity points, for an analytic W.

Carleman variables (Sec. 3.2): v_1 = v, v_3 = v + u, v_4 = v + u',
v_2 = v + u + u', underline-omega = u . u', both u and u' truncated to the
disk B_R.

delta(u.u'):  int du int du' delta(u.u') F = int_0^R dr int_0^{2pi} da
              int_{-R}^{R} dt F(r e_a, t e_a^perp)           (r cancels)
P(1/(u.u')):  u = r e_a, u' = r' e_b gives int dr dr' da P int db
              F / cos(a - b); the principal value in b is taken by folding
              around the two poles b = a + pi/2, a + 3pi/2, which leaves a
              regular integrand (Gauss-Legendre in the fold variable).
"""
import numpy as np

SIG = np.array(
    [[[1, 0], [0, 1]], [[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]],
    dtype=np.complex128,
)


def validation_W(v):
    """eq. validationW: W(v) for v[..., 2]; returns [..., 2, 2]."""
    vx, vy = v[..., 0], v[..., 1]
    c0 = (1.0 / (3 * np.pi)) * (1 + vx) * np.exp(-0.5 * (vx - 0.5) ** 2 - 0.5 * (vy + vx) ** 2)
    c1 = (3 * np.sqrt(6 / 5) / (55 * np.pi)) * (1 - vx - vy / 6) ** 2 * np.exp(
        -(2 * vx + vy) ** 2 / 12 - vy**2 / 10
    )
    c2 = (1.0 / (4 * np.pi * np.sqrt(2))) * np.exp(-((vx - 1) ** 2) / 8 - vy**2 / 4)
    c3 = (9.0 / (56 * np.pi)) * (1 / 3 + vx) ** 2 * np.exp(-((vx - vy) ** 2) / 8 - (vx + 2 * vy) ** 2 / 8)
    return (
        c0[..., None, None] * SIG[0]
        + c1[..., None, None] * SIG[1]
        + c2[..., None, None] * SIG[2]
        + c3[..., None, None] * SIG[3]
    )


def periodized(Wfun, L):
    """W on the torus [-L, L)^2 (the periodization of Sec. 3.2)."""
    return lambda v: Wfun(np.mod(v + L, 2 * L) - L)


def _tr(A):
    return A[..., 0, 0] + A[..., 1, 1]


def _mm(A, B):
    return np.einsum("...ab,...bc->...ac", A, B)


def _I(shape):
    return np.broadcast_to(np.eye(2, dtype=np.complex128), shape + (2, 2))


def A_form(W1, W2, W3, W4):
    """A[W]_{1234} of eq. Cd."""
    I = _I(W1.shape[:-2])
    Wt2, Wt4 = I - W2, I - W4
    t = -_mm(_mm(W4, Wt2), W3) + W4 * _tr(_mm(Wt2, W3))[..., None, None]
    inner = (
        _mm(Wt4, W3)
        - _mm(Wt4, W2)
        - _mm(Wt2, W3)
        + Wt4 * _tr(W2)[..., None, None]
        - Wt4 * _tr(W3)[..., None, None]
        + I * _tr(_mm(W3, Wt2))[..., None, None]
    )
    return t - _mm(inner, W1)


def heff_integrand(W2, W3, W4):
    """Integrand of eq. Heff."""
    return (
        _mm(W3, W4)
        - _mm(W2, W3)
        - _mm(W3, W2)
        - W3 * _tr(W4)[..., None, None]
        + W3 * _tr(W2)[..., None, None]
        + W2
    )


def _gl(n, a, b):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def Cd_at(W, v, R, n_r=48, n_a=96, n_t=64):
    """C_d[W](v) (eq. Cd) by tensor quadrature of the delta-reduced integral."""
    r, wr = _gl(n_r, 0.0, R)
    t, wt = _gl(n_t, -R, R)
    a = 2 * np.pi * np.arange(n_a) / n_a
    wa = np.full(n_a, 2 * np.pi / n_a)
    e = np.stack([np.cos(a), np.sin(a)], -1)               # [a, 2]
    ep = np.stack([-np.sin(a), np.cos(a)], -1)
    u = r[:, None, None, None] * e[None, :, None, :]        # [r, a, 1, 2]
    up = t[None, None, :, None] * ep[None, :, None, :]      # [1, a, t, 2]
    v = np.asarray(v, float)
    W1 = W(v[None, None, None, :])
    W3 = W(v + u)
    W4 = W(v + up)
    W2 = W(v + u + up)
    shp = np.broadcast_shapes(W3.shape[:-2], W4.shape[:-2])
    W1 = np.broadcast_to(W1, shp + (2, 2))
    W3 = np.broadcast_to(W3, shp + (2, 2))
    W4 = np.broadcast_to(W4, shp + (2, 2))
    Af = A_form(W1, W2, W3, W4)
    integrand = Af + np.conj(np.swapaxes(Af, -1, -2))
    wts = wr[:, None, None] * wa[None, :, None] * wt[None, None, :]
    return np.pi * np.einsum("rat,ratxy->xy", wts, integrand)


def Cc_at(W, v, R, n_r=40, n_a=64, n_s=40):
    """C_c[W](v) = -i [H_eff(v), W(v)] (eq. Cc, eq. Heff), principal value
    taken by folding around the poles of 1/cos(a - b)."""
    r, wr = _gl(n_r, 0.0, R)
    s, ws = _gl(n_s, 0.0, np.pi / 2)
    a = 2 * np.pi * np.arange(n_a) / n_a
    wa = np.full(n_a, 2 * np.pi / n_a)
    v = np.asarray(v, float)
    H = np.zeros((2, 2), dtype=np.complex128)
    ea = np.stack([np.cos(a), np.sin(a)], -1)
    u = r[:, None, None, None] * ea[None, :, None, :]       # [r, a, 1, 2]
    W3 = W(v + u)
    for pole, sgn in ((np.pi / 2, -1.0), (3 * np.pi / 2, +1.0)):
        # 1/cos(a - b) at b = a + pole + s equals sgn / sin(s)
        for side in (+1.0, -1.0):
            b = a[:, None] + pole + side * s[None, :]        # [a, s]
            eb = np.stack([np.cos(b), np.sin(b)], -1)        # [a, s, 2]
            for k in range(len(r)):
                up = r[k] * eb[None, :, :, :]               # [1, a, s, 2]
                W4 = W(v + up)
                W2 = W(v + u + up)                          # [r, a, s]
                W3b = np.broadcast_to(W3, W2.shape)
                W4b = np.broadcast_to(W4, W2.shape)
                K = heff_integrand(W2, W3b, W4b)
                # odd fold: (g(+s) - g(-s)) / sin(s), times sgn
                wts = (
                    wr[:, None, None] * wr[k] * wa[None, :, None]
                    * (ws / np.sin(s))[None, None, :] * sgn * side
                )
                H += np.einsum("ras,rasxy->xy", wts, K)
    W1 = W(v)
    return -1j * (H @ W1 - W1 @ H)
