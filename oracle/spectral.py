"""Fourier grids and naive DFTs (Sec. 3.2, eq. fourier_grid; Sec. 5.1).

Velocity grid: v_n = (2L/N) n for n in Xi = [-N/2, N/2-1]^2 (Sec. 5.1); array
index i along an axis holds n = i - N/2.  The first array axis is v_x.

Mean-value Fourier coefficients (Sec. 3.2):
    f_hat(xi) = N^-2 sum_n f(v_n) exp(-2 pi i xi . n / N),   xi in Xi,
so that f(v) = sum_xi f_hat(xi) exp(i pi xi . v / L).

Padded grid for the convolutions ("double zero padding", Sec. 3.2):
P = 2N points per axis, frequencies b in [-N, N-1]^2, real-space points
v'_p = (L/N) p with p in [-N, N-1]^2 (half the velocity spacing).  Products
of band-limited functions on this grid are exact cyclic convolutions of
their coefficient arrays; every convolution below is evaluated that way.

All transforms are dense DFT matrices applied with matrix products.

Reading (Nyquist rule): Xi has an unpaired frequency -N/2 per axis.  The
coefficients with xi_x = -N/2 or xi_y = -N/2 are set to zero on input and
on output, so that every real-space intermediate is real.
"""
import numpy as np


def freqs(N):
    """Integer frequencies of Xi along one axis: -N/2 .. N/2-1."""
    return np.arange(N) - N // 2


def pfreqs(N):
    """Integer frequencies of the padded grid along one axis: -N .. N-1."""
    return np.arange(2 * N) - N


def velocity_axis(N, L):
    """v along one axis: (2L/N) * (i - N/2)."""
    return (2.0 * L / N) * freqs(N)


def _dft_matrix(kf, nf, n_period, sign):
    return np.exp(sign * 2j * np.pi * np.outer(kf, nf) / n_period)


def _apply2(A, X, B):
    """A @ X @ B^T over the last two axes of a stack X[..., n, m]."""
    X = np.asarray(X, dtype=np.complex128)
    lead = X.shape[:-2]
    n, m = X.shape[-2:]
    Y = (X.reshape(-1, m) @ B.T).reshape(lead + (n, B.shape[0]))
    Y = np.swapaxes(Y, -1, -2)
    k = Y.shape[-2]
    Z = (Y.reshape(-1, n) @ A.T).reshape(lead + (k, A.shape[0]))
    return np.swapaxes(Z, -1, -2)


def dft_N(f):
    """f_hat on Xi from samples f[..., N, N] on the velocity grid."""
    N = f.shape[-1]
    F = _dft_matrix(freqs(N), freqs(N), N, -1.0)
    return _apply2(F, f, F) / N**2


def idft_N(fhat):
    """Samples on the velocity grid of sum_{xi in Xi} f_hat(xi) e^{2 pi i xi.n/N}."""
    N = fhat.shape[-1]
    E = _dft_matrix(freqs(N), freqs(N), N, +1.0)
    return _apply2(E, fhat, E)


def dft_P(g):
    """Coefficients on [-N, N-1]^2 of samples g[..., 2N, 2N] on the padded grid."""
    P = g.shape[-1]
    N = P // 2
    F = _dft_matrix(pfreqs(N), pfreqs(N), P, -1.0)
    return _apply2(F, g, F) / P**2


def idft_P(ghat):
    """Samples on the padded grid of sum_b g_hat(b) e^{2 pi i b.p/P}."""
    P = ghat.shape[-1]
    N = P // 2
    E = _dft_matrix(pfreqs(N), pfreqs(N), P, +1.0)
    return _apply2(E, ghat, E)


def pad(fhat):
    """Embed coefficients on Xi into the padded frequency grid (zeros elsewhere)."""
    N = fhat.shape[-1]
    out = np.zeros(fhat.shape[:-2] + (2 * N, 2 * N), dtype=np.complex128)
    out[..., N // 2 : N // 2 + N, N // 2 : N // 2 + N] = fhat
    return out


def truncate(ghat):
    """Restrict coefficients on the padded grid to Xi."""
    P = ghat.shape[-1]
    N = P // 2
    return ghat[..., N // 2 : N // 2 + N, N // 2 : N // 2 + N]


def zero_nyquist(fhat):
    """Reading: zero the unpaired frequency -N/2 along each axis (copy)."""
    out = np.array(fhat, dtype=np.complex128, copy=True)
    out[..., 0, :] = 0.0
    out[..., :, 0] = 0.0
    return out


def delta_hat(N):
    """Coefficients of the constant function 1 on Xi."""
    d = np.zeros((N, N), dtype=np.complex128)
    d[N // 2, N // 2] = 1.0
    return d


def conv(ahat, bhat):
    """Linear convolution (a * b)(k) = sum_q a(q) b(k - q) of two coefficient
    arrays given on the padded grid whose supports sum inside the padded
    range: the product of their padded-grid samples, transformed back."""
    return dft_P(idft_P(ahat) * idft_P(bhat))
