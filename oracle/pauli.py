"""Pauli representation of 2x2 Hermitian Wigner matrices (Sec. 3.1).

W = w0*1 + w1*sigma_1 + w2*sigma_2 + w3*sigma_3 (eq. spin_repr), with the
Pauli matrices of Sec. 2 and the metric eta = diag(1, -1, -1, -1).
"""
import numpy as np

# bold-sigma = (1, sigma_1, sigma_2, sigma_3), Sec. 2 and Sec. 3.1
SIGMA = np.array(
    [
        [[1, 0], [0, 1]],
        [[0, 1], [1, 0]],
        [[0, -1j], [1j, 0]],
        [[1, 0], [0, -1]],
    ],
    dtype=np.complex128,
)

ETA = np.array([1.0, -1.0, -1.0, -1.0])


def to_pauli(W):
    """w_mu = (1/2) Re tr(sigma_mu W) for W[..., 2, 2]; returns w[..., 4].

    For Hermitian W this inverts eq. spin_repr exactly; for any other input
    it returns the components of the Hermitian part (W + W^H)/2.
    """
    W = np.asarray(W, dtype=np.complex128)
    return 0.5 * np.einsum("mab,...ba->...m", SIGMA, W).real


def from_pauli(w):
    """W = sum_mu w_mu sigma_mu for w[..., 4]; returns W[..., 2, 2]."""
    w = np.asarray(w, dtype=np.float64)
    return np.einsum("...m,mab->...ab", w.astype(np.complex128), SIGMA)


def eta_inner(a, b):
    """<a, b>_eta = a^T eta b over the last axis (Sec. 3.1)."""
    return np.einsum("...m,m,...m->...", a, ETA, b)
