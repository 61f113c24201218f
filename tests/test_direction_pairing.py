"""The identity behind the direction pairs of the I_1 / I_4 kernels (two
directions j, j+1 per complex transform), checked with numpy FFTs on the
oracle's own kernel tables (Sec. 3.2): the 1D kernels have fixed parities
(phi_R odd, psi_R even), so for the spectrum of a real field on Xi the
paired evaluation reproduces the per-direction one away from the padded
grid's Nyquist lines, which the collision never reads back (they only meet
the output after a product with a field limited to Xi).  The GPU kernels
themselves are compared with the oracle by the -m gpu parity tests."""
import numpy as np

from oracle import collision as oc
from oracle import quadrature as qd


def test_kernel_parities():
    """phi_R (int_0^R sin) is odd and psi_R (int_-R^R exp) is even."""
    x = np.linspace(-9.1, 9.1, 363)
    for L, R in ((12.0, 7.5), (5.0, 3.0)):
        assert np.abs(qd.phi_R(-x, L, R) + qd.phi_R(x, L, R)).max() < 1e-13
        assert np.abs(qd.psi_R(-x, L, R) - qd.psi_R(x, L, R)).max() < 1e-13


def _setup(N=8, J=8, L=5.0, R=3.0, seed=3):
    t = oc.Tables(N, L, R, J, 4)
    P = 2 * N
    fft_order = lambda a: np.fft.ifftshift(a, axes=(-2, -1))
    b = np.fft.fftfreq(P, 1.0 / P)
    kx, ky = np.meshgrid(b, b, indexing="ij")
    xi = (np.abs(kx) < N // 2) & (np.abs(ky) < N // 2)
    nyq = (kx == -N) | (ky == -N)
    rng = np.random.default_rng(seed)
    # spectrum of a real field, supported on Xi
    w = rng.standard_normal((P, P))
    what = np.where(xi, np.fft.fft2(w), 0.0)
    what = 0.5 * (what + np.conj(what[(-np.arange(P)) % P][:, (-np.arange(P)) % P]))
    f0 = np.fft.ifft2(np.where(xi, np.fft.fft2(rng.standard_normal((P, P))), 0)).real
    tabs = {"odd": (fft_order(t.phip), fft_order(t.phi)), "even": (fft_order(t.psip), fft_order(t.psi))}
    return what, f0, tabs, nyq, J


def test_paired_directions_reproduce_the_field():
    fwd2, inv2 = np.fft.fft2, np.fft.ifft2
    what, f0, tabs, nyq, J = _setup()
    for parity, (tin, tout) in tabs.items():
        odd = parity == "odd"
        # per direction: field = Re inv2(sum_j out_j fwd2(f0 inv2(in_j w_hat)))
        acc = sum(tout[j] * fwd2(f0 * inv2(tin[j] * what)) for j in range(J))
        # two directions per transform, coefficients as in k_terms
        acc2 = 0
        for j in range(0, J, 2):
            i1, i2, o1, o2 = tin[j], tin[j + 1], tout[j], tout[j + 1]
            cin = (i2 - 1j * i1) if odd else (i1 + 1j * i2)
            cout = (o2 + 1j * o1) if odd else (o1 - 1j * o2)
            acc2 = acc2 + cout * fwd2(f0 * inv2(cin * what))
        F1, F2 = fwd2(inv2(acc).real), fwd2(inv2(acc2).real)
        scale = np.abs(F1).max()
        assert np.abs(F1 - F2)[~nyq].max() < 1e-12 * scale, parity
        # the per-direction transforms are real (up to the table's phase),
        # which is what the sharing rests on
        a = inv2(tin[0] * what)
        assert np.abs((a.imag if not odd else a.real)).max() < 1e-13 * np.abs(a).max()


def test_paired_cotangent_is_the_hermitian_part():
    """The reverse pairs: H = sum over pairs of cw conj(fwd2(f0 B)) with
    B = inv2(cb D) has the cotangent of w_hat as its Hermitian part
    (H(k) + conj H(-k)) / 2, as k_grad_pre takes it."""
    fwd2 = np.fft.fft2
    inv2 = lambda z: np.fft.ifft2(z) * z.shape[-1] * z.shape[-2]
    what, f0, tabs, nyq, J = _setup(seed=5)
    P = what.shape[0]
    rng = np.random.default_rng(11)
    fbar = inv2(np.where(np.abs(what) > 0, rng.standard_normal((P, P)), 0)).real * inv2(what).real
    D = fwd2(fbar)
    neg = (-np.arange(P)) % P
    for parity, (tin, tout) in tabs.items():
        odd = parity == "odd"
        wb, H = 0, 0
        for j in range(J):
            b = np.conj(inv2(np.conj(tout[j] * np.conj(D))))
            wb = wb + tin[j] * np.conj(fwd2(np.conj(f0 * b)))
        for j in range(0, J, 2):
            i1, i2, o1, o2 = tin[j], tin[j + 1], tout[j], tout[j + 1]
            cb = (1j * o1 - o2) if odd else (o1 + 1j * o2)
            cw = (1j * i1 - i2) if odd else (i1 + 1j * i2)
            H = H + cw * np.conj(fwd2(f0 * inv2(cb * D)))
        sym = 0.5 * (H + np.conj(H[neg][:, neg]))
        assert np.abs(sym - wb)[~nyq].max() < 1e-12 * np.abs(wb).max(), parity
