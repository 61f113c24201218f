"""Brute-force evaluation of the discrete collision operator in matrix form,
used to pin the oracle on tiny grids.  Independent of the oracle: no Pauli
algebra, no FFT or padding; direct sums over Fourier triples.

The scheme of Sec. 3.2 replaces every integral over (u, u') by a sum over
Fourier modes xi_i of the fields at the points v_1 = v, v_2 = v + u + u',
v_3 = v + u, v_4 = v + u' with the kernel K(xi_2 + xi_3, xi_2 + xi_4):
  * C_c: the Carleman form eq. CcPauliCarleman,
        i (2 w0(v+u) - 1) (W(v+u+u') W(v) - W(v) W(v+u+u')),
    kernel G_J (eq. approxG);
  * C_d: pi (A + A*) of eq. Cd, symmetrized over v_3 <-> v_4, kernel H_JM
    (eq. approxH-JM) for the products that involve v_2, v_3 and v_4 together
    (the I_3 type) and H_J (eq. approxH-J) for all others.
Each integrand is affine in each W_i, so its part that depends on exactly
the points in S is extracted by inclusion-exclusion and summed over the
Fourier modes of those points.
"""
import itertools

import numpy as np

SIG = np.array(
    [[[1, 0], [0, 1]], [[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]],
    dtype=np.complex128,
)
I2 = np.eye(2, dtype=np.complex128)


def _mm(A, B):
    return np.einsum("...ab,...bc->...ac", A, B)


def _tr(A):
    return (A[..., 0, 0] + A[..., 1, 1])[..., None, None]


def A_poly(W1, W2, W3, W4):
    Wt2, Wt4 = I2 - W2, I2 - W4
    inner = (_mm(Wt4, W3) - _mm(Wt4, W2) - _mm(Wt2, W3)
             + Wt4 * _tr(W2) - Wt4 * _tr(W3) + I2 * _tr(_mm(W3, Wt2)))
    return -_mm(_mm(W4, Wt2), W3) + W4 * _tr(_mm(Wt2, W3)) - _mm(inner, W1)


def A_dag_poly(W1, W2, W3, W4):
    """Polynomial equal to A(W)^H whenever every W_i is Hermitian."""
    Wt2, Wt4 = I2 - W2, I2 - W4
    inner_dag = (_mm(W3, Wt4) - _mm(W2, Wt4) - _mm(W3, Wt2)
                 + Wt4 * _tr(W2) - Wt4 * _tr(W3) + I2 * _tr(_mm(W3, Wt2)))
    return -_mm(_mm(W3, Wt2), W4) + W4 * _tr(_mm(Wt2, W3)) - _mm(W1, inner_dag)


def Fd(W1, W2, W3, W4):
    s = A_poly(W1, W2, W3, W4) + A_dag_poly(W1, W2, W3, W4)
    t = A_poly(W1, W2, W4, W3) + A_dag_poly(W1, W2, W4, W3)
    return 0.5 * (s + t)


def Fc(W1, W2, W3, W4):
    f0 = _tr(W3) - 1.0         # 2 w0(v+u) - 1, with 2 w0 = tr W
    return 1j * f0 * (_mm(W2, W1) - _mm(W1, W2))


def _phi(x, L, R):
    out = np.zeros_like(x)
    nz = x != 0
    out[nz] = 2 * L / (np.pi * x[nz]) * np.sin(np.pi * R * x[nz] / (2 * L)) ** 2
    return out


def _psi(x, L, R):
    out = np.full_like(x, 2.0 * R)
    nz = x != 0
    out[nz] = 2 * L / (np.pi * x[nz]) * np.sin(np.pi * R * x[nz] / L)
    return out


def kernels(L, R, J, M):
    """Functions of integer frequency pairs (a[..., 2], b[..., 2])."""
    ang = np.pi * np.arange(J) / J
    angp = np.pi * (np.arange(J) + 0.5) / J
    th = np.stack([np.cos(ang), np.sin(ang)], -1)
    thp = np.stack([np.cos(angp), np.sin(angp)], -1)
    thr = np.stack([-np.sin(ang), np.cos(ang)], -1)
    wG = -((2 * np.pi / J) ** 2) / np.cos(ang[:, None] - angp[None, :])
    x, w = np.polynomial.legendre.leggauss(M)
    rho, wm = R * x, R * w

    def G(a, b):
        pa = _phi(a @ th.T, L, R)            # [..., J]
        pb = _phi(b @ thp.T, L, R)
        return np.einsum("...j,jk,...k->...", pa, wG, pb)

    def HJ(a, b):
        return (np.pi / J) * np.sum(_psi(a @ th.T, L, R) * _psi(b @ thr.T, L, R), -1)

    def HJM(a, b):
        ph = np.exp(1j * np.pi * rho[:, None] * (a @ th.T)[..., None, :] / L)   # [..., M, J]
        s = np.einsum("m,...mj->...j", wm, ph)
        return (np.pi / J) * np.sum(s * _psi(b @ thr.T, L, R), -1)

    return G, HJ, HJM


def matrix_coeffs(W):
    """W_hat(xi) = N^-2 sum_n W(v_n) e^{-2 pi i xi.n/N} by direct summation,
    Nyquist rows/columns zeroed; W[N, N, 2, 2] -> [N, N, 2, 2]."""
    N = W.shape[0]
    k = np.arange(N) - N // 2
    E = np.exp(-2j * np.pi * np.outer(k, k) / N)
    out = np.einsum("ai,bj,ijxy->abxy", E, E, W) / N**2
    out[0, :] = 0
    out[:, 0] = 0
    return out


def collision_hat(W, L, R, J, M):
    """C_hat(xi) on Xi as 2x2 matrices (before the output Nyquist rule)."""
    N = W.shape[0]
    Wh = matrix_coeffs(W)
    G, HJ, HJM = kernels(L, R, J, M)
    k = np.arange(N) - N // 2
    modes = np.stack(np.meshgrid(k, k, indexing="ij"), -1).reshape(-1, 2)  # [N^2, 2]
    coef = Wh.reshape(-1, 2, 2)
    out = np.zeros((N, N, 2, 2), dtype=np.complex128)
    zero = np.zeros((2, 2), dtype=np.complex128)

    for S_size in range(0, 4):
        for S in itertools.combinations((1, 2, 3, 4), S_size):
            # modes of the points in S: all combinations
            if S:
                idx = np.array(list(itertools.product(range(len(modes)), repeat=len(S))),
                               dtype=np.int64)
            else:
                idx = np.zeros((1, 0), dtype=np.int64)
            xi = {p: modes[idx[:, n]] for n, p in enumerate(S)}
            tot = sum(xi.values()) if S else np.zeros((1, 2), np.int64)
            keep = np.all((tot >= -N // 2) & (tot <= N // 2 - 1), axis=-1)
            idx = idx[keep]
            xi = {p: v[keep] for p, v in xi.items()}
            tot = tot[keep]
            cnt = len(idx) if S else 1
            zeros2 = lambda p: xi[p] if p in xi else np.zeros((cnt, 2), np.int64)
            a = (zeros2(2) + zeros2(3)).astype(float)
            b = (zeros2(2) + zeros2(4)).astype(float)
            # multilinear part in exactly the points S (inclusion-exclusion)
            def evalF(F, T):
                args = []
                for p in (1, 2, 3, 4):
                    if p in T:
                        args.append(coef[idx[:, S.index(p)]])
                    else:
                        args.append(np.broadcast_to(zero, (cnt, 2, 2)))
                return F(*args)
            part_c = np.zeros((cnt, 2, 2), dtype=np.complex128)
            part_d = np.zeros((cnt, 2, 2), dtype=np.complex128)
            for r in range(len(S) + 1):
                for T in itertools.combinations(S, r):
                    sgn = (-1) ** (len(S) - r)
                    part_c += sgn * evalF(Fc, T)
                    part_d += sgn * evalF(Fd, T)
            kd = HJM(a, b) if {2, 3, 4} <= set(S) else HJ(a, b)
            kc = G(a, b)
            contrib = kc[:, None, None] * part_c + np.pi * kd[:, None, None] * part_d
            oi = tot + N // 2
            np.add.at(out, (oi[:, 0], oi[:, 1]), contrib)
    return out
