"""Time-splitting step (Sec. 4) and fluid moments (Sec. 2).

One step of length dt:  half a step of transport, the collision and the
magnetic field together, half a step of transport.
Reading: the paper does not name the integrator of the middle sub-step; it
is one Heun (two-stage second-order Runge-Kutta) step of length dt for
dW/dt = C[W] - i[B . sigma, W], per spatial cell.
The field term in Pauli components: -i[B . sigma, W] = 2 (B x w_vec) . sigma
(commutator identity of Sec. 3.1), w0 unchanged.
"""
import numpy as np

from . import transport as tp
from .collision import Tables, collision_pauli


def magnetic(w, B):
    """2 (B x w_vec) as Pauli components, w[Nx, N, N, 4], B[Nx, 3]."""
    out = np.zeros_like(w)
    Bb = np.asarray(B, np.float64)[:, None, None, :]
    out[..., 1:4] = 2.0 * np.cross(np.broadcast_to(Bb, w[..., 1:4].shape), w[..., 1:4])
    return out


def rhs(w, B, L, tables):
    """C[W] + field term per cell."""
    c = np.stack([collision_pauli(w[i], L, tables.R, tables.J, tables.M, tables) for i in range(w.shape[0])])
    return c + magnetic(w, B)


def heun(w, B, dt, L, tables):
    """Heun step of length dt."""
    w1 = w + dt * rhs(w, B, L, tables)
    return 0.5 * (w + w1 + dt * rhs(w1, B, L, tables))


def rotate(w, B, tau):
    """Exact flow of the field term over time tau: dw/dt = 2 B x w (w0
    fixed) turns the Bloch vector about B(x) by the angle 2 |B| tau
    (Rodrigues' rotation formula)."""
    B = np.asarray(B, np.float64)
    nb = np.linalg.norm(B, axis=-1)
    th = 2.0 * nb * tau
    k = np.where(nb[:, None] > 0, B / np.where(nb > 0, nb, 1.0)[:, None], 0.0)[:, None, None, :]
    c, s = np.cos(th)[:, None, None, None], np.sin(th)[:, None, None, None]
    v = w[..., 1:]
    kv = np.sum(k * v, axis=-1, keepdims=True)
    out = w.copy()
    out[..., 1:] = v * c + np.cross(k, v) * s + k * kv * (1.0 - c)
    return out


def step(w, B, dt, L, R, J, M, bc_left, bc_right, tables=None, limiter="minmod", field="heun"):
    """T(dt/2) o Heun(dt) o T(dt/2) for w[Nx, N, N, 4].

    Variants (Sec. 4): `limiter` selects the slope limiter of the transport
    half-steps; field="rotation" takes the field term out of the Heun step
    and applies its exact flow for dt/2 on either side of it,
    T(dt/2) o F(dt/2) o Heun_C(dt) o F(dt/2) o T(dt/2)."""
    N = w.shape[1]
    t = tables if tables is not None else Tables(N, L, R, J, M)
    w = tp.transport_step(w, 0.5 * dt, bc_left, bc_right, L, limiter)
    if field == "rotation":
        w = rotate(w, B, 0.5 * dt)
        w = heun(w, np.zeros_like(np.asarray(B, np.float64)), dt, L, t)
        w = rotate(w, B, 0.5 * dt)
    else:
        w = heun(w, B, dt, L, t)
    return tp.transport_step(w, 0.5 * dt, bc_left, bc_right, L, limiter)


def moments(w, L):
    """Per cell: rho_mu = h_v^2 sum_v w_mu (eq. density, Pauli components),
    momentum h_v^2 sum_v v tr W (eq. velocity, times tr rho), energy
    h_v^2 sum_v |v|^2/2 tr W; returns [Nx, 7] = (rho_0..3, p_x, p_y, e)."""
    N = w.shape[1]
    h = 2.0 * L / N
    v = h * (np.arange(N) - N // 2)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    tr = 2.0 * w[..., 0]
    out = np.zeros((w.shape[0], 7))
    out[:, 0:4] = h * h * w.sum(axis=(1, 2))
    out[:, 4] = h * h * (vx * tr).sum(axis=(1, 2))
    out[:, 5] = h * h * (vy * tr).sum(axis=(1, 2))
    out[:, 6] = h * h * (0.5 * (vx**2 + vy**2) * tr).sum(axis=(1, 2))
    return out
