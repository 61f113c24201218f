"""Finite-volume transport with the minmod slope limiter (Sec. 4,
eq. slopeLimiterStep and eq. minmod) and the boundary conditions of Sec. 2.

State layout: w[Nx, N, N, 4] (Pauli components), cell j centred at
x_j = (j + 1/2) dx, dx = 1/Nx, Omega = (0, 1).  The first velocity axis is v_x.

Readings:
* minmod acts on each of the 4 real Pauli components separately, and is 0
  whenever a b <= 0.
* Ghost cells: two on each side.  Periodic: wrap.  At a wall, for velocities
  entering the domain both ghost cells hold the inflow state; for the other
  velocities both ghost cells copy the adjacent interior cell.
* Dirichlet inflow: the given boundary state Phi(v).
* Maxwell inflow: (1 - alpha) W_b(-v_x, v_y) + alpha W_FD(v) Fbar / Z, with
  W_b the adjacent interior cell, Fbar = h_v^2 sum_{out} tr W_b |v_x| and
  Z = h_v^2 sum_{in, mirrored} tr W_FD |v_x|.  On the grid v_x = (2L/N)(i - N/2)
  the mirror of row i is row N - i; row i = 0 (v_x = -L) has no mirror and
  is handled like an outgoing row (copy of the interior cell).
"""
import numpy as np


def minmod(a, b):
    """eq. minmod, elementwise."""
    return np.where(a * b > 0.0, np.where(np.abs(a) <= np.abs(b), a, b), 0.0)


# Other slope limiters (Sec. 4 allows them; the standard choices of
# LeVeque's finite-volume text), as slopes from the two one-sided
# differences a = W_{j+1} - W_j and b = W_j - W_{j-1}:


def superbee(a, b):
    """The larger in magnitude of minmod(a, 2b) and minmod(2a, b)."""
    s1, s2 = minmod(a, 2.0 * b), minmod(2.0 * a, b)
    return np.where(np.abs(s1) >= np.abs(s2), s1, s2)


def monotonized_central(a, b):
    """minmod of the central difference (a + b)/2, 2a and 2b."""
    return minmod(0.5 * (a + b), minmod(2.0 * a, 2.0 * b))


def van_leer(a, b):
    """(a |b| + |a| b) / (|a| + |b|), i.e. the harmonic mean 2ab / (a + b)
    for ab > 0 and 0 otherwise."""
    den = np.abs(a) + np.abs(b)
    return np.where(den > 0.0, (a * np.abs(b) + np.abs(a) * b) / np.where(den > 0.0, den, 1.0), 0.0)


LIMITERS = {"minmod": minmod, "superbee": superbee, "mc": monotonized_central, "van_leer": van_leer}


def mirror_rows(N):
    """For each v_x row i the mirrored row N - i, or -1 for i = 0."""
    m = N - np.arange(N)
    m[0] = -1
    return m


def maxwell_inflow(wb, w_fd, alpha, side, vx, hv2):
    """Maxwell inflow state at a wall from the adjacent interior cell wb[N,N,4].
    side = 'left' (x = 0, inflow v_x > 0) or 'right' (x = 1, inflow v_x < 0).
    Returns (state[N,N,4], inflow_mask[N] over v_x rows)."""
    N = wb.shape[0]
    mir = mirror_rows(N)
    if side == "left":
        inflow = vx > 0
        outflow = vx < 0
    else:
        inflow = (vx < 0) & (mir >= 0)
        outflow = vx > 0
    trb = 2.0 * wb[..., 0]                       # tr W = 2 w0
    trfd = 2.0 * w_fd[..., 0]
    Fbar = hv2 * np.sum(trb[outflow] * np.abs(vx[outflow])[:, None])
    Z = hv2 * np.sum(trfd[inflow] * np.abs(vx[inflow])[:, None])
    state = np.zeros_like(wb)
    rows = np.nonzero(inflow)[0]
    state[rows] = (1.0 - alpha) * wb[mir[rows]] + alpha * w_fd[rows] * (Fbar / Z)
    return state, inflow


def ghosts(w, bc_left, bc_right, vx, hv2):
    """Extend w[Nx,...] by two ghost cells per side; returns [Nx+4, ...]."""
    Nx = w.shape[0]
    if bc_left["kind"] == "periodic" or bc_right["kind"] == "periodic":
        if not (bc_left["kind"] == "periodic" and bc_right["kind"] == "periodic"):
            raise ValueError("periodic on one side only")
        return w[np.arange(-2, Nx + 2) % Nx]
    out = np.concatenate([w[:1], w[:1], w, w[-1:], w[-1:]], axis=0)
    for side, bc, interior, gidx in (
        ("left", bc_left, w[0], (0, 1)),
        ("right", bc_right, w[-1], (Nx + 2, Nx + 3)),
    ):
        if bc["kind"] == "dirichlet":
            state = bc["state"]
            inflow = vx > 0 if side == "left" else vx < 0
        elif bc["kind"] == "maxwell":
            state, inflow = maxwell_inflow(interior, bc["state"], bc["alpha"], side, vx, hv2)
        else:
            raise ValueError(bc["kind"])
        for g in gidx:
            out[g][inflow] = state[inflow]
    return out


def transport_step(w, dt, bc_left, bc_right, L, limiter="minmod"):
    """One step of eq. slopeLimiterStep of length dt, for every velocity;
    `limiter` names the slope limiter in place of minmod (LIMITERS)."""
    Nx, N = w.shape[0], w.shape[1]
    dx = 1.0 / Nx
    vx = (2.0 * L / N) * (np.arange(N) - N // 2)
    hv2 = (2.0 * L / N) ** 2
    we = ghosts(w, bc_left, bc_right, vx, hv2)            # [Nx+4, N, N, 4]
    d = we[1:] - we[:-1]                                  # d[k] = we[k+1] - we[k]
    S = np.zeros_like(we)
    S[1:-1] = LIMITERS[limiter](d[1:], d[:-1])            # S_k, k = 1..Nx+2
    v = vx[None, :, None, None]
    av = np.abs(v)
    nu = dt * v / dx
    lim = 0.5 * (np.sign(nu) - nu)
    Wm, W0, Wp = we[1:-3], we[2:-2], we[3:-1]
    Sm, S0, Sp = S[1:-3], S[2:-2], S[3:-1]
    upd = (
        -v * (Wp - Wm)
        + av * (Wp - 2.0 * W0 + Wm)
        + lim * (-v * (Sp - Sm) + av * (Sp - 2.0 * S0 + Sm))
    )
    return W0 + (dt / (2.0 * dx)) * upd


def face_fluxes(w, dt, bc_left, bc_right, L, limiter="minmod"):
    """The step of eq. slopeLimiterStep in flux form,
    W_j <- W_j - (dt/dx) (F_{j+1/2} - F_{j-1/2}), with
    F_{j+1/2} = (v (W_j + W_{j+1}) - |v| (W_{j+1} - W_j)) / 2
              + l (v (S_j + S_{j+1}) - |v| (S_{j+1} - S_j)) / 2,
    l = (sgn nu - nu) / 2: the fluxes through the Nx + 1 faces j + 1/2,
    j = -1 .. Nx - 1 (the first and last are the walls), [Nx + 1, N, N, 4]."""
    Nx, N = w.shape[0], w.shape[1]
    dx = 1.0 / Nx
    vx = (2.0 * L / N) * (np.arange(N) - N // 2)
    hv2 = (2.0 * L / N) ** 2
    we = ghosts(w, bc_left, bc_right, vx, hv2)
    d = we[1:] - we[:-1]
    S = np.zeros_like(we)
    S[1:-1] = LIMITERS[limiter](d[1:], d[:-1])
    v = vx[None, :, None, None]
    av = np.abs(v)
    lim = 0.5 * (np.sign(dt * v / dx) - dt * v / dx)
    a, b = we[1:Nx + 2], we[2:Nx + 3]
    Sa, Sb = S[1:Nx + 2], S[2:Nx + 3]
    return 0.5 * (v * (a + b) - av * (b - a)) + 0.5 * lim * (v * (Sa + Sb) - av * (Sb - Sa))


def wall_inflow_moments(w, dt, bc_left, bc_right, L, limiter="minmod"):
    """Net inflow through the two walls during one step of length dt, as the
    change it makes to the per-cell moments of step.moments summed over the
    cells: (dt/dx) h_v^2 sum_v phi(v) (F_{1/2} - F_{Nx+1/2}) with phi the
    functionals (rho_0..3, p_x, p_y, energy); returns [7]."""
    Nx, N = w.shape[0], w.shape[1]
    F = face_fluxes(w, dt, bc_left, bc_right, L, limiter)
    net = F[0] - F[-1]
    h = 2.0 * L / N
    vx, vy = np.meshgrid(h * (np.arange(N) - N // 2), h * (np.arange(N) - N // 2), indexing="ij")
    tr = 2.0 * net[..., 0]
    out = np.concatenate([net.sum(axis=(0, 1)),
                          [(vx * tr).sum(), (vy * tr).sum(), (0.5 * (vx**2 + vy**2) * tr).sum()]])
    return dt * Nx * h * h * out
