"""Seeded synthetic workloads for the spatially inhomogeneous matrix-valued
quantum Boltzmann solver.  Input generation only: no part of the numerical
scheme lives here.  Both the HIP library (through its tests and bench.py)
and the CPU oracle take their inputs from this module.

Common settings (Sec. 5): velocity box [-L, L]^2 with L = 12, truncation
radius R = 7.5, J = 32 angles, M = N Gauss-Legendre radii, omega = |v|^2/2,
v-grid v_i = (2L/N)(i - N/2); cells x_j = (j + 1/2)/Nx on (0, 1).

RNG: numpy Generator(PCG64(14081782 + c)) for configuration c; every array
is drawn in bulk, C order over [x][v_x][v_y] then component.

Configurations (the workload shapes the solver is measured on):
  1  Nx=16,  N=16, periodic, B = 0, W = U diag(l1, l2) U^H with
     l ~ U(0.05, 0.95), U Haar-random; dt = 1e-3, 10 steps, complex128.
  2  Nx=128, N=32, periodic, Fermi-Dirac beta=1, mu(x) = 0.5 sin(2 pi x),
     plus a Hermitian perturbation of amplitude 0.05; B = (0, 0, 0.5);
     dt = 1e-3, 100 steps, complex128 and complex64.
  3  Nx=256, N=64, Dirichlet left (Table 1 left state), Maxwell right
     (alpha = 0.5, wall beta = 2, mu = 0); initial Fermi-Dirac beta=1, mu=0
     plus perturbation; smooth seeded B with max |B| = 1; dt = 5e-4,
     500 steps, float32 bulk with float64 moments.
  4  64 independent periodic problems, Nx in {32..512}, N in {32, 64},
     configuration-2-type data, B = 0, dt = 2.5e-4, 50 steps.
  5  configuration 2 state and field, 200 steps, complex128, gradients.
"""
from dataclasses import dataclass, field

import numpy as np

L_BOX = 12.0
R_TRUNC = 7.5
J_ANGLES = 32
SEED_BASE = 14081782

SIGMA = np.array(
    [[[1, 0], [0, 1]], [[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]],
    dtype=np.complex128,
)


@dataclass
class BC:
    kind: str                      # "periodic" | "dirichlet" | "maxwell"
    inv_kT: float = 1.0
    mu_up: float = 0.0
    mu_down: float = 0.0
    U: np.ndarray = field(default_factory=lambda: np.eye(2, dtype=np.complex128))
    alpha: float = 0.0


@dataclass
class Workload:
    name: str
    Nx: int
    N: int
    L: float
    R: float
    J: int
    M: int
    dt: float
    steps: int
    W0: np.ndarray                 # [Nx, N, N, 2, 2] complex128
    B: np.ndarray                  # [Nx, 3] float64
    left: BC
    right: BC


def rng_for(config, stream=0):
    return np.random.Generator(np.random.PCG64(SEED_BASE + config + 1000 * stream))


def velocity_axis(N, L=L_BOX):
    return (2.0 * L / N) * (np.arange(N) - N // 2)


def cell_centres(Nx):
    return (np.arange(Nx) + 0.5) / Nx


def haar_unitary(rng, shape):
    """Haar-distributed 2x2 unitaries: QR of a complex Ginibre matrix with
    the phase of R's diagonal moved into Q (Mezzadri's construction)."""
    z = rng.standard_normal(shape + (2, 2, 2))
    Z = (z[..., 0] + 1j * z[..., 1]) / np.sqrt(2.0)
    Q, Rm = np.linalg.qr(Z)
    d = np.diagonal(Rm, axis1=-2, axis2=-1)
    return Q * (d / np.abs(d))[..., None, :]


def fd_occupation(vx, vy, beta, mu):
    return 1.0 / (np.exp(beta * (0.5 * (vx**2 + vy**2) - mu)) + 1.0)


def perturbed_fd(rng, Nx, N, beta, mu_of_x, amp=0.05, L=L_BOX):
    """f(x, v) 1 + amp * 4 f (1 - f) * sum_mu h_mu sigma_mu, h ~ U(-1/4, 1/4);
    eigenvalues stay inside [0, 1]."""
    v = velocity_axis(N, L)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    x = cell_centres(Nx)
    f = fd_occupation(vx[None], vy[None], beta, np.asarray(mu_of_x(x))[:, None, None])
    h = rng.uniform(-0.25, 0.25, (Nx, N, N, 4))
    pert = amp * 4.0 * f * (1.0 - f)
    W = f[..., None, None] * SIGMA[0]
    W = W + np.einsum("xab,xabm,mij->xabij", pert, h, SIGMA)
    return W


def haar_state(rng, Nx, N):
    lam = rng.uniform(0.05, 0.95, (Nx, N, N, 2))
    U = haar_unitary(rng, (Nx, N, N))
    D = np.zeros((Nx, N, N, 2, 2), dtype=np.complex128)
    D[..., 0, 0] = lam[..., 0]
    D[..., 1, 1] = lam[..., 1]
    return U @ D @ np.conj(np.swapaxes(U, -1, -2))


def smooth_field(rng, Nx, nmodes=3):
    """B_k(x) = sum_n a_kn cos(2 pi n x) + b_kn sin(2 pi n x), a, b ~ N(0, 1),
    rescaled so that max_j |B(x_j)| = 1."""
    ab = rng.standard_normal((3, nmodes, 2))
    x = cell_centres(Nx)
    n = np.arange(1, nmodes + 1)
    c = np.cos(2 * np.pi * np.outer(x, n))
    s = np.sin(2 * np.pi * np.outer(x, n))
    B = c @ ab[:, :, 0].T + s @ ab[:, :, 1].T          # [Nx, 3]
    return B / np.max(np.linalg.norm(B, axis=1))


def config(c, Nx=None, N=None, steps=None):
    """Workload of configuration c (1, 2, 3 or 5); Nx / N / steps may be
    reduced for oracle-sized variants (same recipe, same seed stream)."""
    periodic = BC("periodic")
    if c == 1:
        Nx, N = Nx or 16, N or 16
        rng = rng_for(1)
        W0 = haar_state(rng, Nx, N)
        B = np.zeros((Nx, 3))
        return Workload("haar_periodic", Nx, N, L_BOX, R_TRUNC, J_ANGLES, N, 1e-3,
                        steps or 10, W0, B, periodic, periodic)
    if c in (2, 5):
        Nx, N = Nx or 128, N or 32
        rng = rng_for(2)
        W0 = perturbed_fd(rng, Nx, N, 1.0, lambda x: 0.5 * np.sin(2 * np.pi * x))
        B = np.tile(np.array([0.0, 0.0, 0.5]), (Nx, 1))
        return Workload("fd_periodic_B" if c == 2 else "adjoint_fd_periodic_B",
                        Nx, N, L_BOX, R_TRUNC, J_ANGLES, N, 1e-3,
                        steps or (100 if c == 2 else 200), W0, B, periodic, periodic)
    if c == 3:
        Nx, N = Nx or 256, N or 64
        rng = rng_for(3)
        W0 = perturbed_fd(rng, Nx, N, 1.0, lambda x: np.zeros_like(x))
        B = smooth_field(rng, Nx)
        left = BC("dirichlet", inv_kT=0.8, mu_up=1.5, mu_down=-1.5)
        right = BC("maxwell", inv_kT=2.0, mu_up=0.0, mu_down=0.0, alpha=0.5)
        return Workload("dirichlet_maxwell_slab", Nx, N, L_BOX, R_TRUNC, J_ANGLES, N, 5e-4,
                        steps or 500, W0, B, left, right)
    raise ValueError(c)


def batch_config(nprob=64, steps=50):
    """Configuration 4: independent periodic problems with uneven shapes."""
    rng = rng_for(4)
    Nxs = rng.choice([32, 64, 128, 256, 512], size=nprob)
    Ns = rng.choice([32, 64], size=nprob)
    out = []
    for p in range(nprob):
        r = rng_for(4, stream=p + 1)
        W0 = perturbed_fd(r, int(Nxs[p]), int(Ns[p]), 1.0,
                          lambda x: 0.5 * np.sin(2 * np.pi * x))
        out.append(Workload(f"batch{p}", int(Nxs[p]), int(Ns[p]), L_BOX, R_TRUNC, J_ANGLES,
                            int(Ns[p]), 2.5e-4, steps, W0, np.zeros((int(Nxs[p]), 3)),
                            BC("periodic"), BC("periodic")))
    return out


def adjoint_loss_weight(Nx, config_id=5):
    """Seeded Gaussian g(x) = exp(-(x - x0)^2 / (2 s^2)), x0 ~ U(0.3, 0.7),
    s ~ U(0.05, 0.15); the loss is dx h_v^2 sum g(x_j) tr(sigma_z W)."""
    rng = rng_for(config_id, stream=7)
    x0 = rng.uniform(0.3, 0.7)
    s = rng.uniform(0.05, 0.15)
    x = cell_centres(Nx)
    return np.exp(-((x - x0) ** 2) / (2 * s * s))


def validation_state(N, L=L_BOX):
    """The fixed Wigner state of the validation of Sec. 5.1 (eq. validationW)
    on the velocity grid (2L/N) Xi: [N, N, 2, 2] complex."""
    vx, vy = np.meshgrid(velocity_axis(N, L), velocity_axis(N, L), indexing="ij")
    w0 = (1.0 / (3 * np.pi)) * (1 + vx) * np.exp(-0.5 * (vx - 0.5) ** 2 - 0.5 * (vy + vx) ** 2)
    w1 = (3 * np.sqrt(6 / 5) / (55 * np.pi)) * (1 - vx - vy / 6) ** 2 * np.exp(
        -(2 * vx + vy) ** 2 / 12 - vy**2 / 10)
    w2 = (1 / (4 * np.pi * np.sqrt(2))) * np.exp(-((vx - 1) ** 2) / 8 - vy**2 / 4)
    w3 = (9 / (56 * np.pi)) * (1 / 3 + vx) ** 2 * np.exp(-((vx - vy) ** 2) / 8 - (vx + 2 * vy) ** 2 / 8)
    W = np.zeros((N, N, 2, 2), np.complex128)
    W[..., 0, 0] = w0 + w3
    W[..., 1, 1] = w0 - w3
    W[..., 0, 1] = w1 - 1j * w2
    W[..., 1, 0] = w1 + 1j * w2
    return W


# ------------------------------------------------------------------ physics runs (Sec. 5.2, 5.3)
def rotation_generator(vx, vy):
    """X(v) of eq. W0homogeneous as [..., 2, 2]: sin(v_y^2) 1 + (v_x - 1) s1
    + 2 / (v_x^2 + |v_y| + 1) s2 + cos(v_x + v_y / 2) s3."""
    c = (np.sin(vy**2), vx - 1.0, 2.0 / (vx**2 + np.abs(vy) + 1.0), np.cos(vx + 0.5 * vy))
    return sum(ci[..., None, None] * SIGMA[i] for i, ci in enumerate(c))


def _expm_herm(X, s):
    """exp(s X) for Hermitian 2x2 X and complex scalar s (eigendecomposition)."""
    lam, V = np.linalg.eigh(X)
    return (V * np.exp(s * lam)[..., None, :]) @ np.conj(np.swapaxes(V, -1, -2))


HOMOGENEOUS_U0 = np.array([[np.cos(np.pi / 5), -1j * np.sin(np.pi / 5)],
                           [np.sin(np.pi / 5), 1j * np.cos(np.pi / 5)]])


def rotated_fd_state(N, kT, mu_up, mu_down, v0, L=L_BOX):
    """exp(-i X(v)) U0 diag(f_up, f_down)(v - v0) U0^* exp(i X(v)), the
    Fermi-Dirac state rotated by v-dependent unitaries (eq. W0homogeneous);
    kT, mu_up, mu_down and v0 = (v0x, v0y) may be arrays over cells (a
    leading axis), giving [Nx, N, N, 2, 2], else [N, N, 2, 2]."""
    v = velocity_axis(N, L)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    kT, mu_up, mu_down = (np.asarray(a, dtype=float)[..., None, None] for a in (kT, mu_up, mu_down))
    v0x = np.asarray(v0[0], dtype=float)[..., None, None]
    v0y = np.asarray(v0[1], dtype=float)[..., None, None]
    e = 0.5 * ((vx - v0x) ** 2 + (vy - v0y) ** 2)
    D = np.zeros(np.broadcast(e, mu_up).shape + (2, 2), np.complex128)
    D[..., 0, 0] = 1.0 / (np.exp((e - mu_up) / kT) + 1.0)
    D[..., 1, 1] = 1.0 / (np.exp((e - mu_down) / kT) + 1.0)
    Q = _expm_herm(rotation_generator(vx, vy), -1j) @ HOMOGENEOUS_U0
    return Q @ D @ np.conj(np.swapaxes(Q, -1, -2))


def fd_wall_state(N, inv_kT, mu_up, mu_down, U, L=L_BOX):
    """U diag(f_up, f_down) U^* at rest on the velocity grid (eq. W_FermiDirac)."""
    v = velocity_axis(N, L)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    D = np.zeros((N, N, 2, 2), np.complex128)
    D[..., 0, 0] = fd_occupation(vx, vy, inv_kT, mu_up)
    D[..., 1, 1] = fd_occupation(vx, vy, inv_kT, mu_down)
    U = np.asarray(U, np.complex128)
    return U @ D @ np.conj(U.T)


ROT45 = np.array([[1.0, -1.0], [1.0, 1.0]], np.complex128) / np.sqrt(2.0)


def physics_run(name, N=32, Nx=None, t_end=None):
    """The simulations of Sec. 5.2 and 5.3 (N = 32, L = 12, J = M = 32,
    R = 7.5), as workloads; t_end sets the number of steps.
      E2   homogeneous relaxation (one periodic cell), eq. W0homogeneous with
           kT = 5/4, mu = (1, 3/2), v0 = (0.4, -0.1); dt = 0.001.
      E3   periodic, dx = 0.1, dt = 0.008; the same state with x-dependent
           kT = 5/4 + cos(2 pi x) / 4, mu_up = 1 + cos(2 pi x) / 2,
           mu_down = 3/2 - cos(2 pi x) / 2, v0 = (0.4, -0.1) sin(2 pi x).
      E4   E3 with B(x) = (0, cos 2 pi x, sin 2 pi x) (eq. Bext_rot), t = 1.
      E5   Dirichlet walls of Table 1, dx = 0.025, dt = 0.002.
      E6i, E6ii  Maxwell walls of Table 2 (alpha = 0.4), dx = 0.025,
           dt = 0.002, t = 4.
    The wall runs start from the Fermi-Dirac state at rest whose inverse
    temperature and chemical potentials are the means of the two walls'
    (spin basis 1)."""
    periodic = BC("periodic")
    if name == "E2":
        Nx = Nx or 1
        W = np.broadcast_to(rotated_fd_state(N, 1.25, 1.0, 1.5, (0.4, -0.1)), (Nx, N, N, 2, 2)).copy()
        dt = 1e-3
        return Workload(name, Nx, N, L_BOX, R_TRUNC, J_ANGLES, N, dt, int(round((t_end or 1.0) / dt)),
                        W, np.zeros((Nx, 3)), periodic, periodic)
    if name in ("E3", "E4"):
        Nx = Nx or 10
        x = cell_centres(Nx)
        c, s = np.cos(2 * np.pi * x), np.sin(2 * np.pi * x)
        W = rotated_fd_state(N, 1.25 + 0.25 * c, 1.0 + 0.5 * c, 1.5 - 0.5 * c, (0.4 * s, -0.1 * s))
        B = np.zeros((Nx, 3))
        if name == "E4":
            B = np.stack([np.zeros(Nx), c, s], axis=1)
        dt = 0.008
        return Workload(name, Nx, N, L_BOX, R_TRUNC, J_ANGLES, N, dt,
                        int(round((t_end or (1.0 if name == "E4" else 2.0)) / dt)), W, B, periodic, periodic)
    walls = {
        "E5": (BC("dirichlet", 0.8, 1.5, -1.5), BC("dirichlet", 1.2, 1.5, -1.5, ROT45)),
        "E6i": (BC("maxwell", 0.6, -0.4, 1.8, alpha=0.4), BC("maxwell", 1.1, 1.3, -0.9, alpha=0.4)),
        "E6ii": (BC("maxwell", 1.0, 1.5, -1.5, alpha=0.4), BC("maxwell", 1.0, 1.5, -1.5, ROT45, alpha=0.4)),
    }
    if name in walls:
        Nx = Nx or 40
        left, right = walls[name]
        mid = fd_wall_state(N, 0.5 * (left.inv_kT + right.inv_kT), 0.5 * (left.mu_up + right.mu_up),
                            0.5 * (left.mu_down + right.mu_down), np.eye(2))
        W = np.broadcast_to(mid, (Nx, N, N, 2, 2)).copy()
        dt = 0.002
        return Workload(name, Nx, N, L_BOX, R_TRUNC, J_ANGLES, N, dt, int(round((t_end or 4.0) / dt)),
                        W, np.zeros((Nx, 3)), left, right)
    raise ValueError(name)
