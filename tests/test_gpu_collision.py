"""GPU parity of qb_collision against the CPU oracle (Sec. 3.2 scheme).

Bar: normwise relative error max|C_gpu - C_ref| / max|C_ref| below 1e-11
for the float64 path and 2e-5 for the float32 path (same inputs, same
quadrature parameters), at sizes the oracle finishes in seconds.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import collision as oc
from oracle import pauli

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-11, "f32": 2e-5}


def _gpu_collision(W, J, M, precision, L=wl.L_BOX, R=wl.R_TRUNC):
    import torch
    import paper_1408_1782_amd as qb

    ncells, N = W.shape[0], W.shape[1]
    plan = qb.Plan(qb.Problem(ncells, N, J, M, L, R, precision))
    dt = torch.complex128 if precision == "f64" else torch.complex64
    Wd = torch.from_numpy(W).to(dt).cuda().contiguous()
    C = plan.collision(Wd)
    torch.cuda.synchronize()
    out = C.cpu().numpy().astype(np.complex128)
    plan.close()
    return out


def _oracle(W, J, M, L=wl.L_BOX, R=wl.R_TRUNC):
    t = oc.Tables(W.shape[1], L, R, J, M)
    return np.stack([oc.collision(W[c], L, R, J, M, t) for c in range(W.shape[0])])


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("N,J,M,ncells", [(16, 8, 8, 3), (32, 6, 6, 2), (64, 4, 4, 1)])
def test_collision_matches_oracle_haar(N, J, M, ncells, precision):
    """Random Haar-rotated states (the configuration-1 recipe): every tile
    size of the padded grid (P = 32, 64, 128), several cells."""
    print(f"collision parity N={N} J={J} M={M} cells={ncells} {precision}", flush=True)
    W = wl.haar_state(wl.rng_for(1, stream=N), ncells, N)
    ref = _oracle(W, J, M)
    got = _gpu_collision(W, J, M, precision)
    err = _rel(got, ref)
    print(f"  rel err {err:.3e}", flush=True)
    assert err < TOL[precision]


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_collision_matches_oracle_full_quadrature_N16(precision):
    """Configuration-1 parameters in full: N = 16, J = 32, M = 16."""
    W = wl.config(1, Nx=2).W0
    ref = _oracle(W, 32, 16)
    got = _gpu_collision(W, 32, 16, precision)
    err = _rel(got, ref)
    print(f"  rel err {err:.3e}", flush=True)
    assert err < TOL[precision]


def test_collision_near_equilibrium_f64():
    """Perturbed Fermi-Dirac data (configuration-2 recipe), where gain and
    loss nearly cancel."""
    W = wl.config(2, Nx=2, N=32).W0
    ref = _oracle(W, 8, 8)
    got = _gpu_collision(W, 8, 8, "f64")
    err = _rel(got, ref)
    print(f"  rel err {err:.3e}", flush=True)
    assert err < TOL["f64"]


def test_collision_output_is_hermitian_and_traceless_commutator():
    """C[W] is Hermitian; for W proportional to 1 its Bloch part is zero."""
    N = 16
    rng = np.random.default_rng(3)
    f = rng.uniform(0.1, 0.9, (1, N, N))
    W = f[..., None, None] * np.eye(2)
    got = _gpu_collision(W, 8, 8, "f64")
    assert np.abs(got - np.conj(np.swapaxes(got, -1, -2))).max() == 0.0
    c = pauli.to_pauli(got)
    assert np.abs(c[..., 1:]).max() < 1e-13 * np.abs(c[..., 0]).max()
