"""GPU parity of the reverse mode (qb_collision_vjp, qb_transport_vjp,
qb_adjoint_step, and the checkpointed autograd integration) against the
oracle's reverse-mode derivatives (oracle/adjoint.py, pinned by exact
polynomial JVPs and branchwise differences on the CPU).

Gradients cross the C ABI in torch's complex convention: the cotangent of a
state is G = (1/2) sum_mu g_mu sigma_mu with g_mu the gradient with respect
to the Pauli component w_mu, so g = 2 to_pauli(G)."""
import os

import numpy as np
import pytest

import workloads as wl
from oracle import adjoint as oad
from oracle import collision as oc
from oracle import pauli
from oracle.fermi_dirac import fd_matrix

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = {"f64": 1e-11, "f32": 2e-5}


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def to_dev(x, precision):
    import torch
    dt = torch.complex128 if precision == "f64" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(x)).to(dt).cuda().contiguous()


def cot_api(g):
    """Pauli gradient -> API cotangent (1/2) sum g_mu sigma_mu."""
    return pauli.from_pauli(0.5 * g)


def cot_pauli(G):
    return 2.0 * pauli.to_pauli(G.cpu().numpy().astype(np.complex128))


def bc_dict(b, N, L):
    if b.kind == "periodic":
        return {"kind": "periodic"}
    v = (2 * L / N) * (np.arange(N) - N // 2)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    st = pauli.to_pauli(fd_matrix(vx, vy, b.inv_kT, b.mu_up, b.mu_down, b.U))
    return {"kind": b.kind, "state": st, "alpha": b.alpha}


def make_plan(w, precision, J, M, Nx=None):
    import paper_1408_1782_amd as qb
    p = qb.Plan(qb.Problem(Nx or w.Nx, w.N, J, M, w.L, w.R, precision,
                           qb.BC.from_workload(w.left), qb.BC.from_workload(w.right)))
    p.enable_adjoint()
    return p


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("N,J,M,ncells", [(16, 8, 8, 3), (32, 6, 5, 2), (64, 4, 4, 1)])
def test_collision_vjp_matches_oracle(precision, N, J, M, ncells):
    """C'(W)^T lam on P = 32, 64, 128 (one workgroup per (cell, j) for I_3,
    several cells, odd M)."""
    import torch
    rng = np.random.default_rng(N + J)
    w = wl.config(2, Nx=ncells, N=N)
    plan = make_plan(w, precision, J, M)
    lam = rng.standard_normal((ncells, N, N, 4))
    G = plan.collision_vjp(to_dev(w.W0, precision), to_dev(cot_api(lam), precision))
    torch.cuda.synchronize()
    got = cot_pauli(G)
    t = oc.Tables(N, w.L, w.R, J, M)
    s = pauli.to_pauli(w.W0)
    ref = np.stack([oad.collision_pauli_vjp(s[c], lam[c], w.L, w.R, J, M, t) for c in range(ncells)])
    assert rel(got, ref) < TOL[precision]
    plan.close()


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("N,E,M", [(16, 8, 5), (32, 16, 4), (32, 8, 5), (64, 32, 3), (64, 16, 4)])
def test_collision_vjp_every_kernel_variant(precision, N, E, M, variant):
    """Both I_3 adjoint kernels (row w cotangents in memory / registers) on
    every tile shape family, odd and even M, against the oracle."""
    import torch
    rng = np.random.default_rng(7 * N + M)
    w = wl.config(3, Nx=2, N=N)
    plan = make_plan(w, precision, 4, M)
    # the reverse-mode pipeline on its own tile (the forward keeps the default)
    plan.set_adjoint_tile(E)
    assert plan.config()["adjoint_tile"] == E
    plan.set_adjoint_variant(variant)
    lam = rng.standard_normal((2, N, N, 4))
    G = plan.collision_vjp(to_dev(w.W0, precision), to_dev(cot_api(lam), precision))
    torch.cuda.synchronize()
    t = oc.Tables(N, w.L, w.R, 4, M)
    s = pauli.to_pauli(w.W0)
    ref = np.stack([oad.collision_pauli_vjp(s[c], lam[c], w.L, w.R, 4, M, t) for c in range(2)])
    assert rel(cot_pauli(G), ref) < TOL[precision]
    plan.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("cfg", [2, 3])
def test_transport_vjp_matches_oracle(cfg, precision):
    """Transpose of the limited transport step: periodic (configuration 2)
    and Dirichlet / Maxwell walls (configuration 3)."""
    import torch
    rng = np.random.default_rng(cfg)
    w = wl.config(cfg, Nx=12, N=16)
    plan = make_plan(w, precision, 4, 4)
    s = pauli.to_pauli(w.W0) + 0.01 * rng.standard_normal((w.Nx, w.N, w.N, 4))
    lam = rng.standard_normal(s.shape)
    dt = 0.7 / (w.L * w.Nx)
    G = plan.transport_vjp(to_dev(pauli.from_pauli(s), precision), dt, to_dev(cot_api(lam), precision))
    torch.cuda.synchronize()
    ref = oad.transport_step_vjp(s, lam, dt, bc_dict(w.left, w.N, w.L), bc_dict(w.right, w.N, w.L), w.L)
    assert rel(cot_pauli(G), ref) < TOL[precision]
    plan.close()


@pytest.mark.parametrize("use_record", [False, True])
@pytest.mark.parametrize("cfg", [2, 3])
def test_adjoint_step_matches_oracle(cfg, use_record):
    """One reverse splitting step (float64), from the state or from a
    qb_step_trace record, with the field cotangent."""
    import torch
    rng = np.random.default_rng(10 + cfg)
    w = wl.config(cfg, Nx=4, N=16)
    J, M = 6, 6
    plan = make_plan(w, "f64", J, M)
    s = pauli.to_pauli(w.W0)
    lam = rng.standard_normal(s.shape)
    B = torch.from_numpy(w.B).cuda().contiguous()
    gB = torch.zeros((w.Nx, 3), dtype=torch.float64, device="cuda")
    W = to_dev(w.W0, "f64")
    if use_record:
        trace = plan.new_trace(1)
        plan.step_trace(W.clone(), B, w.dt, 1, trace)
        G = plan.adjoint_step(to_dev(cot_api(lam), "f64"), B, w.dt, record=trace, gB=gB)
    else:
        G = plan.adjoint_step(to_dev(cot_api(lam), "f64"), B, w.dt, W=W, gB=gB)
    torch.cuda.synchronize()
    t = oc.Tables(w.N, w.L, w.R, J, M)
    gw, gb = oad.step_vjp(s, w.B, w.dt, lam, w.L, w.R, J, M, bc_dict(w.left, w.N, w.L),
                          bc_dict(w.right, w.N, w.L), t)
    assert rel(cot_pauli(G), gw) < 1e-11
    assert rel(gB.cpu().numpy(), gb) < 1e-11
    plan.close()


def test_step_trace_matches_step():
    """qb_step_trace advances the state exactly as qb_step does."""
    import torch
    w = wl.config(2, Nx=4, N=16)
    plan = make_plan(w, "f64", 4, 4)
    B = torch.from_numpy(w.B).cuda().contiguous()
    a, b = to_dev(w.W0, "f64"), to_dev(w.W0, "f64")
    plan.step(a, B, w.dt, 3)
    plan.step_trace(b, B, w.dt, 3, plan.new_trace(3))
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.close()


@pytest.mark.parametrize("every", [6, 0])
def test_evolve_gradient_matches_oracle_reduced_configuration5(every):
    """Gradient of dx h^2 sum g(x_j) tr(sigma_z W(T)) after 20 steps
    (configuration-5 recipe, Nx = 8, N = 16, J = M = 8) in the initial state
    and the field, through torch autograd with checkpoints every 6 steps
    (segments 6, 6, 6, 2) and with every step's record kept, against the
    stored oracle gradient."""
    import torch
    import paper_1408_1782_amd as qb
    p = os.path.join(GOLDEN, "c5_reduced_grad.npz")
    assert os.path.exists(p), "c5_reduced_grad.npz missing (python tests/golden/make_golden.py c5)"
    g = np.load(p)
    w = wl.config(5, Nx=8, N=16)
    plan = make_plan(w, "f64", 8, 8)
    W0 = to_dev(w.W0, "f64").requires_grad_(True)
    B = torch.from_numpy(w.B).cuda().contiguous().requires_grad_(True)
    WT = qb.evolve(plan, W0, B, w.dt, 20, checkpoint_every=every)
    h2 = (2 * w.L / w.N) ** 2
    wt = torch.from_numpy(g["weight"]).cuda()
    # tr(sigma_z W) = W_00 - W_11
    loss = h2 / w.Nx * (wt[:, None, None] * (WT[..., 0, 0] - WT[..., 1, 1]).real).sum()
    loss.backward()
    torch.cuda.synchronize()
    assert rel(pauli.to_pauli(WT.detach().cpu().numpy()), g["final"]) < 1e-11
    assert abs(loss.item() - float(g["loss"])) < 1e-11 * abs(float(g["loss"]))
    assert rel(cot_pauli(W0.grad), g["grad_w0"]) < 1e-10
    assert rel(B.grad.cpu().numpy(), g["grad_B"]) < 1e-10
    plan.close()


def test_evolve_gradient_finite_differences():
    """Directional derivatives of the observable by central differences of
    the GPU forward run against the adjoint gradient: four field components
    and two Hermitian directions of the initial state, 10 steps of the
    configuration-5 recipe at N = 32 on 16 cells, float64.  The limiter is
    not differentiable where neighbouring differences vanish (the
    Fermi-Dirac tails), so the initial state gets an O(0.05) Hermitian
    perturbation that keeps every difference far from zero; the state step
    h = 1e-7 keeps the difference quotients on one branch, and the field,
    which moves the state only through dt-small rotations, takes h = 1e-4."""
    import torch
    import paper_1408_1782_amd as qb
    rng = np.random.default_rng(55)
    w = wl.config(5, Nx=16, N=32)
    J, M = 8, 8
    plan = make_plan(w, "f64", J, M)
    steps = 10
    h2 = (2 * w.L / w.N) ** 2
    wt = torch.from_numpy(wl.adjoint_loss_weight(w.Nx)).cuda()

    def loss_of(WT):
        return h2 / w.Nx * (wt[:, None, None] * (WT[..., 0, 0] - WT[..., 1, 1]).real).sum()

    base = w.W0 + pauli.from_pauli(0.05 * rng.standard_normal((w.Nx, w.N, w.N, 4)))
    W0 = to_dev(base, "f64").requires_grad_(True)
    B = torch.from_numpy(w.B).cuda().contiguous().requires_grad_(True)
    loss_of(qb.evolve(plan, W0, B, w.dt, steps, checkpoint_every=4)).backward()

    def run(Wi, Bi):
        W = Wi.detach().clone().contiguous()
        plan.step(W, Bi.detach().contiguous(), w.dt, steps)
        return loss_of(W).item()

    for _ in range(4):
        c, k = int(rng.integers(w.Nx)), int(rng.integers(3))
        dB = torch.zeros_like(B)
        dB[c, k] = 1.0
        h = 1e-4
        fd = (run(W0, B + h * dB) - run(W0, B - h * dB)) / (2 * h)
        ad = B.grad[c, k].item()
        assert abs(fd - ad) <= 1e-5 * abs(ad) + 1e-10, (c, k, fd, ad)
    for _ in range(2):
        d = pauli.from_pauli(0.05 * rng.standard_normal((w.Nx, w.N, w.N, 4)))
        dW = to_dev(d, "f64")
        h = 1e-7
        fd = (run(W0 + h * dW, B) - run(W0 - h * dW, B)) / (2 * h)
        ad = torch.sum((torch.conj(W0.grad) * dW).real).item()
        assert abs(fd - ad) <= 1e-5 * abs(ad) + 1e-10, (fd, ad)
    plan.close()


def test_evolve_gradient_finite_differences_full_shape():
    """The gradient workload at its full shape (128 cells, N = 32,
    J = M = 32, float64), 20 steps with checkpoints every 5 (three segments
    recomputed): central differences with h = 1e-6 on 16 field components
    and h = 1e-7 on 8 Hermitian directions of the (perturbed, see above)
    initial state against the adjoint gradient."""
    import torch
    import paper_1408_1782_amd as qb
    rng = np.random.default_rng(56)
    w = wl.config(5)
    plan = make_plan(w, "f64", w.J, w.M)
    steps = 20
    h2 = (2 * w.L / w.N) ** 2
    wt = torch.from_numpy(wl.adjoint_loss_weight(w.Nx)).cuda()

    def loss_of(WT):
        return h2 / w.Nx * (wt[:, None, None] * (WT[..., 0, 0] - WT[..., 1, 1]).real).sum()

    base = w.W0 + pauli.from_pauli(0.05 * rng.standard_normal((w.Nx, w.N, w.N, 4)))
    W0 = to_dev(base, "f64").requires_grad_(True)
    B = torch.from_numpy(w.B).cuda().contiguous().requires_grad_(True)
    loss_of(qb.evolve(plan, W0, B, w.dt, steps, checkpoint_every=5)).backward()

    def run(Wi, Bi):
        W = Wi.detach().clone().contiguous()
        plan.step(W, Bi.detach().contiguous(), w.dt, steps)
        return loss_of(W).item()

    # field components where the observable's weight is not negligible; a
    # difference quotient carries a rounding error of about eps |loss| / h
    # (a few 1e-12 here), so components far below the largest are held to
    # an absolute bar of 1e-6 of the largest field gradient
    g = wl.adjoint_loss_weight(w.Nx)
    cells = np.argsort(g)[-32:]
    gmax = B.grad.abs().max().item()
    picks = rng.choice(len(cells) * 3, 16, replace=False)
    for pk in picks:
        c, k = int(cells[pk // 3]), int(pk % 3)
        dB = torch.zeros_like(B)
        dB[c, k] = 1.0
        h = 1e-6
        fd = (run(W0, B + h * dB) - run(W0, B - h * dB)) / (2 * h)
        ad = B.grad[c, k].item()
        print(f"field component ({c}, {k}): fd {fd:.10e} adjoint {ad:.10e} (largest {gmax:.3e})", flush=True)
        assert abs(fd - ad) <= 1e-5 * abs(ad) + 1e-6 * gmax, (c, k, fd, ad, gmax)
    for i in range(8):
        d = pauli.from_pauli(0.05 * rng.standard_normal((w.Nx, w.N, w.N, 4)))
        dW = to_dev(d, "f64")
        h = 1e-7
        fd = (run(W0 + h * dW, B) - run(W0 - h * dW, B)) / (2 * h)
        ad = torch.sum((torch.conj(W0.grad) * dW).real).item()
        print(f"state direction {i}: fd {fd:.10e} adjoint {ad:.10e}", flush=True)
        assert abs(fd - ad) <= 1e-5 * abs(ad) + 1e-12, (fd, ad)
    plan.close()
