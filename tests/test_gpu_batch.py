"""GPU tests of the FFT tile shapes, the autotuner and batched problems
(qb_plan_set_tile, qb_plan_tune, qb_batch_*): every tile shape against the
oracle, batches against the single-problem path (bitwise, the arithmetic
per cell is the same), HIP-graph replays against eager runs, chunked
launches, and one batched step against the oracle."""
import numpy as np
import pytest

import workloads as wl
from oracle import collision as oc
from oracle import pauli
from oracle import step as ostep
from oracle.fermi_dirac import fd_matrix

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-11, "f32": 2e-5}


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def to_dev(x, precision):
    import torch
    dt = torch.complex128 if precision == "f64" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(x)).to(dt).cuda().contiguous()


def bc_dict(b, N, L):
    if b.kind == "periodic":
        return {"kind": "periodic"}
    v = (2 * L / N) * (np.arange(N) - N // 2)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    st = pauli.to_pauli(fd_matrix(vx, vy, b.inv_kT, b.mu_up, b.mu_down, b.U))
    return {"kind": b.kind, "state": st, "alpha": b.alpha}


def problem(w, precision, J, M, Nx=None):
    import paper_1408_1782_amd as qb
    return qb.Problem(Nx or w.Nx, w.N, J, M, w.L, w.R, precision,
                      qb.BC.from_workload(w.left), qb.BC.from_workload(w.right))


@pytest.mark.parametrize("paired", [True, False])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("N,E", [(16, 16), (16, 8), (32, 32), (32, 16), (32, 8), (64, 32), (64, 16)])
def test_every_tile_matches_oracle(precision, N, E, paired):
    """Every tile shape, I_3 with and without node pairing (odd M: the
    middle node runs alone)."""
    import torch
    import paper_1408_1782_amd as qb
    w = wl.config(2, Nx=2, N=N)
    J, M = 6, 5
    plan = qb.Plan(problem(w, precision, J, M))
    plan.set_tile(E)
    plan.set_pairing(paired)
    C = plan.collision(to_dev(w.W0, precision))
    torch.cuda.synchronize()
    t = oc.Tables(N, w.L, w.R, J, M)
    ref = np.stack([oc.collision(w.W0[c], w.L, w.R, J, M, t) for c in range(w.Nx)])
    assert rel(C.cpu().numpy().astype(np.complex128), ref) < TOL[precision]
    plan.close()


def test_tune_picks_a_compiled_tile_and_caches_it():
    import paper_1408_1782_amd as qb
    w = wl.config(2, Nx=8, N=32)
    plan = qb.Plan(problem(w, "f32", 8, 8))
    e1 = plan.tune()
    assert e1 in qb.Plan.TILES[64]
    assert plan.tune() == e1
    with pytest.raises(qb.QBError):
        plan.set_tile(4)
    plan.close()


def _batch_members(precision):
    """Uneven problems: two grid sizes, periodic and walled, with and
    without field."""
    a = wl.config(2, Nx=5, N=16)
    b = wl.config(3, Nx=7, N=32)
    c = wl.config(1, Nx=3, N=16)
    d = wl.config(2, Nx=9, N=32)
    return [(a, a.B), (b, b.B), (c, None), (d, d.B)]


@pytest.mark.parametrize("persistent,graph", [(False, False), (True, False), (True, True)])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_batch_equals_single_problem_runs(precision, persistent, graph):
    """Each problem of a batch ends bitwise where its own plan (one
    workgroup per task) takes it, with the same moments: with one workgroup
    per task, with the persistent launches that stride over every problem's
    tasks, and with the persistent launches recorded in a graph."""
    import torch
    import paper_1408_1782_amd as qb
    J, M = 4, 4
    mem = _batch_members(precision)
    dt, steps = 2.5e-4, 2
    batch = qb.Batch([problem(w, precision, J, M) for w, _ in mem])
    batch.set_persistent(persistent)
    Ws = [to_dev(w.W0, precision) for w, _ in mem]
    Bs = [None if B is None else torch.from_numpy(B).cuda().contiguous() for _, B in mem]
    moms = [torch.zeros((steps + 1, w.Nx, 7), dtype=torch.float64, device="cuda") for w, _ in mem]
    batch.step(Ws, Bs, dt, steps, moms, graph=graph)
    for k, (w, _) in enumerate(mem):
        plan = qb.Plan(problem(w, precision, J, M))
        plan.set_persistent(False)
        W = to_dev(w.W0, precision)
        m = torch.zeros((steps + 1, w.Nx, 7), dtype=torch.float64, device="cuda")
        plan.step(W, Bs[k], dt, steps, m)
        torch.cuda.synchronize()
        assert torch.equal(W, Ws[k]), k
        assert torch.equal(m, moms[k]), k
        plan.close()
    batch.close()


def test_batch_graph_replays_match_eager():
    """The recorded HIP graph, replayed three times with eager work in
    between, reproduces the eager batched run each time."""
    import torch
    import paper_1408_1782_amd as qb
    J, M = 4, 4
    mem = _batch_members("f32")
    dt, steps = 2.5e-4, 2
    batch = qb.Batch([problem(w, "f32", J, M) for w, _ in mem])
    init = [to_dev(w.W0, "f32") for w, _ in mem]
    Bs = [None if B is None else torch.from_numpy(B).cuda().contiguous() for _, B in mem]
    ref = [x.clone() for x in init]
    batch.step(ref, Bs, dt, steps)
    Ws = [x.clone() for x in init]
    for r in range(3):
        for W, x in zip(Ws, init):
            W.copy_(x)
        batch.step(Ws, Bs, dt, steps, graph=True)
        torch.cuda.synchronize()
        for k in range(len(mem)):
            assert torch.equal(Ws[k], ref[k]), (r, k)
        # unrelated eager work between replays
        a = torch.randn(256, 256, device="cuda")
        (a @ a).sum().item()
    batch.close()


def test_batch_chunked_launches():
    """A group of 600 cells runs its collision in two launches of the plan's
    workspace; the result matches the single-problem runs bitwise."""
    import torch
    import paper_1408_1782_amd as qb
    a = wl.config(2, Nx=300, N=16)
    b = wl.config(1, Nx=300, N=16)
    dt = 2.5e-4
    batch = qb.Batch([problem(w, "f32", 4, 4) for w in (a, b)])
    Ws = [to_dev(w.W0, "f32") for w in (a, b)]
    batch.step(Ws, None, dt, 1)
    for w, Wb in zip((a, b), Ws):
        plan = qb.Plan(problem(w, "f32", 4, 4))
        W = to_dev(w.W0, "f32")
        plan.step(W, None, dt, 1)
        torch.cuda.synchronize()
        assert torch.equal(W, Wb)
        plan.close()
    batch.close()


def test_batched_step_matches_oracle():
    """One batched step of three uneven problems (float64) against the
    oracle's splitting step for each."""
    import torch
    import paper_1408_1782_amd as qb
    J, M = 4, 4
    mem = _batch_members("f64")[:3]
    dt = 2.5e-4
    batch = qb.Batch([problem(w, "f64", J, M) for w, _ in mem])
    Ws = [to_dev(w.W0, "f64") for w, _ in mem]
    Bs = [None if B is None else torch.from_numpy(B).cuda().contiguous() for _, B in mem]
    batch.step(Ws, Bs, dt, 1)
    torch.cuda.synchronize()
    for (w, B), W in zip(mem, Ws):
        t = oc.Tables(w.N, w.L, w.R, J, M)
        Bn = np.zeros((w.Nx, 3)) if B is None else B
        s = ostep.step(pauli.to_pauli(w.W0), Bn, dt, w.L, w.R, J, M, bc_dict(w.left, w.N, w.L),
                       bc_dict(w.right, w.N, w.L), t)
        assert rel(pauli.to_pauli(W.cpu().numpy()), s) < 1e-11
    batch.close()
