"""The wall inflow returned by qb_step_fluxes (moments of the net flux
through the two walls during each step, from the flux form of
eq. slopeLimiterStep) against the oracle's, and the conservation budget it
closes: the total density changes only through the walls (the collision
conserves it to quadrature accuracy and the field term leaves w0 alone).
Bars as for the step: 1e-11 (float64) and 2e-5 (float32) normwise."""
import numpy as np
import pytest

import workloads as wl
from oracle import collision as oc
from oracle import pauli
from oracle import step as ostep
from oracle import transport as tp
from test_gpu_step import TOL, bc_dict, make_plan, rel, to_dev

pytestmark = pytest.mark.gpu


def _oracle_inflow(w0, B, dt, steps, L, J, M, bl, br, t):
    s = w0
    out, moms = [], [ostep.moments(s, L).sum(0)]
    for _ in range(steps):
        a = tp.wall_inflow_moments(s, 0.5 * dt, bl, br, L)
        s = tp.transport_step(s, 0.5 * dt, bl, br, L)
        s = ostep.heun(s, B, dt, L, t)
        out.append(a + tp.wall_inflow_moments(s, 0.5 * dt, bl, br, L))
        s = tp.transport_step(s, 0.5 * dt, bl, br, L)
        moms.append(ostep.moments(s, L).sum(0))
    return np.stack(out), s, np.stack(moms)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_wall_inflow_matches_oracle_on_the_slab(precision):
    import torch
    w = wl.config(3, Nx=12, N=16)
    J, M = 4, 4
    plan = make_plan(w, precision, J=J, M=M)
    Wd = to_dev(w.W0, precision)
    B = torch.from_numpy(w.B).cuda().contiguous()
    steps = 3
    dt = 0.7 / (w.L * w.Nx)
    inflow = torch.zeros((steps, 7), dtype=torch.float64, device="cuda")
    mom = torch.zeros((steps + 1, w.Nx, 7), dtype=torch.float64, device="cuda")
    plan.step(Wd, B, dt, steps, mom, inflow)
    torch.cuda.synchronize()
    t = oc.Tables(w.N, w.L, w.R, J, M)
    bl, br = bc_dict(w.left, w.N, w.L), bc_dict(w.right, w.N, w.L)
    ref, s, ref_m = _oracle_inflow(pauli.to_pauli(w.W0), w.B, dt, steps, w.L, J, M, bl, br, t)
    got = inflow.cpu().numpy()
    for k in range(7):
        assert np.abs(got[:, k] - ref[:, k]).max() <= TOL[precision] * np.abs(ref[:, k]).max() + 1e-300, k
    assert rel(pauli.to_pauli(Wd.cpu().numpy().astype(np.complex128)), s) < TOL[precision]
    # budget residual (total change minus wall inflow: what the collision
    # and field sub-steps changed; with this coarse quadrature J = M = 4 the
    # collision's density error is large) equal on both sides, per moment
    m = mom.cpu().numpy().sum(axis=1)
    res = (m[-1] - m[0]) - got.sum(axis=0)
    ref_res = (ref_m[-1] - ref_m[0]) - ref.sum(axis=0)
    assert np.all(np.abs(res - ref_res) <= TOL[precision] * np.abs(ref_m).max(axis=0))
    plan.close()


def test_density_budget_closes_with_the_working_quadrature():
    """With J = 32 and M = N the collision conserves density to quadrature
    accuracy, so the total density changes only through the walls."""
    import torch
    w = wl.config(3, Nx=12, N=16)
    plan = make_plan(w, "f64", J=32, M=16)
    Wd = to_dev(w.W0, "f64")
    B = torch.from_numpy(w.B).cuda().contiguous()
    steps = 3
    dt = 0.7 / (w.L * w.Nx)
    inflow = torch.zeros((steps, 7), dtype=torch.float64, device="cuda")
    mom = torch.zeros((steps + 1, w.Nx, 7), dtype=torch.float64, device="cuda")
    plan.step(Wd, B, dt, steps, mom, inflow)
    torch.cuda.synchronize()
    m = mom.cpu().numpy().sum(axis=1)
    inf = inflow.cpu().numpy().sum(axis=0)
    assert abs(inf[0]) > 1e-3 * abs(m[0, 0])  # the walls do move density
    assert abs((m[-1, 0] - m[0, 0]) - inf[0]) < 1e-6 * abs(m[0, 0])
    plan.close()


def test_periodic_walls_have_no_inflow():
    import torch
    w = wl.config(2, Nx=8, N=16)
    plan = make_plan(w, "f64", J=4, M=4)
    Wd = to_dev(w.W0, "f64")
    inflow = torch.ones((2, 7), dtype=torch.float64, device="cuda")
    plan.step(Wd, None, w.dt, 2, None, inflow)
    torch.cuda.synchronize()
    assert np.abs(inflow.cpu().numpy()).max() < 1e-13
    plan.close()
