"""GPU parity of the scheme variants (qb_plan_set_scheme; Sec. 4: slope
limiters other than minmod, the field term as its exact flow split around
the collision step) against the oracle.  Bar as for the default scheme:
normwise relative error below 1e-11 (float64) and 2e-5 (float32)."""
import numpy as np
import pytest

import workloads as wl
from oracle import collision as oc
from oracle import pauli
from oracle import step as ostep
from oracle import transport as tp
from test_gpu_step import TOL, bc_dict, make_plan, rel, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("cfg", [2, 3])
@pytest.mark.parametrize("limiter", ["superbee", "mc", "van_leer"])
def test_transport_with_limiter_matches_oracle(limiter, cfg, precision):
    """Periodic (configuration 2) and Dirichlet / Maxwell walls
    (configuration 3), five steps at CFL 0.7."""
    import torch
    w = wl.config(cfg, Nx=24, N=16)
    plan = make_plan(w, precision, J=4, M=4)
    plan.set_scheme(limiter=limiter)
    Wd = to_dev(w.W0, precision)
    s = pauli.to_pauli(w.W0)
    bl, br = bc_dict(w.left, w.N, w.L), bc_dict(w.right, w.N, w.L)
    dt = 0.7 / (w.L * w.Nx)
    for _ in range(5):
        plan.transport_step(Wd, dt)
        s = tp.transport_step(s, dt, bl, br, w.L, limiter)
    torch.cuda.synchronize()
    got = pauli.to_pauli(Wd.cpu().numpy().astype(np.complex128))
    assert rel(got, s) < TOL[precision]
    plan.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("cfg,limiter", [(2, "minmod"), (3, "van_leer")])
def test_step_with_field_rotation_matches_oracle(cfg, limiter, precision):
    """T(dt/2) F(dt/2) Heun_C(dt) F(dt/2) T(dt/2), two steps, with the
    field of configuration 2 (uniform) and 3 (varying in x)."""
    import torch
    w = wl.config(cfg, Nx=6, N=16)
    J, M = 6, 6
    plan = make_plan(w, precision, J=J, M=M)
    plan.set_scheme(limiter=limiter, field="rotation")
    Wd = to_dev(w.W0, precision)
    B = torch.from_numpy(w.B).cuda().contiguous()
    plan.step(Wd, B, w.dt, 2)
    torch.cuda.synchronize()
    t = oc.Tables(w.N, w.L, w.R, J, M)
    s = pauli.to_pauli(w.W0)
    bl, br = bc_dict(w.left, w.N, w.L), bc_dict(w.right, w.N, w.L)
    for _ in range(2):
        s = ostep.step(s, w.B, w.dt, w.L, w.R, J, M, bl, br, t, limiter=limiter, field="rotation")
    got = pauli.to_pauli(Wd.cpu().numpy().astype(np.complex128))
    assert rel(got, s) < TOL[precision]
    plan.close()


def test_reverse_mode_rejects_variants():
    import torch
    import paper_1408_1782_amd as qb
    w = wl.config(2, Nx=4, N=16)
    plan = make_plan(w, "f64", J=4, M=4)
    plan.enable_adjoint()
    Wd = to_dev(w.W0, "f64")
    B = torch.from_numpy(w.B).cuda().contiguous()
    dt = 0.5 / (w.L * w.Nx)
    plan.set_scheme(limiter="mc")
    with pytest.raises(qb.QBError):
        plan.transport_vjp(Wd, dt, Wd)
    plan.set_scheme(field="rotation")
    with pytest.raises(qb.QBError):
        plan.step_trace(Wd, B, dt, 1, plan.new_trace(1))
    plan.set_scheme()
    plan.step_trace(Wd, B, dt, 1, plan.new_trace(1))
    torch.cuda.synchronize()
    plan.close()
