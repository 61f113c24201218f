"""Pins of the oracle's scheme variants (Sec. 4: slope limiters other than
minmod; the field term as its exact flow instead of inside the Heun step)
against textbook forms and properties that do not use the variant's code:

* each limiter, written from the two one-sided differences, equals the
  ratio form sigma = a phi(b / a) of Sweby's diagram (minmod
  max(0, min(1, t)); superbee max(0, min(1, 2t), min(2, t)); monotonized
  central max(0, min((1 + t)/2, 2, 2t)); van Leer (t + |t|)/(1 + |t|)),
  with phi(1) = 1 (second order on linear data);
* every limited step conserves the periodic sum and is total-variation
  diminishing at CFL <= 1, and is second order on smooth data;
* the field flow keeps w0 and |w| and is a one-parameter group whose
  generator is the field term 2 B x w; for B along e_3 it is the closed-form
  rotation;
* the two splittings of the field agree to second order in dt;
* the flux form of the limited step (face fluxes written out from
  eq. slopeLimiterStep) gives back the step cell by cell, so the change of
  the total moments over a transport step is exactly the wall inflow.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import collision as oc
from oracle import pauli
from oracle import step as ostep
from oracle import transport as tp

L = 12.0

PHI = {
    "minmod": lambda t: np.maximum(0.0, np.minimum(1.0, t)),
    "superbee": lambda t: np.maximum.reduce([np.zeros_like(t), np.minimum(1.0, 2 * t), np.minimum(2.0, t)]),
    "mc": lambda t: np.maximum(0.0, np.minimum.reduce([(1 + t) / 2, 2.0 * np.ones_like(t), 2 * t])),
    "van_leer": lambda t: (t + np.abs(t)) / (1 + np.abs(t)),
}


@pytest.mark.parametrize("name", sorted(tp.LIMITERS))
def test_limiter_equals_ratio_form(name):
    rng = np.random.default_rng(0)
    a = rng.standard_normal(10000)
    a[np.abs(a) < 1e-3] = 1e-3
    b = rng.standard_normal(10000) * rng.choice([0.1, 1.0, 10.0], 10000)
    got = tp.LIMITERS[name](a, b)
    assert np.allclose(got, a * PHI[name](b / a), rtol=1e-14, atol=1e-15)
    assert np.all(got[a * b <= 0] == 0)
    one = np.array([1.0])
    assert PHI[name](one)[0] == 1.0 and tp.LIMITERS[name](one * 0.3, one * 0.3)[0] == 0.3


def _tv(w):
    return np.abs(np.diff(np.concatenate([w, w[:1]], axis=0), axis=0)).sum(axis=0)


@pytest.mark.parametrize("name", sorted(tp.LIMITERS))
def test_limited_step_conserves_and_is_tvd(name):
    rng = np.random.default_rng(1)
    Nx, N = 24, 8
    w = rng.standard_normal((Nx, N, N, 4))
    per = {"kind": "periodic"}
    dt = 0.9 / (L * Nx)  # |nu| <= 0.9
    tv0 = _tv(w)
    w1 = w
    for _ in range(5):
        w1 = tp.transport_step(w1, dt, per, per, L, name)
    assert np.allclose(w1.sum(axis=0), w.sum(axis=0), rtol=1e-13, atol=1e-12)
    assert np.all(_tv(w1) <= tv0 + 1e-12)


def test_limiters_are_second_order_on_smooth_data():
    """Advect a smooth periodic profile (exact solution: a shift by v t);
    halving dx at fixed CFL cuts the error about fourfold (a little less at
    the clipped extrema), and the compressive limiters beat minmod."""
    N = 8
    per = {"kind": "periodic"}
    errs = {}
    for name in tp.LIMITERS:
        e = []
        for Nx in (64, 128):
            x = (np.arange(Nx) + 0.5) / Nx
            vx = (2 * L / N) * (np.arange(N) - N // 2)
            dt = 0.5 / (L * Nx)
            steps = Nx // 4
            T = steps * dt
            prof = lambda xx: np.sin(2 * np.pi * xx) + 0.5 * np.cos(4 * np.pi * xx)
            # cell averages of the profile (exact for sines: sinc factors)
            avg = lambda xx, k: np.sinc(k / Nx)
            w = np.zeros((Nx, N, N, 4))
            w[..., 0] = (np.sin(2 * np.pi * x) * avg(x, 1) + 0.5 * np.cos(4 * np.pi * x) * avg(x, 2))[:, None, None]
            for _ in range(steps):
                w = tp.transport_step(w, dt, per, per, L, name)
            xs = x[:, None] - vx[None, :] * T
            ex = np.sin(2 * np.pi * xs) * avg(xs, 1) + 0.5 * np.cos(4 * np.pi * xs) * avg(xs, 2)
            e.append(np.abs(w[..., 0] - ex[:, :, None]).mean())
        errs[name] = e
        assert e[0] / e[1] > 2.5, (name, e)
    for name in ("superbee", "mc", "van_leer"):
        assert errs[name][1] < errs["minmod"][1]


def test_field_flow_is_the_rotation_generated_by_the_field_term():
    rng = np.random.default_rng(2)
    w = rng.standard_normal((3, 4, 4, 4))
    B = rng.standard_normal((3, 3))
    r = ostep.rotate(w, B, 0.37)
    assert np.allclose(r[..., 0], w[..., 0], rtol=0, atol=0)
    assert np.allclose(np.linalg.norm(r[..., 1:], axis=-1), np.linalg.norm(w[..., 1:], axis=-1), rtol=1e-14)
    assert np.allclose(ostep.rotate(ostep.rotate(w, B, 0.2), B, 0.17), r, rtol=1e-13, atol=1e-14)
    D = lambda s: (ostep.rotate(w, B, s) - ostep.rotate(w, B, -s)) / (2 * s)
    gen = (4 * D(5e-4) - D(1e-3)) / 3
    assert np.allclose(gen, ostep.magnetic(w, B), rtol=1e-9, atol=1e-11)
    Bz = np.array([[0.0, 0.0, 0.8]])
    w1 = np.zeros((1, 1, 1, 4))
    w1[..., 1] = 1.0
    th = 2 * 0.8 * 0.3
    assert np.allclose(ostep.rotate(w1, Bz, 0.3)[0, 0, 0], [0.0, np.cos(th), np.sin(th), 0.0], atol=1e-15)


def test_field_splittings_agree_to_second_order():
    """One step with the field inside Heun and one with its exact flow split
    around Heun differ by O(dt^3)."""
    Nx, N, J, M = 2, 8, 4, 4
    w0 = pauli.to_pauli(wl.config(2, Nx=Nx, N=N).W0)
    B = np.array([[0.3, -0.2, 0.5], [0.1, 0.4, -0.6]])
    t = oc.Tables(N, L, 7.5, J, M)
    per = {"kind": "periodic"}
    diff = []
    for dt in (4e-3, 2e-3):
        a = ostep.step(w0, B, dt, L, 7.5, J, M, per, per, t, field="heun")
        b = ostep.step(w0, B, dt, L, 7.5, J, M, per, per, t, field="rotation")
        diff.append(np.abs(a - b).max())
    assert diff[0] / diff[1] > 6.0, diff


@pytest.mark.parametrize("kind", ["periodic", "dirichlet", "maxwell"])
@pytest.mark.parametrize("name", ["minmod", "van_leer"])
def test_flux_form_reproduces_the_step(kind, name):
    """The face fluxes written out from eq. slopeLimiterStep give back the
    step cell by cell, so the change of the cell-summed moments is exactly
    the wall inflow."""
    rng = np.random.default_rng(8)
    Nx, N = 10, 8
    w = pauli.to_pauli(wl.config(3, Nx=Nx, N=N).W0) + 0.01 * rng.standard_normal((Nx, N, N, 4))
    v = (2 * L / N) * (np.arange(N) - N // 2)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    from oracle.fermi_dirac import fd_matrix
    st = lambda ikT: pauli.to_pauli(fd_matrix(vx, vy, ikT, 0.3, -0.2))
    if kind == "periodic":
        bl = br = {"kind": "periodic"}
    elif kind == "dirichlet":
        bl, br = {"kind": "dirichlet", "state": st(0.8)}, {"kind": "dirichlet", "state": st(2.0)}
    else:
        bl, br = {"kind": "dirichlet", "state": st(0.8)}, {"kind": "maxwell", "state": st(2.0), "alpha": 0.5}
    dt = 0.7 / (L * Nx)
    w1 = tp.transport_step(w, dt, bl, br, L, name)
    F = tp.face_fluxes(w, dt, bl, br, L, name)
    assert np.allclose(w1, w - dt * Nx * (F[1:] - F[:-1]), rtol=0, atol=1e-14 * np.abs(w).max())
    dm = ostep.moments(w1, L).sum(0) - ostep.moments(w, L).sum(0)
    inflow = tp.wall_inflow_moments(w, dt, bl, br, L, name)
    assert np.allclose(dm, inflow, rtol=0, atol=1e-12 * np.abs(ostep.moments(w, L)).sum(0).max())
    if kind == "periodic":
        assert np.abs(inflow).max() < 1e-13
