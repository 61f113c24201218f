"""Write the stored expected values of the GPU parity tests.

Calls only the CPU oracle (oracle/) on inputs from the seeded generators
(workloads/); nothing here touches the HIP library.  Run from the repository
root:  python tests/golden/make_golden.py [name ...]
Each output is an .npz next to this script:

  c1_trajectory.npz   configuration 1 in full (Nx = 16, N = 16, J = 32,
                      M = 16, dt = 1e-3, periodic, B = 0): Pauli state after
                      each of the 10 steps and the float64 moments.
  c2_reduced.npz      configuration 2 recipe on 8 cells (N = 32, J = 32,
                      M = 32, B = (0, 0, 0.5), dt = 1e-3): 2 steps.
  c3_cells.npz        configuration 3 (N = 64, J = 32, M = 64): C[W] of the
                      initial state at 8 sampled cells (both wall cells,
                      their neighbours and four interior cells).
  c5_reduced_grad.npz configuration 5 recipe on a reduced instance (Nx = 8,
                      N = 16, J = M = 8, 20 steps, dt = 1e-3, B = (0, 0, 0.5),
                      periodic): the final state, the observable
                      dx h^2 sum g(x_j) tr(sigma_z W(T)) and its gradients in
                      the initial Pauli state and in B.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import adjoint as oad  # noqa: E402
from oracle import collision as oc  # noqa: E402
from oracle import pauli  # noqa: E402
from oracle import step as ostep  # noqa: E402
from oracle.fermi_dirac import fd_matrix  # noqa: E402


def bc_dict(b, N, L):
    if b.kind == "periodic":
        return {"kind": "periodic"}
    v = (2 * L / N) * (np.arange(N) - N // 2)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    st = pauli.to_pauli(fd_matrix(vx, vy, b.inv_kT, b.mu_up, b.mu_down, b.U))
    return {"kind": b.kind, "state": st, "alpha": b.alpha}


def trajectory(w, steps):
    t = oc.Tables(w.N, w.L, w.R, w.J, w.M)
    s = pauli.to_pauli(w.W0)
    states, moms = [s], [ostep.moments(s, w.L)]
    bl, br = bc_dict(w.left, w.N, w.L), bc_dict(w.right, w.N, w.L)
    for k in range(steps):
        t0 = time.time()
        s = ostep.step(s, w.B, w.dt, w.L, w.R, w.J, w.M, bl, br, t)
        states.append(s)
        moms.append(ostep.moments(s, w.L))
        print(f"  step {k + 1}/{steps} {time.time() - t0:.1f} s", flush=True)
    return np.stack(states), np.stack(moms)


def make_c1():
    w = wl.config(1)
    states, moms = trajectory(w, w.steps)
    np.savez_compressed(os.path.join(HERE, "c1_trajectory.npz"), states=states, moments=moms)


def make_c2():
    w = wl.config(2, Nx=8)
    states, moms = trajectory(w, 2)
    np.savez_compressed(os.path.join(HERE, "c2_reduced.npz"), states=states, moments=moms)


C3_CELLS = (0, 1, 37, 101, 128, 200, 254, 255)


def make_c3():
    w = wl.config(3)
    t = oc.Tables(w.N, w.L, w.R, w.J, w.M)
    s = pauli.to_pauli(w.W0)
    out = []
    for c in C3_CELLS:
        t0 = time.time()
        out.append(oc.collision_pauli(s[c], w.L, w.R, w.J, w.M, t))
        print(f"  cell {c} {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "c3_cells.npz"), cells=np.array(C3_CELLS), c=np.stack(out))


C5_REDUCED = dict(Nx=8, N=16, J=8, M=8, steps=20)


def make_c5():
    r = C5_REDUCED
    w = wl.config(5, Nx=r["Nx"], N=r["N"])
    t = oc.Tables(w.N, w.L, w.R, r["J"], r["M"])
    per = {"kind": "periodic"}
    g = wl.adjoint_loss_weight(w.Nx)
    lam = oad.observable_weights(g, w.N, w.L)
    t0 = time.time()
    wT, gw, gB = oad.trajectory_gradient(pauli.to_pauli(w.W0), w.B, w.dt, r["steps"], lam, w.L, w.R,
                                         r["J"], r["M"], per, per, t)
    print(f"  {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "c5_reduced_grad.npz"), final=wT, loss=np.sum(lam * wT),
                        grad_w0=gw, grad_B=gB, weight=g)


if __name__ == "__main__":
    todo = sys.argv[1:] or ["c1", "c2", "c3", "c5"]
    for name in todo:
        print(name, flush=True)
        {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c5": make_c5}[name]()
