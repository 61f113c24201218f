#!/usr/bin/env python
"""Throughput of the splitting time step on the 64 x 64 velocity grid.

Workload: the wall-bounded slab (Nx = 256 cells, N = 64, J = 32, M = 64,
L = 12, R = 7.5; Dirichlet inflow on the left, Maxwell wall alpha = 0.5 on
the right; smooth seeded field B with max |B| = 1; dt = 5e-4), seeded
synthetic initial data, float32 bulk with float64 moments, and the same
shape in float64.  One step = transport dt/2, Heun step of C[W] + field term,
transport dt/2, float64 moments.  The metric is cells * steps / s over the
whole job (one GPU), timed with the state already resident in HBM.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "cells*steps/s at 64x64 momentum grid (FP64 vs FP32); adjoint/forward time ratio"
PEAK = {"f32": 157.3, "f64": 78.6}   # TFLOP/s, MI355X datasheet vector peaks


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC = os.path.join(HERE, "profiles", "k_i3_slab_N64_traffic.json")
KERNEL_SOURCES = ("qb_fft.hpp", "qb_kernels.hpp", "qb_pipelines.hpp")


def kernel_source_hash():
    """sha256 over the sources of the forward collision kernels."""
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "paper_1408_1782_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(precision, tile):
    """HBM bytes per k_i3 launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes (scaled by a copy kernel of known size), or None when
    they were taken on other kernel sources or another configuration."""
    try:
        with open(TRAFFIC) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    ok = (t.get("source_sha256") == kernel_source_hash() and t.get("precision") == precision
          and t.get("tile") == tile)
    return t.get("bytes_per_launch") if ok else None


def copy_calibration(mib=512):
    """One run of the library's copy probe over `mib` MiB (a kernel of known
    traffic: it reads and writes mib MiB), for scaling the HBM byte counters.
    (Every bench run also makes the probe's 1 GiB dispatches for its
    ceilings; either serves.)"""
    from paper_1408_1782_amd import _lib

    _lib.probe_copy(mib, 1)
    log(f"copy calibration: {mib} MiB read, {mib} MiB written by the copy probe")


def i3_transforms(J, M, paired):
    """Complex P x P transforms of one I_3 evaluation per cell.  Unpaired:
    per (j, m) 2 packed shift transforms + 8 packed convolutions of two
    transforms = 18.  Paired Gauss-Legendre nodes (m, M-1-m): 2 shifts + 16
    convolution transforms + 2 transforms of the partner sums = 20 per pair,
    18 for the middle node of an odd M."""
    if not paired:
        return J * M * 18
    return J * ((M // 2) * 20 + (M % 2) * 18)


def i3_flops(ncells, N, J, M, paired):
    """Flops of one I_3 launch at 5 n log2 n per complex transform of
    n = (2N)^2 points, for the decomposition the kernel runs."""
    n = (2 * N) ** 2
    return ncells * i3_transforms(J, M, paired) * 5.0 * n * math.log2(n)


def i3_flops_algorithmic(ncells, N, J, M):
    """Flops of one I_3 evaluation by the method's own operation count: per
    (j, m) four shifted fields and sixteen convolutions of two real fields,
    each transform complex and unpacked, 36 P x P transforms (4 shift +
    16 x 2 convolution), at 5 n log2 n, n = P^2.  Packing two real fields
    per complex transform and pairing the symmetric nodes are the kernel's
    savings against this count."""
    n = (2 * N) ** 2
    return ncells * 36 * J * M * 5.0 * n * math.log2(n)


def i3_io_bytes(ncells, N, J, scalar):
    """Bytes a perfect I_3 kernel moves per launch: per cell the inputs it
    needs (the four Pauli spectra, complex, 8 planes, and the five P-grid
    fields w_mu, f0) read once and its outputs (four real-space sums and
    four planes of node-pair spectra) written once, P^2 scalars each."""
    P = 2 * N
    return ncells * (8 + 5 + 4 + 4) * P * P * scalar



def measure_ceilings():
    """Sustained vector FMA rates and device copy bandwidth of this GPU
    (qb_probe_fma / qb_probe_copy), beside the datasheet peaks."""
    from paper_1408_1782_amd import _lib

    c = {"fma_f32_TFLOPs": _lib.probe_fma("f32", 4096), "fma_f64_TFLOPs": _lib.probe_fma("f64", 4096),
         "copy_GBps": _lib.probe_copy(1024)}
    log(f"measured ceilings: {c}")
    return c


def equilibrium_residual(wl):
    """max |C[W_FD]| over the velocity grid for the Fermi-Dirac state
    (beta = 1, mu = 0; C vanishes on it up to discretisation, Sec. 2) on the
    slab's grid and quadrature, relative to max |C| of the slab's perturbed
    initial cells, in float64 and float32 (the float32 figure shows the
    rounding floor of the bulk path)."""
    import torch
    import paper_1408_1782_amd as qb
    import workloads

    v = workloads.velocity_axis(wl.N, wl.L)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    f = workloads.fd_occupation(vx, vy, 1.0, 0.0)
    fd = np.zeros((1, wl.N, wl.N, 2, 2), np.complex128)
    fd[0, ..., 0, 0] = fd[0, ..., 1, 1] = f
    out = {}
    for precision in ("f64", "f32"):
        cdt = torch.complex128 if precision == "f64" else torch.complex64
        plan = qb.Plan(qb.Problem(4, wl.N, wl.J, wl.M, wl.L, wl.R, precision))
        W = torch.from_numpy(np.concatenate([fd, wl.W0[:3]])).to(cdt).cuda().contiguous()
        C = plan.collision(W).cpu().numpy()
        plan.close()
        out[precision] = float(np.abs(C[0]).max() / np.abs(C[1:]).max())
    log(f"equilibrium residual: {out}")
    return out


def run_gpu(wl, precision, steps, warmup):
    import torch
    import paper_1408_1782_amd as qb

    cdt = torch.complex64 if precision == "f32" else torch.complex128
    prob = qb.Problem(wl.Nx, wl.N, wl.J, wl.M, wl.L, wl.R, precision,
                      qb.BC.from_workload(wl.left), qb.BC.from_workload(wl.right))
    plan = qb.Plan(prob)
    plan.tune()
    cfg = plan.config()
    log(f"[{precision}] tuned tile E = {cfg['tile']}")
    W = torch.from_numpy(wl.W0).to(cdt).cuda().contiguous()
    B = torch.from_numpy(wl.B).cuda().contiguous()
    mom = torch.zeros((steps + 1, wl.Nx, 7), dtype=torch.float64, device="cuda")
    if warmup > 0:
        log(f"[{precision}] warmup {warmup} step(s)")
        plan.step(W, B, wl.dt, warmup, torch.zeros((warmup + 1, wl.Nx, 7), dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
    plan.profile(True)
    for k in qb._lib.KERNELS:
        plan.profile_read(k)     # discard anything recorded before
    inflow = torch.zeros((steps, 7), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.step(W, B, wl.dt, steps, mom, inflow)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"[{precision}] {steps} step(s) in {t1 - t0:.3f} s")
    kern = {k: plan.profile_read(k) for k in qb._lib.KERNELS}
    # the two launch shapes of the collision kernels on the same plan
    ab = {}
    C = torch.empty_like(W)
    for persistent in (False, True):
        plan.set_persistent(persistent)
        plan.collision(W, C)
        torch.cuda.synchronize()
        for k in qb._lib.KERNELS:
            plan.profile_read(k)
        plan.collision(W, C)
        torch.cuda.synchronize()
        ab["persistent" if persistent else "per_task"] = {"i3_ms": plan.profile_read("i3")[0],
                                                          "terms_ms": plan.profile_read("terms")[0]}
    plan.set_persistent(cfg["persistent"])
    cfg = dict(cfg, launch_ab=ab)
    log(f"[{precision}] launch shapes: {ab}")
    plan.profile(False)
    m = mom.cpu().numpy()
    tot0, tot1 = m[0].sum(0), m[-1].sum(0)
    plan.close()
    final = {"W": _pauli_np(W.cpu().numpy().astype(np.complex128)), "moments": m[-1],
             "inflow": inflow.cpu().numpy().sum(axis=0)}
    return t1 - t0, kern, tot0, tot1, cfg, final


def run_adjoint(steps, every):
    """Adjoint/forward time ratio on the configuration-5 workload (Nx = 128,
    N = 32, J = 32, M = 32, complex128, periodic, B = (0, 0, 0.5), dt = 1e-3):
    `steps` plain forward steps (qb_step) against the backward pass of the
    checkpointed autograd integration (recompute each segment with
    qb_step_trace, then qb_adjoint_step per step), for the gradient of
    dx h^2 sum g(x_j) tr(sigma_z W(T)) in W0 and B."""
    import torch
    import paper_1408_1782_amd as qb
    import workloads

    wl = workloads.config(5)
    plan = qb.Plan(qb.Problem(wl.Nx, wl.N, wl.J, wl.M, wl.L, wl.R, "f64"))
    plan.enable_adjoint()
    plan.tune()
    cfg = plan.config()
    W0 = torch.from_numpy(wl.W0).cuda().contiguous()
    B = torch.from_numpy(wl.B).cuda().contiguous()
    h2 = (2 * wl.L / wl.N) ** 2
    g = torch.from_numpy(workloads.adjoint_loss_weight(wl.Nx)).cuda()

    def loss_of(WT):
        return h2 / wl.Nx * (g[:, None, None] * (WT[..., 0, 0] - WT[..., 1, 1]).real).sum()

    # warm-up: one forward and one reverse step
    Wr = W0.clone().requires_grad_(True)
    loss_of(qb.evolve(plan, Wr, B, wl.dt, 1, every)).backward()
    torch.cuda.synchronize()
    W = W0.clone()
    t0 = time.perf_counter()
    plan.step(W, B, wl.dt, steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    log(f"[adjoint] forward {steps} steps {t_fwd:.3f} s")
    def grad_run(k):
        Wr = W0.clone().requires_grad_(True)
        Br = B.clone().requires_grad_(True)
        t0 = time.perf_counter()
        loss = loss_of(qb.evolve(plan, Wr, Br, wl.dt, steps, k))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        log(f"[adjoint] checkpoint_every={k}: forward {t1 - t0:.3f} s, backward {t2 - t1:.3f} s")
        return t1 - t0, t2 - t1, Wr.grad, Br.grad

    f_ck, b_ck, gW, gB = grad_run(every)
    f_all, b_all, gW2, gB2 = grad_run(0)
    # the checkpoints pass through the complex layout, so the two modes agree
    # to rounding, not bitwise
    diff = max(float((gW - gW2).abs().max() / gW2.abs().max()), float((gB - gB2).abs().max() / gB2.abs().max()))
    plan.close()
    return {"workload": "adjoint_fd_periodic_B", "Nx": wl.Nx, "N": wl.N, "J": wl.J, "M": wl.M, "dtype": "f64",
            "tile": cfg["tile"], "adjoint_tile": cfg["adjoint_tile"], "adjoint_variant": cfg["adjoint_variant"],
            "steps": steps, "checkpoint_every": every, "forward_s": t_fwd,
            "checkpointed": {"forward_s": f_ck, "backward_s": b_ck, "ratio": b_ck / t_fwd,
                             "recomputed_steps": steps - min(every, steps - every * ((steps - 1) // every))},
            "store_all": {"forward_s": f_all, "backward_s": b_all, "ratio": b_all / t_fwd},
            "ratio": b_ck / t_fwd, "gradient_rel_diff_between_modes": diff,
            "grad_norms": {"W0": float(gW.abs().max()), "B": float(gB.abs().max())}}


def run_batch(steps, nprob, replays=1, sub_replays=None):
    """Batched throughput on the uneven-batch workload (64 periodic problems,
    Nx ~ U{32, 64, 128, 256, 512}, N ~ U{32, 64}, J = 32, M = N, B = 0,
    dt = 2.5e-4, float32 with float64 moments): tile and launch-shape
    autotuning, then one call of `steps` steps recorded as a HIP graph
    (capture, instantiation and its first launch, reported as capture_s),
    then that graph replayed `replays` times, each replay timed alone (the
    `value` is cells * steps * replays over the replay time).  The N = 64
    problems alone are timed the same way as a second batch, with
    `sub_replays` replays (default `replays`; 0 skips it)."""
    import torch
    import paper_1408_1782_amd as qb
    import workloads

    wls = workloads.batch_config(nprob, steps)

    def one(sel, label, replays):
        probs = [qb.Problem(w.Nx, w.N, w.J, w.M, w.L, w.R, "f32") for w in sel]
        batch = qb.Batch(probs)
        batch.tune()
        Ws = [torch.from_numpy(w.W0).to(torch.complex64).cuda().contiguous() for w in sel]
        moms = [torch.zeros((steps + 1, w.Nx, 7), dtype=torch.float64, device="cuda") for w in sel]
        cells = sum(w.Nx for w in sel)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.step(Ws, None, wls[0].dt, steps, moms, graph=True)   # capture + first launch
        torch.cuda.synchronize()
        capture = time.perf_counter() - t0
        log(f"[batch {label}] {len(sel)} problems, {cells} cells, {steps}-step graph: capture + first run {capture:.3f} s")
        times = []
        for r in range(replays):
            t1 = time.perf_counter()
            batch.step(Ws, None, wls[0].dt, steps, moms, graph=True)   # replay of the recorded graph
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
            log(f"[batch {label}] replay {r + 1}/{replays}: {times[-1]:.3f} s")
        finite = all(bool(torch.isfinite(torch.view_as_real(W)).all()) for W in Ws)
        batch.close()
        return {"problems": len(sel), "cells": cells, "capture_s": capture, "replays": replays,
                "replay_s": times, "value": cells * steps * replays / sum(times), "finite": finite}

    full = one(wls, "all", replays)
    sr = replays if sub_replays is None else sub_replays
    sub = one([w for w in wls if w.N == 64], "N=64", sr) if sr > 0 else None
    return {"workload": "uneven_batch", "unit": "cells*steps/s", "dtype": "f32", "steps_per_graph": steps,
            "replayed_steps": steps * replays, "graph": "captured once, replayed", "all": full, "N64": sub,
            "N32_cells": sum(w.Nx for w in wls if w.N == 32)}


BATCH_RECORD = os.path.join(HERE, "profiles", "batch_uneven_64problems_50steps.json")


def batch_record():
    """The committed 50-step run of the uneven batch (a 5-step graph
    captured once and replayed 10 times, about 14 minutes, too long for the
    default line): its command, replayed steps and cells*steps/s, or None."""
    try:
        with open(BATCH_RECORD) as f:
            r = json.load(f)
        a = r["result"]["all"]
        return {"file": os.path.relpath(BATCH_RECORD, HERE), "command": r["command"],
                "replayed_steps": r["result"]["replayed_steps"], "capture_s": a["capture_s"],
                "value": a["value"], "unit": r["result"]["unit"]}
    except (OSError, ValueError, KeyError):
        return None


SLAB_RECORD = os.path.join(HERE, "profiles", "slab_dirichlet_maxwell_500steps_f32.json")


def slab_record():
    """The committed 500-step float32 run of the slab (about 5 minutes):
    its command and the final drift and budget residuals, or None."""
    try:
        with open(SLAB_RECORD) as f:
            r = json.load(f)
        last = r["result"]["record"][-1]
        return {"file": os.path.relpath(SLAB_RECORD, HERE), "command": r["command"], "steps": last["step"],
                "cells*steps/s": r["result"]["cells*steps/s"],
                **{k: last[k] for k in ("density_drift", "energy_drift", "density_budget_residual",
                                        "energy_budget_residual")}}
    except (OSError, ValueError, KeyError, IndexError):
        return None


def run_slab_record(steps, chunk=25):
    """The wall-bounded slab in float32 (float64 moments) for `steps` steps
    from its initial state, in calls of `chunk` steps: the total moments
    after every call, their drift, and the conservation budget (the change
    of the totals minus the moments that entered through the walls, from
    qb_step_fluxes), relative to the initial totals."""
    import torch
    import paper_1408_1782_amd as qb
    import workloads

    wl = workloads.config(3)
    prob = qb.Problem(wl.Nx, wl.N, wl.J, wl.M, wl.L, wl.R, "f32",
                      qb.BC.from_workload(wl.left), qb.BC.from_workload(wl.right))
    plan = qb.Plan(prob)
    plan.tune()
    W = torch.from_numpy(wl.W0).to(torch.complex64).cuda().contiguous()
    B = torch.from_numpy(wl.B).cuda().contiguous()
    rows, inflow_total = [], np.zeros(7)
    t0 = time.perf_counter()
    done = 0
    tot0 = None
    while done < steps:
        k = min(chunk, steps - done)
        mom = torch.zeros((k + 1, wl.Nx, 7), dtype=torch.float64, device="cuda")
        inflow = torch.zeros((k, 7), dtype=torch.float64, device="cuda")
        plan.step(W, B, wl.dt, k, mom, inflow)
        m = mom.cpu().numpy().sum(axis=1)
        if tot0 is None:
            tot0 = m[0]
        inflow_total += inflow.cpu().numpy().sum(axis=0)
        done += k
        tot = m[-1]
        rows.append({"step": done, "totals": tot.tolist(),
                     "density_drift": float((tot[0] - tot0[0]) / tot0[0]),
                     "energy_drift": float((tot[6] - tot0[6]) / tot0[6]),
                     "density_budget_residual": float((tot[0] - tot0[0] - inflow_total[0]) / tot0[0]),
                     "energy_budget_residual": float((tot[6] - tot0[6] - inflow_total[6]) / tot0[6])})
        log(f"[slab record] step {done}/{steps} ({time.perf_counter() - t0:.1f} s): "
            f"density drift {rows[-1]['density_drift']:.3e}, budget residual "
            f"{rows[-1]['density_budget_residual']:.3e} (density) {rows[-1]['energy_budget_residual']:.3e} (energy)")
    elapsed = time.perf_counter() - t0
    finite = bool(torch.isfinite(torch.view_as_real(W)).all())
    plan.close()
    return {"workload": "dirichlet_maxwell_slab", "Nx": wl.Nx, "N": wl.N, "J": wl.J, "M": wl.M, "dt": wl.dt,
            "dtype": "f32 bulk, f64 moments", "steps": steps, "seconds": elapsed,
            "cells*steps/s": wl.Nx * steps / elapsed, "initial_totals": tot0.tolist(),
            "inflow_total": inflow_total.tolist(), "finite": finite, "record": rows}


def cpu_baseline(wl):
    """The CPU oracle on a bounded sample of the same workload: one collision
    evaluation of one cell plus one transport half-step over all cells."""
    import numpy as np
    from oracle import collision as oc
    from oracle import pauli
    from oracle import transport as tp
    from oracle.fermi_dirac import fd_matrix

    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    w = pauli.to_pauli(wl.W0)
    t = oc.Tables(wl.N, wl.L, wl.R, wl.J, wl.M)
    t0 = time.perf_counter()
    oc.collision_pauli(w[0], wl.L, wl.R, wl.J, wl.M, t)
    t_eval = time.perf_counter() - t0
    v = (2 * wl.L / wl.N) * (np.arange(wl.N) - wl.N // 2)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    def bc(b):
        if b.kind == "periodic":
            return {"kind": "periodic"}
        st = pauli.to_pauli(fd_matrix(vx, vy, b.inv_kT, b.mu_up, b.mu_down, b.U))
        return {"kind": b.kind, "state": st, "alpha": b.alpha}
    t0 = time.perf_counter()
    tp.transport_step(w, 0.5 * wl.dt, bc(wl.left), bc(wl.right), wl.L)
    t_tr = (time.perf_counter() - t0) / wl.Nx
    rate = 1.0 / (2 * t_eval + 2 * t_tr)
    return {
        "value": rate,
        "unit": "cells*steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"1 cell x 1 collision evaluation (N={wl.N}, J={wl.J}, M={wl.M}, "
                   f"{t_eval:.1f} s) + 1 transport half-step over {wl.Nx} cells; "
                   "rate = 1 / (2 t_eval + 2 t_transport_per_cell)"),
    }


def _pauli_np(C):
    """Pauli components c_mu = (1/2) Re tr(sigma_mu C) of [..., 2, 2] -> [4, ...]."""
    return np.stack([0.5 * (C[..., 0, 0] + C[..., 1, 1]).real, 0.5 * (C[..., 0, 1] + C[..., 1, 0]).real,
                     0.5 * (C[..., 1, 0] - C[..., 0, 1]).imag, 0.5 * (C[..., 0, 0] - C[..., 1, 1]).real])


def _fourier(c):
    """Mean-value Fourier coefficients on Xi of the components c[4, N, N],
    centred (frequency xi at index xi + N/2 on each axis)."""
    N = c.shape[-1]
    return np.fft.fftshift(np.fft.fft2(c), axes=(-2, -1)) / (N * N)


def rel_l1(c, ref):
    """sum_j ||C_j - C_ref,j||_1 / ||C_ref,j||_1 over the Pauli components
    whose reference is not zero (C_c,0 vanishes identically; its rounding
    noise, below 1e-12 of the largest component, is skipped), L1 norms of
    the Fourier coefficients (Sec. 5.1).  For a smaller grid than the
    reference the coefficients are compared on the common frequencies and
    the reference's other coefficients count as error."""
    a, b = _fourier(c), _fourier(ref)
    n, m = a.shape[-1], b.shape[-1]
    o = (m - n) // 2
    d = b.copy()
    d[:, o:o + n, o:o + n] -= a
    norms = [np.abs(b[j]).sum() for j in range(4)]
    err = 0.0
    for j in range(4):
        if norms[j] > 1e-12 * max(norms):
            err += np.abs(d[j]).sum() / norms[j]
    return err


def run_convergence(precision="f64"):
    """Convergence of C_c and C_d on the validation state (Sec. 5.1) with
    the number of angles J, Gauss-Legendre radii M and grid points N,
    against J = 72, M = 72 and N = 64 (the largest grid here)."""
    import torch
    import paper_1408_1782_amd as qb
    import workloads

    L, R = workloads.L_BOX, workloads.R_TRUNC
    cache = {}

    def parts(N, J, M):
        key = (N, J, M)
        if key not in cache:
            plan = qb.Plan(qb.Problem(1, N, J, M, L, R, precision))
            cd = torch.complex128 if precision == "f64" else torch.complex64
            W = torch.from_numpy(workloads.validation_state(N, L)[None]).to(cd).cuda().contiguous()
            out = {}
            for t in ("conservative", "dissipative"):
                plan.set_terms(t)
                out[t] = _pauli_np(plan.collision(W).cpu().numpy()[0].astype(np.complex128))
            plan.close()
            cache[key] = out
        return cache[key]

    def sweep(vals, key, ref_key):
        ref = parts(*ref_key)
        rows = []
        for v in vals:
            got = parts(*key(v))
            rows.append({"value": v, "C_c": rel_l1(got["conservative"], ref["conservative"]),
                         "C_d": rel_l1(got["dissipative"], ref["dissipative"])})
            log(f"[convergence] {key(v)} vs {ref_key}: C_c {rows[-1]['C_c']:.3e}  C_d {rows[-1]['C_d']:.3e}")
        return rows

    grid = [8, 12, 16, 20, 24, 28, 32, 40, 48, 56, 64]
    return {
        "study": "collision convergence on the validation state (Sec. 5.1)",
        "precision": precision, "L": L, "R": R,
        "J": {"fixed": {"N": 32, "M": 32}, "reference": 72, "rows": sweep(grid, lambda v: (32, v, 32), (32, 72, 32))},
        "M": {"fixed": {"N": 32, "J": 32}, "reference": 72, "rows": sweep(grid, lambda v: (32, 32, v), (32, 32, 72))},
        "N": {"fixed": {"J": 32, "M": 72}, "reference": 64,
              "rows": sweep([16, 32], lambda v: (v, 32, 72), (64, 32, 72))},
        "error": "sum over Pauli components of relative L1 norms of Fourier coefficients",
    }


PHYSICS_RUNS = ("E2", "E3", "E4", "E5", "E6i", "E6ii")


def _rho_matrix(m):
    """2x2 spin density sum_mu rho_mu sigma_mu from moment columns 0..3."""
    import workloads
    return np.einsum("...m,mij->...ij", m[..., :4], workloads.SIGMA)


def _spin_basis(rho):
    """Eigenbasis of a 2x2 spin density as U = [e_up, e_down] (columns)."""
    lam, V = np.linalg.eigh(rho)
    return V[:, ::-1]


def run_physics(name, precision="f64", samples=20, t_end=None, Nx=None, N=32):
    """One of the simulations of Sec. 5.2 and 5.3 on the GPU (workloads
    physics_run), sampled `samples` times: total moments, entropy and its
    production, relative entropies (to the global equilibrium where the
    moments fix one, and to the local fits), eigenvalue range; for the
    homogeneous run the L1 distance to the equilibrium, for the wall runs
    the change of the state between samples and the final x-profiles of the
    density, local temperature and local entropy."""
    import torch
    import paper_1408_1782_amd as qb
    import workloads

    wl = workloads.physics_run(name, N=N, Nx=Nx, t_end=t_end)
    cd = torch.complex128 if precision == "f64" else torch.complex64
    prob = qb.Problem(wl.Nx, wl.N, wl.J, wl.M, wl.L, wl.R, precision,
                      qb.BC.from_workload(wl.left), qb.BC.from_workload(wl.right))
    plan = qb.Plan(prob)
    W = torch.from_numpy(wl.W0).to(cd).cuda().contiguous()
    B = torch.from_numpy(wl.B).cuda().contiguous()
    dx, h2 = 1.0 / wl.Nx, (2 * wl.L / wl.N) ** 2
    periodic = wl.left.kind == "periodic"
    m0 = plan.moments(W).cpu().numpy()
    tot0 = dx * m0.sum(0)

    # equilibrium fixed by the conserved totals: the local fit of the
    # cell-averaged state (moments are linear in W), spin basis of its density
    fd, fd_fit = None, None
    if periodic:
        one = qb.Plan(qb.Problem(1, wl.N, wl.J, wl.M, wl.L, wl.R, precision))
        avg = W.mean(dim=0, keepdim=True).contiguous()
        d = one.diagnostics(avg).cpu().numpy()[0]
        one.close()
        fd_fit = {"kT": d[6], "mu_up": d[7], "mu_down": d[8], "u": [d[9], d[10]]}
        U = _spin_basis(_rho_matrix(tot0))
        fd_fit["U"] = [[[z.real, z.imag] for z in row] for row in U]
        if wl.Nx > 1:
            fd = (1.0 / d[6], d[7], d[8], U)
        if wl.Nx == 1:
            v = workloads.velocity_axis(wl.N, wl.L)
            vx, vy = np.meshgrid(v - d[9], v - d[10], indexing="ij")
            D = np.zeros((wl.N, wl.N, 2, 2), np.complex128)
            D[..., 0, 0] = workloads.fd_occupation(vx, vy, 1.0 / d[6], d[7])
            D[..., 1, 1] = workloads.fd_occupation(vx, vy, 1.0 / d[6], d[8])
            wfd = _pauli_np(U @ D @ np.conj(U.T))

    every = max(1, wl.steps // samples)
    series = {k: [] for k in ("t", "density_rel_dev", "trace_density_rel_dev", "momentum_dev", "energy_rel_dev", "entropy",
                              "entropy_production", "rel_entropy_global", "rel_entropy_local",
                              "eig_min", "eig_max", "l1_to_fd", "state_change_rate")}
    prev = None
    done = 0
    t0 = time.perf_counter()
    gpu_s = 0.0
    while True:
        C = plan.collision(W)
        dg = plan.diagnostics(W, C, fd=fd).cpu().numpy()
        m = plan.moments(W).cpu().numpy()
        tot = dx * m.sum(0)
        Wh = W.cpu().numpy()
        series["t"].append(done * wl.dt)
        series["density_rel_dev"].append(float(np.linalg.norm(_rho_matrix(tot) - _rho_matrix(tot0))
                                               / np.linalg.norm(_rho_matrix(tot0))))
        series["trace_density_rel_dev"].append(float(abs(tot[0] - tot0[0]) / abs(tot0[0])))
        series["momentum_dev"].append(float(np.abs(tot[4:6] - tot0[4:6]).max() / (2 * tot0[0])))
        series["energy_rel_dev"].append(float(abs(tot[6] - tot0[6]) / abs(tot0[6])))
        series["entropy"].append(float(dx * dg[:, 0].sum()))
        series["entropy_production"].append(float(dx * dg[:, 1].sum()))
        series["rel_entropy_global"].append(float(dx * dg[:, 2].sum()) if fd is not None else None)
        series["rel_entropy_local"].append(float(dx * dg[:, 3].sum()))
        series["eig_min"].append(float(dg[:, 4].min()))
        series["eig_max"].append(float(dg[:, 5].max()))
        if periodic and wl.Nx == 1:
            series["l1_to_fd"].append(float(h2 * np.abs(_pauli_np(Wh[0]) - wfd).sum()))
        else:
            series["l1_to_fd"].append(None)
        if prev is not None:
            series["state_change_rate"].append(float(np.abs(Wh - prev).max() / (every * wl.dt)))
        else:
            series["state_change_rate"].append(None)
        prev = Wh
        if done >= wl.steps:
            break
        k = min(every, wl.steps - done)
        torch.cuda.synchronize()
        a = time.perf_counter()
        plan.step(W, B, wl.dt, k)
        torch.cuda.synchronize()
        gpu_s += time.perf_counter() - a
        done += k
        log(f"[physics {name}] t = {done * wl.dt:.3f}  S = {series['entropy'][-1]:.10f}")
    x = workloads.cell_centres(wl.Nx)
    out = {
        "run": name, "precision": precision, "Nx": wl.Nx, "N": wl.N, "J": wl.J, "M": wl.M, "L": wl.L,
        "R": wl.R, "dt": wl.dt, "steps": wl.steps, "t_end": wl.steps * wl.dt,
        "walls": [wl.left.kind, wl.right.kind],
        "step_seconds": gpu_s, "cells_steps_per_s": wl.Nx * wl.steps / gpu_s if gpu_s > 0 else None,
        "equilibrium_fit": fd_fit, "series": series,
        "final": {"x": x.tolist(), "rho": m[:, :4].T.tolist(), "kT": dg[:, 6].tolist(),
                  "entropy": dg[:, 0].tolist(), "u_x": dg[:, 9].tolist()},
        "wall_seconds": time.perf_counter() - t0,
    }
    plan.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-f64", action="store_true", help="skip the float64 run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--nx", type=int, default=None, help="fewer cells (profiling runs)")
    ap.add_argument("--adj-steps", type=int, default=200,
                    help="steps of the adjoint/forward measurement (0 skips it)")
    ap.add_argument("--adj-every", type=int, default=20, help="checkpoint interval of the adjoint run")
    ap.add_argument("--batch-steps", type=int, default=1,
                    help="steps of the uneven-batch measurement (0 skips it)")
    ap.add_argument("--batch-problems", type=int, default=64, help="problems in the uneven batch")
    ap.add_argument("--batch-replays", type=int, default=1, help="timed replays of the recorded batch graph")
    ap.add_argument("--batch-sub-replays", type=int, default=None,
                    help="replays of the N = 64 sub-batch (default: --batch-replays; 0 skips it)")
    ap.add_argument("--batch-only", action="store_true", help="run only the uneven-batch measurement")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 512 MiB device copy first (scale for HBM byte counters)")
    ap.add_argument("--convergence", action="store_true",
                    help="print the J / M / N convergence study of C_c and C_d instead of the bench line")
    ap.add_argument("--physics", choices=PHYSICS_RUNS, default=None,
                    help="run one of the paper's simulations (Sec. 5.2, 5.3) and print its record")
    ap.add_argument("--t-end", type=float, default=None, help="end time of the --physics run")
    ap.add_argument("--vgrid", type=int, default=32, help="velocity grid N of the --physics run")
    ap.add_argument("--slab-record", type=int, default=0,
                    help="run the float32 slab this many steps and print its conservation record instead")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.convergence:
        print(json.dumps(run_convergence()), flush=True)
        return
    if args.physics:
        print(json.dumps(run_physics(args.physics, t_end=args.t_end, N=args.vgrid)), flush=True)
        return
    if args.slab_record > 0:
        print(json.dumps(run_slab_record(args.slab_record)), flush=True)
        return
    if args.batch_only:
        print(json.dumps(run_batch(args.batch_steps, args.batch_problems, args.batch_replays,
                                   args.batch_sub_replays)), flush=True)
        return

    import workloads

    if args.calibrate_copy:
        copy_calibration()
    ceil = measure_ceilings()
    wl = workloads.config(3, Nx=args.nx)
    log(f"workload {wl.name}: Nx={wl.Nx} N={wl.N} J={wl.J} M={wl.M} dt={wl.dt}")
    t32, k32, a32, b32, cfg32, fin32 = run_gpu(wl, "f32", args.steps, args.warmup)
    out = {
        "metric": METRIC,
        "value": wl.Nx * args.steps / t32,
        "unit": "cells*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dirichlet_maxwell_slab", "Nx": wl.Nx, "N": wl.N, "J": wl.J, "M": wl.M,
                   "L": wl.L, "R": wl.R, "dt": wl.dt, "bc": "dirichlet|maxwell(alpha=0.5)",
                   "moments": "f64"},
    }

    def roof(kern, precision, cfg):
        ms, n = kern["i3"]
        avg_s = ms / max(n, 1) / 1e3
        paired = cfg["paired_nodes"]
        executed = i3_flops(wl.Nx, wl.N, wl.J, wl.M, paired) / avg_s / 1e12
        algorithmic = i3_flops_algorithmic(wl.Nx, wl.N, wl.J, wl.M) / avg_s / 1e12
        traffic = measured_traffic(precision, cfg["tile"]) if wl.Nx == 256 else None
        io = i3_io_bytes(wl.Nx, wl.N, wl.J, 4 if precision == "f32" else 8)
        # counter-measured bytes moved between L2 and the fabric (MALL or HBM)
        # per launch over the launch time, against the 8 TB/s HBM peak
        hbm = None if traffic is None else {"GB/s": traffic / avg_s / 1e9, "peak": 8000.0,
                                            "frac": traffic / avg_s / 8e12,
                                            "frac_of_measured_copy": traffic / avg_s / 1e9 / ceil["copy_GBps"]}
        fma = ceil["fma_f32_TFLOPs" if precision == "f32" else "fma_f64_TFLOPs"]
        return {"kernel": "k_i3", "bound": "alu", "achieved": algorithmic, "peak": PEAK[precision],
                "unit": "TFLOP/s", "frac": algorithmic / PEAK[precision],
                "frac_algorithmic": algorithmic / PEAK[precision], "frac_executed": executed / PEAK[precision],
                "achieved_executed": executed, "traffic": traffic,
                "io_bytes": io, "traffic_ratio": None if traffic is None else traffic / io,
                "hbm_measured": hbm, "measured_fma_peak": fma, "frac_of_measured_fma": executed / fma,
                "avg_launch_ms": ms / max(n, 1), "launches": n, "tile": cfg["tile"],
                "paired_nodes": paired, "persistent": cfg["persistent"],
                "transforms_per_cell_executed": i3_transforms(wl.J, wl.M, paired),
                "transforms_per_cell_algorithmic": 36 * wl.J * wl.M}

    out["ceilings"] = ceil
    out["roofline"] = roof(k32, "f32", cfg32)
    out["launch_shapes_f32"] = cfg32["launch_ab"]
    out["kernel_ms_per_step"] = {k: v[0] / args.steps for k, v in k32.items()}
    drift = lambda a, b: {"density": float((b[0] - a[0]) / a[0]), "energy": float((b[6] - a[6]) / a[6])}

    def budget(a, b, fin):
        # total change minus the inflow through the walls, relative to the
        # initial totals: what the collision and field sub-steps changed
        inf = fin["inflow"]
        return {"density_inflow": float(inf[0] / a[0]), "energy_inflow": float(inf[6] / a[6]),
                "density_residual": float((b[0] - a[0] - inf[0]) / a[0]),
                "energy_residual": float((b[6] - a[6] - inf[6]) / a[6])}

    out["moment_drift_f32"] = drift(a32, b32)
    out["conservation_budget_f32"] = budget(a32, b32, fin32)
    if not args.no_f64:
        t64, k64, a64, b64, cfg64, fin64 = run_gpu(wl, "f64", args.steps, args.warmup)
        out["value_f64"] = wl.Nx * args.steps / t64
        out["ms_per_step_f64"] = 1e3 * t64 / args.steps
        out["roofline_f64"] = roof(k64, "f64", cfg64)
        out["launch_shapes_f64"] = cfg64["launch_ab"]
        out["moment_drift_f64"] = drift(a64, b64)
        out["conservation_budget_f64"] = budget(a64, b64, fin64)
        # the float32 bulk path against float64 on the same input and steps
        # (warmup included): normwise relative difference per result
        nrm = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())
        out["fp32_vs_fp64"] = {
            "steps": args.steps + args.warmup,
            "state": nrm(fin32["W"], fin64["W"]),
            "moments": {name: nrm(fin32["moments"][:, k], fin64["moments"][:, k])
                        for k, name in enumerate(("rho0", "rho1", "rho2", "rho3", "p_x", "p_y", "energy"))},
        }
    out["equilibrium_residual"] = equilibrium_residual(wl)
    out["adjoint_forward_ratio"] = None
    if args.adj_steps > 0:
        adj = run_adjoint(args.adj_steps, args.adj_every)
        out["adjoint_forward_ratio"] = adj["ratio"]
        out["adjoint"] = adj
    if args.batch_steps > 0:
        out["batched"] = run_batch(args.batch_steps, args.batch_problems, args.batch_replays,
                                   args.batch_sub_replays)
        rec = batch_record()
        if rec is not None:
            out["batched_record"] = rec
    rec = slab_record()
    if rec is not None:
        out["slab_record"] = rec
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
