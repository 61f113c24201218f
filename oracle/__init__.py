"""Oracle for the matrix-valued quantum Boltzmann scheme of Lu & Mendl
(arXiv:1408.1782): a plain, slow, complex128 CPU implementation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library (no kernels, tables, helpers or constants); both sides get
their inputs from the seeded generators in ``workloads/``.

What it computes, and where the paper defines it:

* ``pauli``      -- Pauli representation w = (w0, w1, w2, w3) and the metric
                    eta (Sec. 3.1, eq. spin_repr).
* ``quadrature`` -- angle grids theta_j / theta'_j (eq. theta_grid), the
                    radial functions phi_R and psi_R, the weights omega_G
                    (eq. approxG), omega_H (eq. approxH-J) and the
                    Gauss-Legendre nodes of eq. approxH-JM (Sec. 3.2).
* ``spectral``   -- the Fourier grid Xi (eq. fourier_grid), the mean-value
                    coefficients, and zero padding to the 2N grid
                    ("double zero padding", Sec. 3.2), all by naive DFT
                    matrices.
* ``collision``  -- the collision operator C[W] = C_c + C_d in Carleman form
                    (eq. CcPauliCarleman and the Carleman form of
                    eq. CdPauli), through the integral types I_1..I_4 with
                    the kernel approximations eq. approxG, approxH-J and
                    approxH-JM, in the order the paper states them.
* ``transport``  -- the minmod finite-volume step (eq. slopeLimiterStep,
                    eq. minmod) with periodic, Dirichlet and Maxwell inflow
                    (Sec. 2, boundary conditions).
* ``fermi_dirac``-- W_FD (eq. W_FermiDirac) and its closed-form moments
                    (eq. momentsFermiDirac).
* ``step``       -- the time-splitting step of Sec. 4 (half transport,
                    collision + magnetic field, half transport) and the
                    fluid moments (eq. density, velocity, internal_energy).
* ``diagnostics``-- local entropy (eq. entropy_def), the entropy
                    production density of the H-theorem, the quantum
                    relative entropy (eq. relentropy_hom), the eigenvalue
                    range and the local Fermi-Dirac fit of Sec. 5.
* ``adjoint``    -- reverse-mode derivatives of the above (the transpose of
                    each forward step, run backwards): C'(w)^T lam, the
                    transport and splitting steps, and the gradient of a
                    final-time observable in the initial state and B(x).

Readings of passages where the paper is silent or garbled are marked
"Reading:" where they are applied.
"""
