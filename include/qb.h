/*
 * qb.h -- C ABI of the MI355X (gfx950) solver for the spatially inhomogeneous
 * matrix-valued quantum Boltzmann equation of Lu & Mendl, arXiv:1408.1782:
 *
 *     d_t W + v_x d_x W = C[W] - i [B . sigma, W]                 (eq. boltzmann)
 *
 * W(x, v) is a 2x2 Hermitian matrix on x in (0, 1) (Nx finite-volume cells,
 * centres (j + 1/2)/Nx) and v on the N x N grid v_i = (2L/N)(i - N/2),
 * i = 0..N-1 (Sec. 5.1); the first velocity axis is v_x.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is a DEVICE pointer (e.g. from torch) unless
 *   noted; calls are asynchronous on `stream` (a hipStream_t; NULL = default
 *   stream).  The library never allocates or frees device memory: plans and
 *   batches are laid out in a workspace the caller allocates (size from
 *   qb_workspace_bytes / qb_batch_workspace_bytes / qb_adjoint_workspace_bytes)
 *   and keeps alive, unmodified, until the plan or batch is destroyed.
 * State layout.  W and C are [cells][N][N][2][2] complex, row-major, complex
 *   interleaved (re, im): complex128 for QB_F64 plans, complex64 for QB_F32.
 *   Only the Hermitian part of W is read (components w_mu =
 *   (1/2) Re tr(sigma_mu W), Sec. 3.1, eq. spin_repr).
 * Field.  B is float64 [Nx][3] (B_1, B_2, B_3) on every plan.
 * Moments.  float64 [Nx][7] per snapshot: rho_0..rho_3 = h^2 sum_v w_mu
 *   (eq. density in Pauli components), p_x, p_y = h^2 sum_v v tr W
 *   (eq. velocity times tr rho), e = h^2 sum_v |v|^2/2 tr W
 *   (eq. internal_energy plus the kinetic part), h = 2L/N.
 * Errors.  Every call validates its arguments before enqueuing anything;
 *   on error it returns a negative qb_status and enqueues nothing.
 *   QB_EHIP reports a failed HIP call (a launch or a copy); the text of
 *   the last error is available from qb_last_error().
 * Threads.  A plan may be used by one stream at a time; distinct plans are
 *   independent.
 */
#ifndef QB_H
#define QB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QB_OK = 0,
  QB_EINVAL = -1,     /* bad argument (null pointer, size, range)          */
  QB_ENOTSUP = -2,    /* valid but unsupported (N not 16/32/64, odd J)      */
  QB_ECFL = -3,       /* (dt/2) max|v_x| / dx > 1 for the transport step    */
  QB_EWORKSPACE = -4, /* workspace too small, or more cells than the plan holds */
  QB_EHIP = -5        /* HIP runtime error                                  */
} qb_status;

typedef enum { QB_F64 = 0, QB_F32 = 1 } qb_precision;

typedef enum { QB_PERIODIC = 0, QB_DIRICHLET = 1, QB_MAXWELL = 2 } qb_bc_kind;

/* Fermi-Dirac state W_FD(v) = U diag(f_up, f_down) U^H,
 * f_s = 1 / (exp((|v|^2/2 - mu_s) inv_kT) + 1)        (eq. W_FermiDirac).
 * U is row-major, its columns are the spin basis (Table 1). */
typedef struct {
  double inv_kT, mu_up, mu_down;
  double U_re[4], U_im[4];
} qb_fd;

/* Boundary condition on one wall (Sec. 2).
 *   QB_PERIODIC : both walls must be periodic.
 *   QB_DIRICHLET: incoming velocities see Phi = W_FD(state).
 *   QB_MAXWELL  : incoming velocities see (1 - alpha) W_b(-v_x, v_y)
 *                 + alpha W_FD(state) Fbar / Z, W_b the adjacent cell,
 *                 Fbar its outgoing number flux, Z the incoming flux of
 *                 W_FD; 0 <= alpha <= 1.
 * Ghost cells (two per wall): the inflow state at incoming v_x, a copy of
 * the adjacent cell otherwise; the row v_x = -L has no mirror and counts as
 * outgoing at the right wall. */
typedef struct {
  int32_t kind; /* qb_bc_kind */
  qb_fd state;
  double alpha;
} qb_bc;

/* Problem description.
 *   Nx    : number of cells (>= 1).
 *   N     : velocity grid side, 16, 32 or 64.
 *   J     : number of angles theta_j (eq. theta_grid), even, 2..128.
 *   M     : Gauss-Legendre radii of eq. approxH-JM, 1..256.
 *   L, R  : velocity half-box (periodization on [-L, L]^2) and truncation
 *           radius of the collision integrals (Sec. 3.2); L > 0, R >= 0.
 *   precision : QB_F64 (complex128 state, float64 arithmetic) or QB_F32
 *           (complex64 state, float32 collision and transport arithmetic,
 *           float64 moments).
 */
typedef struct {
  int32_t Nx, N, J, M;
  double L, R;
  int32_t precision; /* qb_precision */
  qb_bc left, right;
} qb_problem;

typedef struct qb_plan_s* qb_plan;

/* Device bytes of a plan's workspace for `problem` (0 if the problem is
 * invalid): the quadrature tables of Sec. 3.2 for every compiled tile shape,
 * the wall tables, the collision buffers for `max_cells` cells per
 * collision launch (0: min(Nx, 512); larger Nx runs in chunks) and four
 * state-sized buffers.  Pure host arithmetic; no HIP call. */
size_t qb_workspace_bytes(const qb_problem* problem, int32_t max_cells);

/* Create a plan in the caller's device workspace (at least
 * qb_workspace_bytes(problem, max_cells) bytes, any alignment the HIP
 * allocator returns): validates the problem, builds the quadrature tables of
 * Sec. 3.2 (theta grids, phi_R, psi_R, omega_G, omega_H, Gauss-Legendre
 * nodes, modulation phases) on the host in float64 and copies them in.
 * Allocates no device memory.  Synchronous.  The workspace belongs to the
 * plan until qb_plan_destroy.  *out receives the plan (NULL on error).
 * QB_EWORKSPACE if ws_bytes is too small, QB_EINVAL for a null workspace
 * or a negative max_cells. */
qb_status qb_plan_create(const qb_problem* problem, int32_t max_cells, void* workspace, size_t ws_bytes,
                         qb_plan* out);

/* Free the plan's host state (synchronizes the device first); the caller
 * may then release the workspace. */
qb_status qb_plan_destroy(qb_plan plan);

/* Workspace bytes in use by a plan (its adjoint workspace included once
 * enabled), and the number of cells one collision launch covers. */
size_t qb_plan_bytes(qb_plan plan);
int32_t qb_plan_chunk_cells(qb_plan plan);

/* C = C[W] = C_c[W] + C_d[W] for `ncells` independent cells (Sec. 3.2):
 * the conservative part through the principal-value kernel G (eq. approxG)
 * and the dissipative part through H (eq. approxH-J, eq. approxH-JM), in
 * the Carleman form of eq. CcPauli / eq. CdPauli; Fourier coefficients on
 * Xi (eq. fourier_grid) with the -N/2 rows and columns set to zero on input
 * and output, products on the 2N zero-padded grid.
 * W, C: [ncells][N][N][2][2] complex, distinct buffers; 1 <= ncells <= Nx. */
qb_status qb_collision(qb_plan plan, const void* W, void* C, int32_t ncells, void* stream);

/* qb_collision for callers that cannot allocate device memory at all (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same operator and kernels, with every per-cell buffer of
 * the collision pipeline taken from a fixed array of
 * qb_collision_static_bytes() bytes (64 MiB) that the library holds on each
 * GPU it runs on until the process ends; only the plan's tables are read
 * from its workspace.  Cells run in chunks of as many as fit.  Allocates
 * nothing and clears nothing: every scratch value is written before it is
 * read, so the array may hold anything from an earlier call.  All calls on
 * one GPU share its array: calls that overlap in time on one GPU (two
 * streams, two host threads) race and must be serialized by the caller.
 * QB_EWORKSPACE if ncells > Nx or if one cell's buffers exceed the array
 * (qb_last_error says so); other arguments and errors as qb_collision. */
qb_status qb_collision_static(qb_plan plan, const void* W, void* C, int32_t ncells, void* stream);
size_t qb_collision_static_bytes(void);

/* One finite-volume transport step of length dt in place (eq.
 * slopeLimiterStep with the minmod limiter of eq. minmod, applied to the
 * four Pauli components), with the plan's boundary conditions.
 * W: [Nx][N][N][2][2] complex.  QB_ECFL if dt max|v_x| Nx > 1. */
qb_status qb_transport_step(qb_plan plan, void* W, double dt, void* stream);

/* nsteps time steps of the splitting scheme of Sec. 4 in place: transport
 * over dt/2, one Heun (two-stage Runge-Kutta) step of length dt for
 * dW/dt = C[W] - i[B . sigma, W] per cell, transport over dt/2.
 * W: [Nx][N][N][2][2] complex; B: float64 [Nx][3] device array or NULL
 * (no field); moments: float64 [nsteps + 1][Nx][7] device array or NULL
 * (snapshot 0 is the initial state). */
qb_status qb_step(qb_plan plan, void* W, const double* B, double dt, int32_t nsteps, double* moments,
                  void* stream);

/* qb_step that also returns the moments of the net inflow through the two
 * walls during every step (both transport half-steps), float64 device
 * array inflow[nsteps][7] in the units of the per-cell moments summed over
 * the cells: with the scheme written in flux form, W_j <- W_j - (dt/dx)
 * (F_{j+1/2} - F_{j-1/2}) (eq. slopeLimiterStep), the transport changes the
 * cell-summed moments by exactly (dt/dx) h^2 sum_v phi(v) (F_{1/2} -
 * F_{Nx+1/2}), so total moments minus accumulated inflow isolate what the
 * collision and field sub-steps change (the conservation budget of Sec. 2
 * on a bounded slab; zero inflow for periodic walls).  Other arguments and
 * errors as qb_step (QB_EINVAL also for a null inflow). */
qb_status qb_step_fluxes(qb_plan plan, void* W, const double* B, double dt, int32_t nsteps, double* moments,
                         double* inflow, void* stream);

/* float64 moments [Nx][7] of W ([Nx][N][N][2][2] complex). */
qb_status qb_moments(qb_plan plan, const void* W, double* moments, void* stream);

/* ---------------------------------------------------------------------------
 * Scheme variants (Sec. 4: other slope limiters may replace minmod; the
 * field term may be applied apart from the collision).
 *   limiter: the slope S_j of eq. slopeLimiterStep from the one-sided
 *     differences a = W_{j+1} - W_j, b = W_j - W_{j-1}, per Pauli component:
 *     QB_LIMITER_MINMOD (eq. minmod, the default), QB_LIMITER_SUPERBEE (the
 *     larger in magnitude of minmod(a, 2b) and minmod(2a, b)), QB_LIMITER_MC
 *     (monotonized central, minmod((a + b)/2, minmod(2a, 2b))),
 *     QB_LIMITER_VAN_LEER ((a|b| + |a|b) / (|a| + |b|), 0 when both vanish).
 *   field: QB_FIELD_HEUN (the default: F = C + 2 (B x w).sigma inside the
 *     Heun step) or QB_FIELD_ROTATION (the exact flow of the field term, a
 *     rotation of the Bloch vector about B(x) by the angle 2|B| t, for dt/2
 *     before and after a Heun step of C alone).
 * Used by qb_transport_step and qb_step; the reverse mode (qb_transport_vjp, qb_step_trace, qb_adjoint_step) returns
 * QB_ENOTSUP unless both are the defaults.  QB_EINVAL for other values.
 * ------------------------------------------------------------------------- */
#define QB_LIMITER_MINMOD 0
#define QB_LIMITER_SUPERBEE 1
#define QB_LIMITER_MC 2
#define QB_LIMITER_VAN_LEER 3
#define QB_FIELD_HEUN 0
#define QB_FIELD_ROTATION 1
qb_status qb_plan_set_scheme(qb_plan plan, int32_t limiter, int32_t field);

/* ---------------------------------------------------------------------------
 * Term selection (Sec. 3.2 and the validation of Sec. 5.1, which measures
 * the conservative and the dissipative part separately): qb_collision and
 * qb_step assemble C = w_c C_c + w_d C_d with (w_c, w_d) = (1, 0) for
 * QB_TERMS_CONSERVATIVE, (0, 1) for QB_TERMS_DISSIPATIVE and (1, 1) for
 * QB_TERMS_ALL (the default).  The reverse mode (qb_collision_vjp,
 * qb_adjoint_step) returns QB_ENOTSUP unless the plan uses QB_TERMS_ALL.
 * QB_EINVAL for other values.
 * ------------------------------------------------------------------------- */
#define QB_TERMS_CONSERVATIVE 1
#define QB_TERMS_DISSIPATIVE 2
#define QB_TERMS_ALL 3
qb_status qb_plan_set_terms(qb_plan plan, int32_t terms);

/* ---------------------------------------------------------------------------
 * Ceiling probes (measurement instrumentation, not part of the solver):
 * the rates this GPU sustains, for reading the kernels' roofline fractions
 * against measured ceilings beside the datasheet figures.  Both calls block
 * until their launches on `stream` finish (one warm-up launch, then timed
 * repetitions between two HIP events).
 *   qb_probe_fma: vector fused multiply-add throughput in TFLOP/s of the
 *     plan precisions (QB_F32: float, unpacked, as the library is compiled;
 *     QB_F64: double): 4096 x 256 threads, 8 independent chains of 8 x iters
 *     FMAs each.  scratch: device buffer of at least 32768 bytes (written
 *     only if a result takes a value it never takes).
 *   qb_probe_copy: device-to-device copy bandwidth in GB/s (bytes read plus
 *     bytes written per second) of `reps` 16-byte-vector copies of `bytes`
 *     (a multiple of 16) from src to dst (device buffers, not overlapping).
 * QB_EINVAL for null pointers or sizes out of range, QB_EHIP on a failed
 * HIP call.
 * ------------------------------------------------------------------------- */
qb_status qb_probe_fma(int32_t precision, int32_t iters, void* scratch, double* tflops, void* stream);
qb_status qb_probe_copy(const void* src, void* dst, size_t bytes, int32_t reps, double* gbps, void* stream);

/* ---------------------------------------------------------------------------
 * Diagnostics of a state (Sec. 2 and Sec. 5), float64 whatever the plan's
 * precision, one row of QB_DIAG_FIELDS values per cell:
 *   0  local entropy S = -h^2 sum_v tr[W log W + W~ log W~], W~ = 1 - W
 *      (eq. entropy_def);
 *   1  entropy production density -h^2 sum_v tr[(log W - log W~) C] (the
 *      integrand of the H-theorem; its sum times dx is d/dt of the total
 *      entropy under dW/dt = C); 0 when C is NULL;
 *   2  relative entropy h^2 sum_v tr[W (log W - log F) + W~ (log W~ - log F~)]
 *      to the Fermi-Dirac state F = W_FD(global) at rest (eq. relentropy_hom;
 *      times dx summed over cells: eq. relentropy_inhom); 0 when global is NULL;
 *   3  the same relative entropy to the local fit W_FD,loc (eq. relentropy_local);
 *   4, 5  smallest and largest eigenvalue of W(v) over the cell (unclamped);
 *   6..10 the local fit: kT, mu_up, mu_down, u_x, u_y.  u = momentum /
 *      density (eq. velocity); the per-spin densities are the eigenvalues
 *      r_up >= r_down of the spin density h^2 sum_v W, the spin basis its
 *      eigenbasis; kT and mu_s solve r_s = 2 pi kT log(1 + e^{mu_s/kT}) and
 *      eps = e/n - |u|^2/2 = eps_FD (eq. momentsFermiDirac).
 * Eigenvalues are clamped into [0, 1] inside the logarithms and log x reads
 * log(max(x, 1e-300)).  The fit fields and field 3 are NaN where no
 * Fermi-Dirac state matches: r_down <= 0, or kT below r_up / (1200 pi).
 * W, C: [Nx][N][N][2][2] complex of the plan's precision (C may be NULL,
 * e.g. C = qb_collision(W)); global: host struct or NULL (its U need only
 * have a nonzero first column, the spin-up direction); out: float64
 * [Nx][QB_DIAG_FIELDS] device array.  QB_EINVAL for null W / out, or a
 * global state with inv_kT <= 0, non-finite values or a zero first column.
 * ------------------------------------------------------------------------- */
#define QB_DIAG_FIELDS 11
qb_status qb_diagnostics(qb_plan plan, const void* W, const void* C, const qb_fd* global, double* out,
                         void* stream);

/* ---------------------------------------------------------------------------
 * FFT tile shapes.  Every padded-grid transform runs in one workgroup that
 * holds the P x P field in registers, E elements per thread and P / E
 * threads per line.  Compiled shapes: P = 32: E = 16 (default), 8;
 * P = 64: E = 16 (default), 32, 8; P = 128: E = 16 (default), 32.
 * ------------------------------------------------------------------------- */

/* Use tile shape E on this plan (QB_ENOTSUP if not compiled for its P).
 * Synchronous the first time a shape is used (builds its tables). */
qb_status qb_plan_set_tile(qb_plan plan, int32_t E);

/* Autotuner: time the collision pipeline on the plan's first `ncells` cells
 * for every compiled tile shape, with and without Gauss-Legendre node
 * pairing in the I_3 kernel, and keep the fastest; then the two launch
 * shapes (qb_plan_set_persistent) on that tile, the persistent one kept
 * only when it is more than 1 % faster; when the plan's
 * adjoint is enabled, also time the reverse-mode pipeline for every tile
 * shape and both I_3 adjoint kernels (row w cotangents in memory or in
 * registers, see qb_plan_config) and keep the fastest.  Synchronous; overwrites the
 * plan's internal buffers.  Choices are cached per (precision, N, J, M,
 * ncells) for the life of the process.  *tile (may be NULL) receives E. */
qb_status qb_plan_tune(qb_plan plan, int32_t ncells, int32_t* tile, void* stream);

/* I_3 kernel with (1, the default on every tile) or without (0)
 * Gauss-Legendre node pairing; both compute the same operator (the pairing
 * uses rho_{M-1-m} = -rho_m). */
qb_status qb_plan_set_pairing(qb_plan plan, int32_t paired);

/* Tile shape E of the reverse-mode pipeline (qb_collision_vjp and the
 * collision adjoints of qb_adjoint_step), independent of the forward tile;
 * 0 follows the forward tile (the default).  QB_ENOTSUP if E is not
 * compiled for the plan's padded grid.  Synchronous the first time a shape
 * is used (fills its tables). */
qb_status qb_plan_set_adjoint_tile(qb_plan plan, int32_t E);

/* Use I_3 adjoint kernel `variant` (0 or 1, see qb_plan_config). */
qb_status qb_plan_set_adjoint_variant(qb_plan plan, int32_t variant);

/* Launch shape of the two heavy collision kernels (I_1 / I_2 / I_4 and
 * I_3): 0 (the default) launches one workgroup per task, (cell, term) or
 * (cell, j); 1 launches a persistent grid of as many workgroups as are
 * resident at once on the device (a multiple of 8), each striding over the
 * task list.  Both compute the same values bit for bit; qb_plan_tune picks
 * the faster.  For a batch the task list spans every problem of a grid size. */
qb_status qb_plan_set_persistent(qb_plan plan, int32_t persistent);

/* Current tile shape E, I_3 adjoint kernel (0: the shifted-field cotangent
 * of the current rows in registers, 1: also their w cotangent), whether
 * the I_3 kernel of this tile pairs the Gauss-Legendre nodes m and M-1-m
 * (1) or runs every node on its own (0), the reverse-mode tile shape and
 * the launch shape (qb_plan_set_persistent); any pointer may be NULL. */
qb_status qb_plan_config(qb_plan plan, int32_t* tile, int32_t* adjoint_variant, int32_t* paired_nodes,
                         int32_t* adjoint_tile, int32_t* persistent);

/* ---------------------------------------------------------------------------
 * Batches of independent problems (uneven Nx and N) advanced together:
 * problems with the same N share one concatenated cell array, so each
 * collision kernel is one launch over all their cells; transport runs per
 * problem with its own walls.
 * ------------------------------------------------------------------------- */
typedef struct qb_batch_s* qb_batch;

/* Device bytes of the workspace of a batch of nprob problems (each valid for
 * qb_plan_create; all with the same precision, J, L and R; problems with
 * equal N must have equal M); 0 for an invalid batch. */
size_t qb_batch_workspace_bytes(const qb_problem* problems, int32_t nprob);

/* Create a batch in the caller's device workspace (at least
 * qb_batch_workspace_bytes bytes; kept alive until qb_batch_destroy).
 * Allocates no device memory; creates one non-blocking HIP stream on which
 * QB_BATCH_GRAPH records its graphs.  Synchronous.  QB_EWORKSPACE if the
 * workspace is too small. */
qb_status qb_batch_create(const qb_problem* problems, int32_t nprob, void* workspace, size_t ws_bytes,
                          qb_batch* out);
qb_status qb_batch_destroy(qb_batch batch);
size_t qb_batch_bytes(qb_batch batch);

/* Launch shape of the collision kernels of every N group (as
 * qb_plan_set_persistent: each group's kernels stride over the tasks of all
 * its problems' cells from one resident-sized grid); drops a recorded graph. */
qb_status qb_batch_set_persistent(qb_batch batch, int32_t persistent);

/* Run the autotuner (qb_plan_tune) for every N group of the batch. */
qb_status qb_batch_tune(qb_batch batch, void* stream);

#define QB_BATCH_GRAPH 1 /* record the whole call as a HIP graph and replay it */

/* nsteps splitting steps (as qb_step) of every problem, in place.
 *   W       : host array of nprob device pointers, W[m] [Nx_m][N_m][N_m][2][2] complex.
 *   B       : host array of nprob device pointers (float64 [Nx_m][3], or NULL
 *             entries for no field), or NULL.
 *   moments : host array of nprob device pointers (float64
 *             [nsteps + 1][Nx_m][7], or NULL entries), or NULL.
 *   flags   : QB_BATCH_GRAPH records the launch sequence of the call in a HIP
 *             graph on first use and replays it while W, B, moments, dt and
 *             nsteps are unchanged (no HIP graph memset nodes are used).
 * QB_ECFL if (dt/2) L Nx_m > 1 for any problem.  Moments are written
 * straight into each problem's array (no scratch). */
qb_status qb_batch_step(qb_batch batch, void* const* W, const double* const* B, double dt, int32_t nsteps,
                        double* const* moments, int32_t flags, void* stream);

/* ---------------------------------------------------------------------------
 * Reverse mode (adjoint).  Gradients of a real scalar l follow torch's
 * convention for complex arrays: the cotangent G of a state W satisfies
 * dl = Re sum conj(G) dW, i.e. G = dl/dRe W + i dl/dIm W.  Since every map
 * here reads only the Hermitian part of W, the returned G is Hermitian,
 * G = (1/2) sum_mu g_mu sigma_mu with g_mu = dl/dw_mu (Sec. 3.1).  The
 * limiter of eq. minmod is differentiated on the branch it takes at the
 * forward state.
 * ------------------------------------------------------------------------- */

/* Device bytes of the reverse-mode workspace of a plan (cotangent buffers
 * of the collision pipeline and of the states). */
size_t qb_adjoint_workspace_bytes(qb_plan plan);

/* Lay out the reverse-mode buffers in a caller workspace of at least
 * qb_adjoint_workspace_bytes(plan) bytes (kept alive until the plan is
 * destroyed); allocates nothing.  Idempotent: once enabled, later calls
 * return QB_OK and keep the first workspace.  Every call below returns
 * QB_EWORKSPACE until this has succeeded. */
qb_status qb_plan_enable_adjoint(qb_plan plan, void* workspace, size_t ws_bytes);

/* G = C'(W)^T lam for `ncells` cells: the transpose of the linearization of
 * qb_collision at W applied to the cotangent lam of C (Sec. 3.2; C is a
 * polynomial of degree three in the Pauli components of W).
 * W, lam, G: [ncells][N][N][2][2] complex; G distinct from W and lam. */
qb_status qb_collision_vjp(qb_plan plan, const void* W, const void* lam, void* G, int32_t ncells,
                           void* stream);

/* G = T'(W)^T lam for one qb_transport_step of length dt taken at W
 * (eq. slopeLimiterStep, Sec. 2 walls).  W, lam, G: [Nx][N][N][2][2] complex. */
qb_status qb_transport_vjp(qb_plan plan, const void* W, double dt, const void* lam, void* G, void* stream);

/* Bytes of one step record written by qb_step_trace. */
size_t qb_trace_bytes(qb_plan plan);

/* As qb_step (no moments), and for each step n writes a record of
 * qb_trace_bytes(plan) bytes at trace + n * qb_trace_bytes(plan): the step's
 * input state, the Heun stage and the Heun output (internal layout; only
 * qb_adjoint_step reads it).  trace: device buffer of nsteps records. */
qb_status qb_step_trace(qb_plan plan, void* W, const double* B, double dt, int32_t nsteps, void* trace,
                        void* stream);

/* Reverse of one qb_step of length dt (Sec. 4 splitting with the Heun
 * stages):  lam = (dS/dW)^T lam_next and gB += (dS/dB)^T lam_next, S the
 * step taken from the state W with field B.
 *   W        : step input [Nx][N][N][2][2] complex; read only when record is NULL.
 *   record   : NULL (the step's forward stages are recomputed: two collision
 *              evaluations) or this step's record from qb_step_trace.
 *   B        : float64 [Nx][3] or NULL (no field).
 *   lam_next : cotangent of the step output; lam: cotangent of its input
 *              (may alias lam_next).
 *   gB       : float64 [Nx][3], accumulated (+=), or NULL. */
qb_status qb_adjoint_step(qb_plan plan, const void* W, const void* record, const double* B, double dt,
                          const void* lam_next, void* lam, double* gB, void* stream);

/* Kernel timing.  With profiling on, every kernel the plan launches is
 * bracketed by a pair of HIP events on its stream; qb_profile_read
 * synchronizes those events and returns, for one kernel class, the summed
 * duration in milliseconds and the number of launches since the last read
 * (then resets that class).  Profiling adds two event records per launch. */
typedef enum {
  QB_K_DFT_IN = 0,  /* velocity grid -> Fourier coefficients, padded-grid interpolants */
  QB_K_TERMS = 1,   /* I_1 (kernel G), I_4 and I_2 (kernel H_J) */
  QB_K_I3 = 2,      /* I_3 (kernel H_JM), the dominant kernel */
  QB_K_COMBINE = 3, /* Pauli assembly, final transform, output on the grid */
  QB_K_TRANSPORT = 4,
  QB_K_HEUN = 5,
  QB_K_MOMENTS = 6,
  QB_K_I3_ADJOINT = 7, /* transpose of the I_3 kernel */
  QB_K_ADJOINT = 8,    /* the other reverse-mode kernels */
  QB_K_DIAGNOSTICS = 9,
  QB_K_COUNT = 10
} qb_kernel;
qb_status qb_profile(qb_plan plan, int32_t enable);
qb_status qb_profile_read(qb_plan plan, int32_t kernel, double* total_ms, int64_t* launches);

/* Human-readable name of a status; text of the last HIP error seen. */
const char* qb_strerror(qb_status status);
const char* qb_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int32_t qb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QB_H */
