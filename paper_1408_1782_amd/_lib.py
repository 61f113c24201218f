"""ctypes binding of libqb.so (include/qb.h): argument marshalling only.

Every numerical step runs in the HIP library.  Tensors passed in must be
contiguous CUDA (HIP) tensors of the dtype the plan expects; every device
buffer goes through one check (``_dev``: device, contiguity, dtype, shape)
before any library call, the binding passes raw device pointers and the
current torch stream, and raises QBError on any non-zero status.  The
library allocates no device memory: the workspaces of plans and batches are
torch tensors this module allocates and keeps alive beside the handles.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_NAME = "libqb.so"

QB_OK, QB_EINVAL, QB_ENOTSUP, QB_ECFL, QB_EWORKSPACE, QB_EHIP = 0, -1, -2, -3, -4, -5
QB_F64, QB_F32 = 0, 1
QB_PERIODIC, QB_DIRICHLET, QB_MAXWELL = 0, 1, 2
_KINDS = {"periodic": QB_PERIODIC, "dirichlet": QB_DIRICHLET, "maxwell": QB_MAXWELL}
KERNELS = {"dft_in": 0, "terms": 1, "i3": 2, "combine": 3, "transport": 4, "heun": 5, "moments": 6,
           "i3_adjoint": 7, "adjoint": 8, "diagnostics": 9}
QB_DIAG_FIELDS = 11
DIAG_NAMES = ("entropy", "entropy_production", "rel_entropy_global", "rel_entropy_local", "eig_min",
              "eig_max", "kT", "mu_up", "mu_down", "u_x", "u_y")

# names the header declares (checked by the CPU tests)
EXPORTS = (
    "qb_workspace_bytes",
    "qb_plan_create",
    "qb_plan_chunk_cells",
    "qb_adjoint_workspace_bytes",
    "qb_batch_workspace_bytes",
    "qb_plan_destroy",
    "qb_plan_bytes",
    "qb_collision",
    "qb_collision_static",
    "qb_collision_static_bytes",
    "qb_transport_step",
    "qb_step",
    "qb_step_fluxes",
    "qb_moments",
    "qb_diagnostics",
    "qb_probe_fma",
    "qb_probe_copy",
    "qb_plan_enable_adjoint",
    "qb_collision_vjp",
    "qb_transport_vjp",
    "qb_trace_bytes",
    "qb_step_trace",
    "qb_adjoint_step",
    "qb_plan_set_tile",
    "qb_plan_tune",
    "qb_plan_config",
    "qb_plan_set_adjoint_variant",
    "qb_plan_set_adjoint_tile",
    "qb_plan_set_persistent",
    "qb_plan_set_pairing",
    "qb_plan_set_terms",
    "qb_plan_set_scheme",
    "qb_batch_create",
    "qb_batch_destroy",
    "qb_batch_bytes",
    "qb_batch_tune",
    "qb_batch_set_persistent",
    "qb_batch_step",
    "qb_profile",
    "qb_profile_read",
    "qb_strerror",
    "qb_last_error",
    "qb_version",
)


class QBError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        msg = _strerror(status)
        if status == QB_EHIP and _LIB is not None:
            msg += ": " + _LIB.qb_last_error().decode()
        super().__init__(f"{what}: {msg} (status {status})")


class _FD(ctypes.Structure):
    _fields_ = [
        ("inv_kT", ctypes.c_double),
        ("mu_up", ctypes.c_double),
        ("mu_down", ctypes.c_double),
        ("U_re", ctypes.c_double * 4),
        ("U_im", ctypes.c_double * 4),
    ]


class _BC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("state", _FD), ("alpha", ctypes.c_double)]


class _Problem(ctypes.Structure):
    _fields_ = [
        ("Nx", ctypes.c_int32),
        ("N", ctypes.c_int32),
        ("J", ctypes.c_int32),
        ("M", ctypes.c_int32),
        ("L", ctypes.c_double),
        ("R", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("left", _BC),
        ("right", _BC),
    ]


_LIB = None


def lib_path():
    return os.path.join(HERE, LIB_NAME)


def _declare(lib):
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    sz = ctypes.c_size_t
    lib.qb_workspace_bytes.argtypes = [ctypes.POINTER(_Problem), i32]
    lib.qb_workspace_bytes.restype = sz
    lib.qb_plan_create.argtypes = [ctypes.POINTER(_Problem), i32, vp, sz, ctypes.POINTER(vp)]
    lib.qb_plan_create.restype = i32
    lib.qb_plan_chunk_cells.argtypes = [vp]
    lib.qb_plan_chunk_cells.restype = i32
    lib.qb_adjoint_workspace_bytes.argtypes = [vp]
    lib.qb_adjoint_workspace_bytes.restype = sz
    lib.qb_batch_workspace_bytes.argtypes = [ctypes.POINTER(_Problem), i32]
    lib.qb_batch_workspace_bytes.restype = sz
    lib.qb_plan_destroy.argtypes = [vp]
    lib.qb_plan_destroy.restype = i32
    lib.qb_plan_bytes.argtypes = [vp]
    lib.qb_plan_bytes.restype = ctypes.c_size_t
    lib.qb_collision.argtypes = [vp, vp, vp, i32, vp]
    lib.qb_collision.restype = i32
    lib.qb_collision_static.argtypes = [vp, vp, vp, i32, vp]
    lib.qb_collision_static.restype = i32
    lib.qb_collision_static_bytes.argtypes = []
    lib.qb_collision_static_bytes.restype = ctypes.c_size_t
    lib.qb_transport_step.argtypes = [vp, vp, dbl, vp]
    lib.qb_transport_step.restype = i32
    lib.qb_step.argtypes = [vp, vp, vp, dbl, i32, vp, vp]
    lib.qb_step_fluxes.argtypes = [vp, vp, vp, dbl, i32, vp, vp, vp]
    lib.qb_step_fluxes.restype = i32
    lib.qb_step.restype = i32
    lib.qb_moments.argtypes = [vp, vp, vp, vp]
    lib.qb_moments.restype = i32
    lib.qb_diagnostics.argtypes = [vp, vp, vp, ctypes.POINTER(_FD), vp, vp]
    lib.qb_diagnostics.restype = i32
    lib.qb_probe_fma.argtypes = [i32, i32, vp, ctypes.POINTER(dbl), vp]
    lib.qb_probe_fma.restype = i32
    lib.qb_probe_copy.argtypes = [vp, vp, ctypes.c_size_t, i32, ctypes.POINTER(dbl), vp]
    lib.qb_probe_copy.restype = i32
    lib.qb_plan_enable_adjoint.argtypes = [vp, vp, ctypes.c_size_t]
    lib.qb_plan_enable_adjoint.restype = i32
    lib.qb_collision_vjp.argtypes = [vp, vp, vp, vp, i32, vp]
    lib.qb_collision_vjp.restype = i32
    lib.qb_transport_vjp.argtypes = [vp, vp, dbl, vp, vp, vp]
    lib.qb_transport_vjp.restype = i32
    lib.qb_trace_bytes.argtypes = [vp]
    lib.qb_trace_bytes.restype = ctypes.c_size_t
    lib.qb_step_trace.argtypes = [vp, vp, vp, dbl, i32, vp, vp]
    lib.qb_step_trace.restype = i32
    lib.qb_adjoint_step.argtypes = [vp, vp, vp, vp, dbl, vp, vp, vp, vp]
    lib.qb_adjoint_step.restype = i32
    lib.qb_plan_set_tile.argtypes = [vp, i32]
    lib.qb_plan_set_tile.restype = i32
    lib.qb_plan_tune.argtypes = [vp, i32, ctypes.POINTER(i32), vp]
    lib.qb_plan_tune.restype = i32
    lib.qb_plan_config.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                   ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.qb_plan_set_persistent.argtypes = [vp, i32]
    lib.qb_plan_set_persistent.restype = i32
    lib.qb_plan_set_adjoint_tile.argtypes = [vp, i32]
    lib.qb_plan_set_adjoint_tile.restype = i32
    lib.qb_plan_config.restype = i32
    lib.qb_plan_set_adjoint_variant.argtypes = [vp, i32]
    lib.qb_plan_set_adjoint_variant.restype = i32
    lib.qb_plan_set_pairing.argtypes = [vp, i32]
    lib.qb_plan_set_terms.argtypes = [vp, i32]
    lib.qb_plan_set_terms.restype = i32
    lib.qb_plan_set_scheme.argtypes = [vp, i32, i32]
    lib.qb_plan_set_scheme.restype = i32
    lib.qb_plan_set_pairing.restype = i32
    lib.qb_batch_create.argtypes = [ctypes.POINTER(_Problem), i32, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    lib.qb_batch_create.restype = i32
    lib.qb_batch_destroy.argtypes = [vp]
    lib.qb_batch_destroy.restype = i32
    lib.qb_batch_bytes.argtypes = [vp]
    lib.qb_batch_bytes.restype = ctypes.c_size_t
    lib.qb_batch_set_persistent.argtypes = [vp, i32]
    lib.qb_batch_set_persistent.restype = i32
    lib.qb_batch_tune.argtypes = [vp, vp]
    lib.qb_batch_tune.restype = i32
    lib.qb_batch_step.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), dbl, i32, ctypes.POINTER(vp), i32, vp]
    lib.qb_batch_step.restype = i32
    lib.qb_profile.argtypes = [vp, i32]
    lib.qb_profile.restype = i32
    lib.qb_profile_read.argtypes = [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_int64)]
    lib.qb_profile_read.restype = i32
    lib.qb_strerror.argtypes = [i32]
    lib.qb_strerror.restype = ctypes.c_char_p
    lib.qb_last_error.argtypes = []
    lib.qb_last_error.restype = ctypes.c_char_p
    lib.qb_version.argtypes = []
    lib.qb_version.restype = i32


def load():
    """Load libqb.so (built in-tree by build.py); raises if it is missing."""
    global _LIB
    if _LIB is None:
        path = lib_path()
        if not os.path.exists(path):
            raise FileNotFoundError(
                f"{path} is not built; run `python -m paper_1408_1782_amd.build` "
                "(or __graft_entry__.build())"
            )
        lib = ctypes.CDLL(path)
        _declare(lib)
        _LIB = lib
    return _LIB


def _strerror(status):
    if _LIB is None:
        return f"status {status}"
    return _LIB.qb_strerror(status).decode()


def _check(status, what):
    if status != QB_OK:
        raise QBError(status, what)


class BC:
    """Boundary condition on one wall: kind in {'periodic', 'dirichlet',
    'maxwell'}, Fermi-Dirac wall state (inv_kT, mu_up, mu_down, U) and the
    Maxwell accommodation coefficient alpha."""

    def __init__(self, kind="periodic", inv_kT=1.0, mu_up=0.0, mu_down=0.0, U=None, alpha=0.0):
        self.kind, self.inv_kT, self.mu_up, self.mu_down = kind, inv_kT, mu_up, mu_down
        self.U = U
        self.alpha = alpha

    @classmethod
    def from_workload(cls, b):
        return cls(b.kind, b.inv_kT, b.mu_up, b.mu_down, b.U, b.alpha)

    def _c(self):
        c = _BC()
        c.kind = _KINDS[self.kind]
        c.alpha = float(self.alpha)
        c.state.inv_kT = float(self.inv_kT)
        c.state.mu_up = float(self.mu_up)
        c.state.mu_down = float(self.mu_down)
        U = [[1, 0], [0, 1]] if self.U is None else self.U
        for a in range(2):
            for b in range(2):
                z = complex(U[a][b])
                c.state.U_re[2 * a + b] = z.real
                c.state.U_im[2 * a + b] = z.imag
        return c


class Problem:
    def __init__(self, Nx, N, J=32, M=None, L=12.0, R=7.5, precision="f64", left=None, right=None):
        self.Nx, self.N, self.J = int(Nx), int(N), int(J)
        self.M = int(N if M is None else M)
        self.L, self.R = float(L), float(R)
        self.precision = precision
        self.left = left or BC("periodic")
        self.right = right or BC("periodic")

    def _c(self):
        p = _Problem()
        p.Nx, p.N, p.J, p.M = self.Nx, self.N, self.J, self.M
        p.L, p.R = self.L, self.R
        p.precision = QB_F64 if self.precision == "f64" else QB_F32
        p.left, p.right = self.left._c(), self.right._c()
        return p


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dev(t, dtype, shape, name):
    """Check one device buffer before its pointer reaches the library: a
    contiguous CUDA tensor of `dtype` and exactly `shape` (None entries match
    any size).  A host tensor would hand a host pointer to a kernel; a
    non-contiguous view would be read or written in the wrong order."""
    if not hasattr(t, "is_cuda") or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if len(t.shape) != len(shape) or any(e is not None and int(a) != e for a, e in zip(t.shape, shape)):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return _ptr(t)


def _workspace(nbytes):
    """A device workspace of `nbytes` bytes (torch memory, 256-byte aligned)."""
    import torch

    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


class Plan:
    """A qb_plan: quadrature tables and device buffers for one problem."""

    def __init__(self, problem, max_cells=0, adjoint=False):
        """max_cells: cells per collision launch (0: min(Nx, 512)); adjoint:
        lay out the reverse-mode workspace too (else enable_adjoint())."""
        import torch

        self.lib = load()
        self.problem = problem
        self.cdtype = torch.complex128 if problem.precision == "f64" else torch.complex64
        pc = problem._c()
        nbytes = self.lib.qb_workspace_bytes(ctypes.byref(pc), int(max_cells))
        if nbytes == 0:
            _check(QB_EINVAL, "qb_workspace_bytes")
        self.ws = _workspace(nbytes)
        self.ws_adj = None
        h = ctypes.c_void_p()
        _check(self.lib.qb_plan_create(ctypes.byref(pc), int(max_cells), _ptr(self.ws), self.ws.numel(),
                                       ctypes.byref(h)), "qb_plan_create")
        self.handle = h
        if adjoint:
            self.enable_adjoint()

    @property
    def nbytes(self):
        return self.lib.qb_plan_bytes(self.handle)

    @property
    def chunk_cells(self):
        return self.lib.qb_plan_chunk_cells(self.handle)

    def _check_state(self, W, ncells=None):
        p = self.problem
        n = p.Nx if ncells is None else ncells
        _dev(W, self.cdtype, (None, p.N, p.N, 2, 2), "state")
        if W.shape[0] < n:
            raise ValueError(f"expected at least {n} cells, got {W.shape[0]}")

    def collision(self, W, C=None, ncells=None):
        """qb_collision: C[W] for the first `ncells` cells of W."""
        import torch

        n = W.shape[0] if ncells is None else int(ncells)
        self._check_state(W, n)
        if C is None:
            C = torch.empty_like(W)
        self._check_state(C, n)
        _check(self.lib.qb_collision(self.handle, _ptr(W), _ptr(C), n, _stream()), "qb_collision")
        return C

    def collision_static(self, W, C=None, ncells=None):
        """qb_collision_static: C[W] with the library's fixed scratch array
        in place of the plan's collision buffers (allocates nothing)."""
        import torch

        n = W.shape[0] if ncells is None else int(ncells)
        self._check_state(W, n)
        if C is None:
            C = torch.empty_like(W)
        self._check_state(C, n)
        _check(self.lib.qb_collision_static(self.handle, _ptr(W), _ptr(C), n, _stream()), "qb_collision_static")
        return C

    def transport_step(self, W, dt):
        """qb_transport_step: one limited transport step of length dt, in place."""
        self._check_state(W)
        _check(self.lib.qb_transport_step(self.handle, _ptr(W), float(dt), _stream()), "qb_transport_step")
        return W

    def step(self, W, B=None, dt=1e-3, nsteps=1, moments=None, inflow=None):
        """qb_step: nsteps splitting steps in place; B float64 [Nx, 3] or None;
        moments float64 [nsteps + 1, Nx, 7] or None; with inflow (float64
        [nsteps, 7]) qb_step_fluxes, which also returns the moments of the
        net inflow through the walls during each step."""
        import torch

        self._check_state(W)
        p = self.problem
        bp = self._field(B)
        mp = ctypes.c_void_p(0)
        if moments is not None:
            mp = _dev(moments, torch.float64, (nsteps + 1, p.Nx, 7), "moments")
        if inflow is not None:
            ip = _dev(inflow, torch.float64, (nsteps, 7), "inflow")
            _check(self.lib.qb_step_fluxes(self.handle, _ptr(W), bp, float(dt), int(nsteps), mp, ip,
                                           _stream()), "qb_step_fluxes")
            return W
        _check(self.lib.qb_step(self.handle, _ptr(W), bp, float(dt), int(nsteps), mp, _stream()), "qb_step")
        return W

    def _field(self, B):
        import torch

        if B is None:
            return ctypes.c_void_p(0)
        return _dev(B, torch.float64, (self.problem.Nx, 3), "B")

    # ------------------------------------------------------------ reverse mode
    def enable_adjoint(self):
        """qb_plan_enable_adjoint: lay out the reverse-mode buffers in a
        workspace of qb_adjoint_workspace_bytes (once)."""
        if self.ws_adj is not None:
            return
        nbytes = self.lib.qb_adjoint_workspace_bytes(self.handle)
        ws = _workspace(nbytes)
        _check(self.lib.qb_plan_enable_adjoint(self.handle, _ptr(ws), ws.numel()), "qb_plan_enable_adjoint")
        self.ws_adj = ws

    def collision_vjp(self, W, lam, G=None, ncells=None):
        """qb_collision_vjp: G = C'(W)^T lam (torch's complex-gradient convention)."""
        import torch

        n = W.shape[0] if ncells is None else int(ncells)
        self._check_state(W, n)
        self._check_state(lam, n)
        if G is None:
            G = torch.empty_like(W)
        self._check_state(G, n)
        _check(self.lib.qb_collision_vjp(self.handle, _ptr(W), _ptr(lam), _ptr(G), n, _stream()),
               "qb_collision_vjp")
        return G

    def transport_vjp(self, W, dt, lam, G=None):
        """qb_transport_vjp: G = T'(W)^T lam for one transport step of length dt."""
        import torch

        self._check_state(W)
        self._check_state(lam)
        if G is None:
            G = torch.empty_like(W)
        self._check_state(G)
        _check(self.lib.qb_transport_vjp(self.handle, _ptr(W), float(dt), _ptr(lam), _ptr(G), _stream()),
               "qb_transport_vjp")
        return G

    @property
    def trace_bytes(self):
        """qb_trace_bytes: bytes of one step record of qb_step_trace."""
        return self.lib.qb_trace_bytes(self.handle)

    def new_trace(self, nsteps):
        import torch

        return torch.empty(int(nsteps) * self.trace_bytes, dtype=torch.uint8, device="cuda")

    def step_trace(self, W, B, dt, nsteps, trace):
        """qb_step_trace: nsteps steps in place, one record per step in `trace`."""
        import torch

        self._check_state(W)
        tp = _dev(trace, torch.uint8, (None,), "trace")
        if trace.numel() < nsteps * self.trace_bytes:
            raise ValueError("trace too small")
        _check(self.lib.qb_step_trace(self.handle, _ptr(W), self._field(B), float(dt), int(nsteps), tp,
                                      _stream()), "qb_step_trace")
        return W

    def adjoint_step(self, lam_next, B, dt, W=None, record=None, lam=None, gB=None):
        """qb_adjoint_step: cotangent of a step's input from that of its output;
        `record` (a view of a step_trace buffer) or the input state W."""
        import torch

        self._check_state(lam_next)
        if lam is None:
            lam = torch.empty_like(lam_next)
        self._check_state(lam)
        wp = ctypes.c_void_p(0)
        if W is not None:
            self._check_state(W)
            wp = _ptr(W)
        rp = ctypes.c_void_p(0)
        if record is not None:
            rp = _dev(record, torch.uint8, (self.trace_bytes,), "record")
        gp = ctypes.c_void_p(0)
        if gB is not None:
            gp = _dev(gB, torch.float64, (self.problem.Nx, 3), "gB")
        _check(self.lib.qb_adjoint_step(self.handle, wp, rp, self._field(B), float(dt), _ptr(lam_next), _ptr(lam),
                                        gp, _stream()), "qb_adjoint_step")
        return lam

    def diagnostics(self, W, C=None, fd=None, out=None):
        """qb_diagnostics: float64 [Nx, QB_DIAG_FIELDS] per-cell entropy,
        entropy production (with C = C[W]), relative entropies to the global
        Fermi-Dirac state fd = (inv_kT, mu_up, mu_down, U) and to the local
        fit, eigenvalue range and the fit itself (columns: DIAG_NAMES)."""
        import torch

        self._check_state(W)
        cp = ctypes.c_void_p(0)
        if C is not None:
            self._check_state(C)
            cp = _ptr(C)
        gp = None
        if fd is not None:
            inv_kT, mu_up, mu_down, U = fd
            gp = BC("dirichlet", inv_kT, mu_up, mu_down, U)._c().state
        if out is None:
            out = torch.empty((self.problem.Nx, QB_DIAG_FIELDS), dtype=torch.float64, device=W.device)
        op = _dev(out, torch.float64, (self.problem.Nx, QB_DIAG_FIELDS), "out")
        _check(self.lib.qb_diagnostics(self.handle, _ptr(W), cp, None if gp is None else ctypes.byref(gp), op,
                                       _stream()), "qb_diagnostics")
        return out

    def moments(self, W, out=None):
        """qb_moments: float64 [Nx, 7] moments of W."""
        import torch

        self._check_state(W)
        if out is None:
            out = torch.empty((self.problem.Nx, 7), dtype=torch.float64, device=W.device)
        op = _dev(out, torch.float64, (self.problem.Nx, 7), "out")
        _check(self.lib.qb_moments(self.handle, _ptr(W), op, _stream()), "qb_moments")
        return out

    # ------------------------------------------------------------ tiles
    TILES = {32: (16, 8), 64: (16, 32, 8), 128: (16, 32)}

    def set_tile(self, E):
        """qb_plan_set_tile: FFT tile shape (elements per thread) of this plan."""
        _check(self.lib.qb_plan_set_tile(self.handle, int(E)), "qb_plan_set_tile")

    def tune(self, ncells=None):
        """qb_plan_tune: time every compiled tile shape, keep the fastest; returns E."""
        e = ctypes.c_int32()
        n = self.problem.Nx if ncells is None else int(ncells)
        _check(self.lib.qb_plan_tune(self.handle, n, ctypes.byref(e), _stream()), "qb_plan_tune")
        return e.value

    def set_adjoint_tile(self, E):
        """qb_plan_set_adjoint_tile: tile shape of the reverse-mode pipeline
        (0 follows the forward tile)."""
        _check(self.lib.qb_plan_set_adjoint_tile(self.handle, int(E)), "qb_plan_set_adjoint_tile")

    def set_persistent(self, persistent):
        """qb_plan_set_persistent: persistent (grid-stride) launches of the
        heavy collision kernels, or one workgroup per task."""
        _check(self.lib.qb_plan_set_persistent(self.handle, 1 if persistent else 0), "qb_plan_set_persistent")

    def set_adjoint_variant(self, v):
        """qb_plan_set_adjoint_variant: I_3 adjoint kernel 0 or 1."""
        _check(self.lib.qb_plan_set_adjoint_variant(self.handle, int(v)), "qb_plan_set_adjoint_variant")

    def set_pairing(self, paired):
        """qb_plan_set_pairing: I_3 kernel with or without node pairing."""
        _check(self.lib.qb_plan_set_pairing(self.handle, 1 if paired else 0), "qb_plan_set_pairing")

    TERMS = {"conservative": 1, "dissipative": 2, "all": 3}
    LIMITERS = {"minmod": 0, "superbee": 1, "mc": 2, "van_leer": 3}
    FIELDS = {"heun": 0, "rotation": 1}

    def set_scheme(self, limiter="minmod", field="heun"):
        """qb_plan_set_scheme: slope limiter of the transport (LIMITERS) and
        treatment of the field term (FIELDS)."""
        _check(self.lib.qb_plan_set_scheme(self.handle, self.LIMITERS[limiter], self.FIELDS[field]),
               "qb_plan_set_scheme")

    def set_terms(self, terms):
        """qb_plan_set_terms: assemble only C_c ('conservative'), only C_d
        ('dissipative') or both ('all', the default)."""
        _check(self.lib.qb_plan_set_terms(self.handle, self.TERMS[terms]), "qb_plan_set_terms")

    def config(self):
        """qb_plan_config: tile E, I_3 adjoint variant, node pairing and the
        reverse-mode tile in use."""
        e, v, pn, ae, ps = (ctypes.c_int32() for _ in range(5))
        _check(self.lib.qb_plan_config(self.handle, ctypes.byref(e), ctypes.byref(v), ctypes.byref(pn),
                                       ctypes.byref(ae), ctypes.byref(ps)), "qb_plan_config")
        return {"tile": e.value, "adjoint_variant": v.value, "paired_nodes": bool(pn.value),
                "adjoint_tile": ae.value, "persistent": bool(ps.value)}

    def profile(self, enable=True):
        """qb_profile: bracket every launch of this plan with HIP events."""
        _check(self.lib.qb_profile(self.handle, 1 if enable else 0), "qb_profile")

    def profile_read(self, kernel):
        """qb_profile_read: (total ms, launches) of one kernel class since the last read."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(self.lib.qb_profile_read(self.handle, KERNELS[kernel], ctypes.byref(ms), ctypes.byref(n)),
               "qb_profile_read")
        return ms.value, n.value

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.qb_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# C-ABI names, for callers that prefer them
def qb_collision(plan, W, C=None, ncells=None):
    return plan.collision(W, C, ncells)


def qb_transport_step(plan, W, dt):
    return plan.transport_step(W, dt)


def qb_step(plan, W, B=None, dt=1e-3, nsteps=1, moments=None):
    return plan.step(W, B, dt, nsteps, moments)


def qb_moments(plan, W, out=None):
    return plan.moments(W, out)


QB_BATCH_GRAPH = 1


class Batch:
    """A qb_batch: independent problems (uneven Nx, N) advanced together."""

    def __init__(self, problems):
        import torch

        self.lib = load()
        self.problems = list(problems)
        arr = (_Problem * len(self.problems))(*[p._c() for p in self.problems])
        nbytes = self.lib.qb_batch_workspace_bytes(arr, len(self.problems))
        if nbytes == 0:
            _check(QB_EINVAL, "qb_batch_workspace_bytes")
        self.ws = _workspace(nbytes)
        h = ctypes.c_void_p()
        _check(self.lib.qb_batch_create(arr, len(self.problems), _ptr(self.ws), self.ws.numel(), ctypes.byref(h)),
               "qb_batch_create")
        self.handle = h
        prec = {p.precision for p in self.problems}
        self.cdtype = torch.complex128 if prec == {"f64"} else torch.complex64

    @property
    def nbytes(self):
        return self.lib.qb_batch_bytes(self.handle)

    def tune(self):
        _check(self.lib.qb_batch_tune(self.handle, _stream()), "qb_batch_tune")

    def set_persistent(self, persistent):
        """qb_batch_set_persistent: persistent (grid-stride) collision launches."""
        _check(self.lib.qb_batch_set_persistent(self.handle, 1 if persistent else 0), "qb_batch_set_persistent")

    def step(self, Ws, Bs=None, dt=1e-3, nsteps=1, moments=None, graph=False):
        """qb_batch_step: nsteps steps of every problem in place."""
        import torch

        n = len(self.problems)
        if len(Ws) != n:
            raise ValueError("one state per problem")
        vp = ctypes.c_void_p
        Wp = (vp * n)(*[_dev(W, self.cdtype, (p.Nx, p.N, p.N, 2, 2), "state").value for W, p in zip(Ws, self.problems)])
        Bp = None
        if Bs is not None:
            if len(Bs) != n:
                raise ValueError("one field (or None) per problem")
            Bp = (vp * n)(*[0 if B is None else _dev(B, torch.float64, (p.Nx, 3), "B").value
                            for B, p in zip(Bs, self.problems)])
        Mp = None
        if moments is not None:
            if len(moments) != n:
                raise ValueError("one moments array (or None) per problem")
            Mp = (vp * n)(*[0 if m is None else _dev(m, torch.float64, (nsteps + 1, p.Nx, 7), "moments").value
                            for m, p in zip(moments, self.problems)])
        _check(self.lib.qb_batch_step(self.handle, Wp, Bp, float(dt), int(nsteps), Mp,
                                      QB_BATCH_GRAPH if graph else 0, _stream()), "qb_batch_step")
        return Ws

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.qb_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()


def probe_fma(precision="f32", iters=4096):
    """qb_probe_fma: sustained vector FMA rate in TFLOP/s on the current GPU."""
    import torch

    lib = load()
    scratch = torch.empty(32768, dtype=torch.uint8, device="cuda")
    out = ctypes.c_double()
    _check(lib.qb_probe_fma(QB_F64 if precision == "f64" else QB_F32, int(iters), _ptr(scratch), ctypes.byref(out),
                            _stream()), "qb_probe_fma")
    return out.value


def probe_copy(mib=1024, reps=5):
    """qb_probe_copy: device copy bandwidth in GB/s (read + write) over two
    buffers of `mib` MiB."""
    import torch

    lib = load()
    n = int(mib) << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    out = ctypes.c_double()
    _check(lib.qb_probe_copy(_ptr(src), _ptr(dst), n, int(reps), ctypes.byref(out), _stream()), "qb_probe_copy")
    return out.value
