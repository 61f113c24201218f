"""CPU checks of the C-ABI library: it loads without a GPU, exports every
symbol include/qb.h declares, and rejects invalid problems before touching
the device (argument validation runs on the host)."""
import ctypes
import os
import re

import pytest

import paper_1408_1782_amd as qb
from paper_1408_1782_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "qb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)       # drop comments
    return sorted(set(re.findall(r"\b(qb_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_header_symbols():
    lib = qb.load()
    names = header_functions()
    assert names, "no declarations parsed"
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_version_and_strerror():
    lib = qb.load()
    assert lib.qb_version() >= 100
    for s in (0, -1, -2, -3, -4, -5):
        assert lib.qb_strerror(s)


# a stand-in workspace address: every call below returns before the device
# is touched, so the library never dereferences it
FAKE_WS = ctypes.c_void_p(1 << 40)


def _create(**kw):
    lib = qb.load()
    p = qb.Problem(**{**dict(Nx=4, N=16, J=8, M=8), **kw})._c()
    h = ctypes.c_void_p()
    st = lib.qb_plan_create(ctypes.byref(p), 0, FAKE_WS, 1 << 40, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize(
    "kw,status",
    [
        (dict(N=24), _lib.QB_ENOTSUP),
        (dict(N=128), _lib.QB_ENOTSUP),
        (dict(J=7), _lib.QB_ENOTSUP),
        (dict(Nx=0), _lib.QB_EINVAL),
        (dict(M=0), _lib.QB_EINVAL),
        (dict(L=-1.0), _lib.QB_EINVAL),
        (dict(R=-0.5), _lib.QB_EINVAL),
        (dict(left=qb.BC("dirichlet", inv_kT=1.0)), _lib.QB_EINVAL),           # mixed periodic
        (dict(left=qb.BC("maxwell", inv_kT=1.0, alpha=1.5),
              right=qb.BC("dirichlet", inv_kT=1.0)), _lib.QB_EINVAL),       # alpha out of range
        (dict(left=qb.BC("dirichlet", inv_kT=0.0),
              right=qb.BC("dirichlet", inv_kT=1.0)), _lib.QB_EINVAL),       # no temperature
    ],
)
def test_invalid_problems_rejected_on_host(kw, status):
    st, h = _create(**kw)
    assert st == status
    assert not h.value


def test_null_arguments_rejected():
    lib = qb.load()
    assert lib.qb_collision(None, None, None, 1, None) == _lib.QB_EINVAL
    assert lib.qb_step(None, None, None, 1e-3, 1, None, None) == _lib.QB_EINVAL
    assert lib.qb_plan_create(None, 0, None, 0, None) == _lib.QB_EINVAL
    assert lib.qb_plan_enable_adjoint(None, None, 0) == _lib.QB_EINVAL
    assert lib.qb_adjoint_workspace_bytes(None) == 0
    assert lib.qb_batch_create(None, 0, None, 0, None) == _lib.QB_EINVAL
    assert lib.qb_batch_workspace_bytes(None, 0) == 0
    assert lib.qb_plan_chunk_cells(None) == 0
    assert lib.qb_collision_vjp(None, None, None, None, 1, None) == _lib.QB_EINVAL
    assert lib.qb_transport_vjp(None, None, 1e-3, None, None, None) == _lib.QB_EINVAL
    assert lib.qb_step_trace(None, None, None, 1e-3, 1, None, None) == _lib.QB_EINVAL
    assert lib.qb_adjoint_step(None, None, None, None, 1e-3, None, None, None, None) == _lib.QB_EINVAL
    assert lib.qb_trace_bytes(None) == 0
    assert lib.qb_diagnostics(None, None, None, None, None, None) == _lib.QB_EINVAL
    assert lib.qb_plan_set_terms(None, 3) == _lib.QB_EINVAL
    assert lib.qb_plan_set_scheme(None, 0, 0) == _lib.QB_EINVAL
    assert lib.qb_probe_fma(0, 1, None, None, None) == _lib.QB_EINVAL
    assert lib.qb_probe_copy(None, None, 16, 1, None, None) == _lib.QB_EINVAL
    assert lib.qb_step_fluxes(None, None, None, 1e-3, 1, None, None, None) == _lib.QB_EINVAL


# ---------------------------------------------------------------- workspaces
def _problem(**kw):
    return qb.Problem(**{**dict(Nx=4, N=16, J=8, M=8), **kw})._c()


def test_workspace_bytes_on_host():
    """qb_workspace_bytes is host arithmetic: positive for valid problems,
    0 for invalid ones, growing with the cell count per launch and the grid."""
    lib = qb.load()
    small = lib.qb_workspace_bytes(ctypes.byref(_problem()), 0)
    assert small > 0
    assert lib.qb_workspace_bytes(ctypes.byref(_problem(N=24)), 0) == 0
    assert lib.qb_workspace_bytes(ctypes.byref(_problem()), -1) == 0
    assert lib.qb_workspace_bytes(ctypes.byref(_problem()), 1) < small        # one cell per launch
    assert lib.qb_workspace_bytes(ctypes.byref(_problem()), 4) == small       # default: min(Nx, 512)
    assert lib.qb_workspace_bytes(ctypes.byref(_problem()), 100) == small     # clamped to Nx
    assert lib.qb_workspace_bytes(ctypes.byref(_problem(N=32)), 0) > small
    assert lib.qb_workspace_bytes(ctypes.byref(_problem(precision="f32")), 0) < small
    probs = (_lib._Problem * 2)(_problem(), _problem(Nx=6, N=32, M=8))
    assert lib.qb_batch_workspace_bytes(probs, 2) > lib.qb_workspace_bytes(ctypes.byref(_problem(N=32, Nx=6)), 0)
    mixed = (_lib._Problem * 2)(_problem(), _problem(precision="f32"))
    assert lib.qb_batch_workspace_bytes(mixed, 2) == 0


def test_short_workspace_rejected_on_host():
    """A workspace one byte short is refused with QB_EWORKSPACE before any
    HIP call (the check is host arithmetic), for plans and batches."""
    lib = qb.load()
    p = _problem()
    need = lib.qb_workspace_bytes(ctypes.byref(p), 0)
    h = ctypes.c_void_p()
    assert lib.qb_plan_create(ctypes.byref(p), 0, FAKE_WS, need - 1, ctypes.byref(h)) == _lib.QB_EWORKSPACE
    assert not h.value
    assert lib.qb_plan_create(ctypes.byref(p), 0, None, need, ctypes.byref(h)) == _lib.QB_EINVAL
    assert lib.qb_plan_create(ctypes.byref(p), -2, FAKE_WS, need, ctypes.byref(h)) == _lib.QB_EINVAL
    probs = (_lib._Problem * 2)(_problem(), _problem(Nx=6, N=32, M=8))
    bneed = lib.qb_batch_workspace_bytes(probs, 2)
    b = ctypes.c_void_p()
    assert lib.qb_batch_create(probs, 2, FAKE_WS, bneed - 1, ctypes.byref(b)) == _lib.QB_EWORKSPACE
    assert not b.value


def _undefined_symbols(path):
    """Dynamic symbols the library imports (nm -D --undefined-only)."""
    import shutil
    import subprocess

    if shutil.which("nm"):
        out = subprocess.run(["nm", "-D", "--undefined-only", path], capture_output=True, text=True, check=True)
        return {line.split()[-1].split("@")[0] for line in out.stdout.splitlines() if line.strip()}
    raise RuntimeError("nm not found")


def test_library_imports_no_device_allocator():
    """No entry point can allocate device memory: libqb.so imports none of
    HIP's allocation or free routines (its memory is the caller's)."""
    names = _undefined_symbols(_lib.lib_path())
    assert "hipLaunchKernel" in names or any(n.startswith("hip") for n in names)
    banned = {n for n in names if re.match(r"hip(Ext)?(Malloc|Free|HostAlloc|HostMalloc|MallocManaged|"
                                           r"MallocAsync|MallocPitch|Malloc3D|MallocArray|FreeAsync|MemPool)", n)}
    assert not banned, sorted(banned)
