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


def _create(**kw):
    lib = qb.load()
    p = qb.Problem(**{**dict(Nx=4, N=16, J=8, M=8), **kw})._c()
    h = ctypes.c_void_p()
    st = lib.qb_plan_create(ctypes.byref(p), ctypes.byref(h))
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
    assert lib.qb_plan_create(None, None) == _lib.QB_EINVAL
    assert lib.qb_plan_enable_adjoint(None) == _lib.QB_EINVAL
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
