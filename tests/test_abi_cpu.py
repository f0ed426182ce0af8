"""The C-ABI library loads, exports every declared symbol, and validates on the host."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfc355.h")


@pytest.fixture(scope="module")
def L():
    from paper_2503_07953_amd import _lib
    _lib.load()
    return _lib


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return set(re.findall(r"\b(mfc_[a-z0-9_]+)\s*\(", txt))


def test_every_declared_symbol_is_exported(L):
    lib = L.load()
    declared = _declared()
    assert len(declared) >= 14
    missing = [s for s in declared if not hasattr(lib, s)]
    assert not missing, missing
    # the binding knows every declared symbol
    assert declared <= set(L.SIGNATURES)


def _prob(L, **kw):
    base = dict(ndim=2, n=(8, 8), num_fluids=2, dx=(0.1, 0.1), gamma=(6.12, 1.4), pi_inf=(3.43e8, 0.0),
                bc_lo=(1, 1), bc_hi=(1, 1))
    base.update(kw)
    return L.make_problem(**base)


def test_num_eqs(L):
    lib = L.load()
    for nd in (1, 2, 3):
        assert lib.mfc_num_eqs(ctypes.byref(_prob(L, ndim=nd, n=(8,) * nd, dx=(0.1,) * nd))) == 2 * 2 + nd + 1
        assert lib.mfc_num_eqs(ctypes.byref(_prob(L, ndim=nd, n=(8,) * nd, dx=(0.1,) * nd, num_fluids=1))) == nd + 2
    assert lib.mfc_num_eqs(None) == L.MFC_ERR_ARG


@pytest.mark.parametrize("kw,code", [
    (dict(), 0),
    (dict(ndim=4), -3),
    (dict(num_fluids=3), -3),
    (dict(precision=7), -3),
    (dict(n=(2, 8)), -2),
    (dict(n=(8, 8, 2)), -2),
    (dict(n=(0, 8)), -2),
    (dict(n=(-4, 8)), -2),
    (dict(ndim=3, n=(8, 65536, 8), dx=(0.1,) * 3, bc_lo=(1,) * 3, bc_hi=(1,) * 3), -2),
    (dict(ndim=3, n=(8, 8, 65536), dx=(0.1,) * 3, bc_lo=(1,) * 3, bc_hi=(1,) * 3), -2),
    (dict(ndim=3, n=(1 << 21, 1 << 7, 1 << 7), dx=(0.1,) * 3, bc_lo=(1,) * 3, bc_hi=(1,) * 3), -2),
    (dict(ndim=3, n=(1 << 20, 1 << 7, 1 << 7), dx=(0.1,) * 3, bc_lo=(1,) * 3, bc_hi=(1,) * 3), 0),
    (dict(dx=(0.0, 0.1)), -1),
    (dict(gamma=(1.0, 1.4)), -1),
    (dict(pi_inf=(-1.0, 0.0)), -1),
    (dict(bc_lo=(0, 1), bc_hi=(1, 1)), -1),
    (dict(bc_lo=(5, 1)), -1),
    (dict(weno_eps=0.0), -1),
    (dict(weno_eps=1e-40), -1),
    (dict(weno_eps=9.9e-31), -1),
    (dict(weno_eps=1e-30), 0),
    (dict(weno_eps=float("inf")), -1),
    (dict(weno_variant=1), 0),
    (dict(weno_variant=2), 0),
    (dict(weno_variant=3), 0),
    (dict(weno_variant=4), -3),
    (dict(weno_variant=-1), -3),
    (dict(riemann=1), 0),
    (dict(riemann=2), -3),
    (dict(riemann=-1), -3),
    (dict(low_mach=1), 0),
    (dict(low_mach=2), 0),
    (dict(low_mach=2, riemann=1), -3),
    (dict(low_mach=3), -3),
    (dict(model=1), 0),
    (dict(model=1, low_mach=2), 0),
    (dict(model=1, num_fluids=1), -3),
    (dict(model=2), -3),
    (dict(model=-1), -3),
])
def test_validation_codes(L, kw, code):
    lib = L.load()
    assert lib.mfc_validate(ctypes.byref(_prob(L, **kw))) == code


def test_bad_abi_version_rejected_before_any_device_call(L):
    lib = L.load()
    p = _prob(L)
    p.abi_version = 99
    h = ctypes.c_void_p()
    assert lib.mfc_create(ctypes.byref(p), ctypes.byref(h)) == L.MFC_ERR_ARG
    assert not h.value
    p = _prob(L, n=(1, 8))
    assert lib.mfc_create(ctypes.byref(p), ctypes.byref(h)) == L.MFC_ERR_SHAPE


def test_null_context_and_status_strings(L):
    lib = L.load()
    assert lib.mfc_rhs(None, None, None, None) == L.MFC_ERR_ARG
    assert lib.mfc_step(None, None, 0.5, 0.0, 0.0, None, None) == L.MFC_ERR_ARG
    assert lib.mfc_destroy(None) == L.MFC_OK
    assert lib.mfc_last_error(None) == b"null context"
    for c in (0, -1, -2, -3, -4, -5, -6):
        assert L.status_string(c)
    assert lib.mfc_abi_version() == L.MFC_ABI_VERSION


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """No CPU fallback: without the HIP library every entry raises."""
    from paper_2503_07953_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libmfc355.so"))
    with pytest.raises(_lib.LibraryMissing):
        _lib.load()
    from paper_2503_07953_amd.solver import Solver
    with pytest.raises(_lib.LibraryMissing):
        Solver(1, (8,), 1, (0.1,), (1.4, 1.4), (0.0, 0.0), (1,), (1,))


def test_static_step_rejects_before_any_device_call(L):
    """mfc_step_static checks the problem, the arguments and the scratch size on
    the host; a problem whose step does not fit the static scratch is refused
    with MFC_ERR_SHAPE (no HIP call is made, so this runs without a GPU)."""
    lib = L.load()
    buf = (ctypes.c_double * 8)()
    flag = (ctypes.c_int * 1)()
    q, f = ctypes.cast(buf, ctypes.c_void_p), ctypes.cast(flag, ctypes.c_void_p)
    big = _prob(L, ndim=3, n=(128, 128, 128), dx=(0.1,) * 3, bc_lo=(1,) * 3, bc_hi=(1,) * 3)
    assert lib.mfc_step_static(ctypes.byref(big), q, 0.5, 0.0, 0.0, None, f, None) == L.MFC_ERR_SHAPE
    ok = _prob(L)
    assert lib.mfc_step_static(ctypes.byref(ok), q, 0.5, 0.1, 0.0, None, f, None) == L.MFC_ERR_ARG
    assert lib.mfc_step_static(ctypes.byref(ok), q, 0.5, 0.0, 0.0, None, None, None) == L.MFC_ERR_ARG
    assert lib.mfc_step_static(ctypes.byref(ok), None, 0.5, 0.0, 0.0, None, f, None) == L.MFC_ERR_ARG
    bad = _prob(L, weno_eps=0.0)
    assert lib.mfc_step_static(ctypes.byref(bad), q, 0.5, 0.0, 0.0, None, f, None) == L.MFC_ERR_ARG
    assert lib.mfc_step_static(None, q, 0.5, 0.0, 0.0, None, f, None) == L.MFC_ERR_ARG


def test_solver_takes_every_problem_field():
    """Solver.from_case passes the whole problem description (every key of
    Case.problem_kwargs) to the constructor, which must accept each one."""
    import inspect

    import workloads as W
    from paper_2503_07953_amd.solver import Solver
    params = inspect.signature(Solver.__init__).parameters
    c = W.random_case(2, (8, 8), nf=2, seed=0)
    c.faces = (W.stretched_faces(8), None, None)
    keys = c.problem_kwargs().keys()
    assert not [k for k in keys if k not in params]


def test_set_grid_needs_a_context(L):
    lib = L.load()
    buf = (ctypes.c_double * 9)(*range(9))
    assert lib.mfc_set_grid(None, 0, ctypes.cast(buf, ctypes.c_void_p)) == L.MFC_ERR_ARG
