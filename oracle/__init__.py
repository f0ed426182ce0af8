"""CPU FP64 oracle for the five-equation RHS -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The HIP library never loads it, and it shares
no code with the HIP library: the only common input is the seeded primitive
state built by ``workloads``.

Contents
--------
* ``oracle.c`` (built into ``liboracle.so`` with gcc) -- plain loops,
  -O2 -ffp-contract=off, OpenMP across independent lines/cells.
* ``exact_riemann`` -- exact Riemann solution for one stiffened gas (Sod pin).
* ``torch_ref`` -- the same RHS written with plain PyTorch CPU float64 ops,
  used for reference gradients by autograd.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

ORC_OK, ORC_ERR_ARG, ORC_ERR_NONFINITE = 0, -1, -5


def build(verbose: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class OrcProblem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("num_fluids", ctypes.c_int32),
        ("bc_lo", ctypes.c_int32 * 3),
        ("bc_hi", ctypes.c_int32 * 3),
        ("dx", ctypes.c_double * 3),
        ("gamma", ctypes.c_double * 2),
        ("pi_inf", ctypes.c_double * 2),
        ("weno_eps", ctypes.c_double),
        ("weno_variant", ctypes.c_int32),
        ("riemann", ctypes.c_int32),
        ("low_mach", ctypes.c_int32),
        ("model", ctypes.c_int32),
        ("faces", ctypes.POINTER(ctypes.c_double) * 3),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(OrcProblem)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        sig = {
            "orc_num_eqs": (ctypes.c_int, [P]),
            "orc_validate": (ctypes.c_int, [P]),
            "orc_weno5_js_left": (ctypes.c_double, [dp, ctypes.c_double]),
            "orc_weno5_js_right": (ctypes.c_double, [dp, ctypes.c_double]),
            "orc_weno5_z_left": (ctypes.c_double, [dp, ctypes.c_double]),
            "orc_weno5_z_right": (ctypes.c_double, [dp, ctypes.c_double]),
            "orc_weno5_m_left": (ctypes.c_double, [dp, ctypes.c_double]),
            "orc_weno5_m_right": (ctypes.c_double, [dp, ctypes.c_double]),
            "orc_weno_m_map": (ctypes.c_double, [ctypes.c_double, ctypes.c_double]),
            "orc_teno5_left": (ctypes.c_double, [dp, ctypes.c_double, ctypes.c_double]),
            "orc_teno5_right": (ctypes.c_double, [dp, ctypes.c_double, ctypes.c_double]),
            "orc_hllc": (ctypes.c_int, [P, ctypes.c_int, dp, dp, dp, dp]),
            "orc_hll": (ctypes.c_int, [P, ctypes.c_int, dp, dp, dp, dp]),
            "orc_thornber": (None, [P, ctypes.c_int, dp, dp]),
            "orc_kapila_K": (ctypes.c_double, [P, dp]),
            "orc_nu_stencil": (None, [dp, dp, dp, dp, dp, dp, dp]),
            "orc_weno5_nu": (None, [dp, dp, ctypes.c_double, dp, dp]),
            "orc_rhs": (ctypes.c_int, [P, dp, dp]),
            "orc_rhs_cells": (ctypes.c_int, [P, dp, ctypes.c_int64, i64p, dp]),
            "orc_max_signal": (ctypes.c_int, [P, dp, dp]),
            "orc_step": (ctypes.c_int, [P, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]),
            "orc_run": (ctypes.c_int, [P, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]),
            "orc_prim_to_cons": (ctypes.c_int, [P, dp, dp]),
            "orc_cons_to_prim": (ctypes.c_int, [P, dp, dp]),
            "orc_sound_speed_sq": (ctypes.c_int, [P, dp, dp]),
            "orc_conserved_sums": (ctypes.c_int, [P, dp, dp]),
            "orc_abi_version": (ctypes.c_int, []),
            "orc_num_threads": (ctypes.c_int, []),
            "orc_set_num_threads": (None, [ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def problem(ndim, n, num_fluids, dx, gamma, pi_inf, bc_lo, bc_hi, weno_eps=1e-6, weno_variant=0,
            riemann=0, low_mach=0, model=0, faces=None) -> OrcProblem:
    """faces: per axis None (uniform dx) or the n + 1 face coordinates of a
    non-uniform grid.  The arrays are kept on the returned struct."""
    P = OrcProblem()
    P._faces = []
    for d in range(3):
        f = None if faces is None or d >= len(faces) else faces[d]
        if f is None:
            P.faces[d] = ctypes.POINTER(ctypes.c_double)()
        else:
            a = np.ascontiguousarray(f, dtype=np.float64)
            P._faces.append(a)
            P.faces[d] = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    P.ndim = ndim
    n = tuple(n) + (1,) * (3 - len(n))
    for d in range(3):
        P.n[d] = int(n[d])
        P.bc_lo[d] = int(bc_lo[d]) if d < len(bc_lo) else 1
        P.bc_hi[d] = int(bc_hi[d]) if d < len(bc_hi) else 1
        P.dx[d] = float(dx[d]) if d < len(dx) else 1.0
    P.num_fluids = num_fluids
    for i in range(2):
        P.gamma[i] = float(gamma[i]) if i < len(gamma) else float(gamma[0])
        P.pi_inf[i] = float(pi_inf[i]) if i < len(pi_inf) else float(pi_inf[0])
    P.weno_eps = weno_eps
    P.weno_variant = int(weno_variant)
    P.riemann = int(riemann)
    P.low_mach = int(low_mach)
    P.model = int(model)
    return P


def problem_from_case(case) -> OrcProblem:
    return problem(**case.problem_kwargs())


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle returned {code}")
        self.code = code


def _check(rc, allow_nonfinite=False):
    if rc == ORC_OK or (allow_nonfinite and rc == ORC_ERR_NONFINITE):
        return rc
    raise OracleError(rc)


class Oracle:
    """Thin numpy front end to liboracle.so for one problem."""

    def __init__(self, case=None, **kw):
        self.P = problem_from_case(case) if case is not None else problem(**kw)
        self.L = lib()
        if self.L.orc_validate(ctypes.byref(self.P)) != ORC_OK:
            raise OracleError(ORC_ERR_ARG)
        self.neq = self.L.orc_num_eqs(ctypes.byref(self.P))
        self.shape = (self.neq, self.P.n[2], self.P.n[1], self.P.n[0])

    def _arr(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.shape == self.shape, (a.shape, self.shape)
        return a

    def prim_to_cons(self, w):
        w = self._arr(w)
        q = np.empty_like(w)
        _check(self.L.orc_prim_to_cons(ctypes.byref(self.P), _dp(w), _dp(q)))
        return q

    def cons_to_prim(self, q):
        q = self._arr(q)
        w = np.empty_like(q)
        _check(self.L.orc_cons_to_prim(ctypes.byref(self.P), _dp(q), _dp(w)))
        return w

    def sound_speed_sq(self, q):
        q = self._arr(q)
        c2 = np.empty(self.shape[1:])
        _check(self.L.orc_sound_speed_sq(ctypes.byref(self.P), _dp(q), _dp(c2)))
        return c2

    def rhs(self, q, allow_nonfinite=False):
        q = self._arr(q)
        r = np.empty_like(q)
        _check(self.L.orc_rhs(ctypes.byref(self.P), _dp(q), _dp(r)), allow_nonfinite)
        return r

    def rhs_cells(self, q, cells):
        q = self._arr(q)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.empty((cells.size, self.neq))
        _check(self.L.orc_rhs_cells(ctypes.byref(self.P), _dp(q), cells.size,
                                    cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(out)))
        return out

    def max_signal(self, q):
        q = self._arr(q)
        s = ctypes.c_double()
        _check(self.L.orc_max_signal(ctypes.byref(self.P), _dp(q), ctypes.byref(s)))
        return s.value

    def step(self, q, cfl=0.0, dt_fixed=0.0, t_remaining=0.0):
        """Advance q in place by one SSP-RK3 step; returns dt."""
        assert q.dtype == np.float64 and q.flags.c_contiguous and q.shape == self.shape
        dt = ctypes.c_double()
        _check(self.L.orc_step(ctypes.byref(self.P), _dp(q), cfl, dt_fixed, t_remaining,
                               ctypes.byref(dt)))
        return dt.value

    def run(self, q, nsteps, cfl=0.0, dt_fixed=0.0):
        """Advance q in place by nsteps steps; returns the array of dts."""
        assert q.dtype == np.float64 and q.flags.c_contiguous and q.shape == self.shape
        dts = np.empty(max(nsteps, 1))
        _check(self.L.orc_run(ctypes.byref(self.P), _dp(q), nsteps, cfl, dt_fixed, _dp(dts)))
        return dts[:nsteps]

    def run_to(self, q, t_end, cfl):
        """Advance q in place to time t_end with CFL steps clipped at t_end."""
        t, nsteps = 0.0, 0
        while t < t_end:
            dt = self.step(q, cfl=cfl, t_remaining=t_end - t)
            t += dt
            nsteps += 1
        return nsteps

    def conserved_sums(self, q):
        q = self._arr(q)
        s = np.empty(self.neq)
        _check(self.L.orc_conserved_sums(ctypes.byref(self.P), _dp(q), _dp(s)))
        return s

    def hllc(self, d, wl, wr):
        wl = np.ascontiguousarray(wl, dtype=np.float64)
        wr = np.ascontiguousarray(wr, dtype=np.float64)
        F = np.empty(self.neq)
        uf = ctypes.c_double()
        rc = self.L.orc_hllc(ctypes.byref(self.P), d, _dp(wl), _dp(wr), _dp(F), ctypes.byref(uf))
        return F, uf.value, rc

    def thornber(self, d, wl, wr):
        """The low-Mach corrected face states (copies)."""
        wl = np.array(wl, dtype=np.float64)
        wr = np.array(wr, dtype=np.float64)
        self.L.orc_thornber(ctypes.byref(self.P), d, _dp(wl), _dp(wr))
        return wl, wr

    def kapila_K(self, w):
        """Kapila's K (Sec. 2.1.1) of one primitive cell state w (neq values)."""
        w = np.ascontiguousarray(w, dtype=np.float64)
        return self.L.orc_kapila_K(ctypes.byref(self.P), _dp(w))

    def hll(self, d, wl, wr):
        """HLL face flux and face velocity (Sec. 3.2.2)."""
        wl = np.ascontiguousarray(wl, dtype=np.float64)
        wr = np.ascontiguousarray(wr, dtype=np.float64)
        F = np.empty(self.neq)
        uf = ctypes.c_double()
        rc = self.L.orc_hll(ctypes.byref(self.P), d, _dp(wl), _dp(wr), _dp(F), ctypes.byref(uf))
        return F, uf.value, rc


def nu_stencil(h, f=None):
    """Fifth-order reconstruction quantities on a non-uniform grid (Sec. 4.2.2)
    for the centre of five cells of widths h (and averages f): candidates at
    the right and left face, smoothness indicators, ideal weights at both
    faces (the first three are None without f)."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    out = [np.zeros(3) for _ in range(5)]
    fp = _dp(np.ascontiguousarray(f, dtype=np.float64)) if f is not None else None
    lib().orc_nu_stencil(fp, _dp(h), *[_dp(o) for o in out])
    qR, qL, beta, dR, dL = out
    if f is None:
        return None, None, None, dR, dL
    return qR, qL, beta, dR, dL


def weno5_nu(f, h, eps=1e-6):
    """WENO5-JS on a non-uniform grid: (value at the right face, value at the
    left face) of the centre of five cells with widths h and averages f."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    h = np.ascontiguousarray(h, dtype=np.float64)
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().orc_weno5_nu(_dp(f), _dp(h), eps, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP threads of the oracle's parallel loops from now on."""
    lib().orc_set_num_threads(int(n))


def weno5_js_left(f, eps=1e-6):
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().orc_weno5_js_left(_dp(f), eps)


def weno5_js_right(f, eps=1e-6):
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().orc_weno5_js_right(_dp(f), eps)


def weno5_z_left(f, eps=1e-6):
    """Left-biased WENO5-Z value (Sec. 4.2.2) from f[0..4] = f_{i-2..i+2}."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().orc_weno5_z_left(_dp(f), eps)


def weno5_z_right(f, eps=1e-6):
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().orc_weno5_z_right(_dp(f), eps)


def weno5_m_left(f, eps=1e-6):
    """Left-biased WENO5-M value (mapped JS weights, Sec. 3.2.1) from f[0..4]."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().orc_weno5_m_left(_dp(f), eps)


def weno5_m_right(f, eps=1e-6):
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().orc_weno5_m_right(_dp(f), eps)


def weno_m_map(w, d):
    """The weight map g_d(w) of WENO5-M."""
    return lib().orc_weno_m_map(float(w), float(d))


TENO_CT = 1e-5


def teno5_left(f, eps=1e-6, ct=TENO_CT):
    """Left-biased TENO5 value (Sec. 4.2.2) from f[0..4] = f_{i-2..i+2}."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().orc_teno5_left(_dp(f), eps, ct)


def teno5_right(f, eps=1e-6, ct=TENO_CT):
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().orc_teno5_right(_dp(f), eps, ct)
