"""Python front end of libmfc355: one context per problem, torch device tensors.

Every method marshals arguments to one C-ABI call of the same name; the
computation runs in the library's HIP kernels on the current torch stream.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """Owns one mfc_ctx.  `precision` is "fp64" or "fp32" (the mixed FP32 form)."""

    def __init__(self, ndim, n, num_fluids, dx, gamma, pi_inf, bc_lo, bc_hi, weno_eps=1e-6,
                 precision="fp64", device="cuda", weno_variant=0, riemann=0, low_mach=0, model=0, faces=None):
        self.lib = L.load()
        self.precision = precision
        prec = L.MFC_FP64 if precision == "fp64" else L.MFC_FP32_MIXED
        self.prob = L.make_problem(ndim, n, num_fluids, dx, gamma, pi_inf, bc_lo, bc_hi, weno_eps, prec, weno_variant,
                                   riemann, low_mach, model)
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.device = torch.device(device)
        rc = self.lib.mfc_validate(ctypes.byref(self.prob))
        if rc != L.MFC_OK:
            raise L.MfcError(rc, "invalid problem")
        self.neq = self.lib.mfc_num_eqs(ctypes.byref(self.prob))
        self.n = tuple(self.prob.n)
        self.shape = (self.neq, self.n[2], self.n[1], self.n[0])
        self.ndim = ndim
        self.num_fluids = num_fluids
        self.dx = tuple(self.prob.dx)
        with torch.cuda.device(self.device):
            h = ctypes.c_void_p()
            rc = self.lib.mfc_create(ctypes.byref(self.prob), ctypes.byref(h))
        if rc != L.MFC_OK:
            raise L.MfcError(rc, "mfc_create")
        self.ctx = h
        self._dev_index = self.device.index if self.device.index is not None else torch.cuda.current_device()
        if faces is not None:
            for d, f in enumerate(faces):
                if f is not None:
                    self.set_grid(d, f)
        self._scal = torch.zeros(4, dtype=torch.float64, device=self.device)

    @classmethod
    def from_case(cls, case, precision="fp64", device="cuda"):
        return cls(**case.problem_kwargs(), precision=precision, device=device)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            try:
                self.lib.mfc_destroy(ctx)
            except Exception:
                pass
            self.ctx = None

    # -------------------------------------------------------------- helpers
    def _check(self, rc, what):
        if rc != L.MFC_OK:
            msg = self.lib.mfc_last_error(self.ctx).decode()
            raise L.MfcError(rc, f"{what}: {msg}")

    def _arr(self, t, name="q"):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if (t.dtype != self.dtype or t.device.type != "cuda" or t.device.index != self._dev_index
                or tuple(t.shape) != self.shape or not t.is_contiguous()):
            raise ValueError(f"{name}: expected contiguous {self.dtype} cuda tensor of shape {self.shape}, "
                             f"got {t.dtype} {t.device} {tuple(t.shape)}")
        return t

    def empty(self):
        return torch.empty(self.shape, dtype=self.dtype, device=self.device)

    def to_device(self, a):
        return torch.as_tensor(a).to(device=self.device, dtype=self.dtype).contiguous()

    # -------------------------------------------------------------- entry points
    def prim_to_cons(self, w, out=None):
        w = self._arr(w, "w")
        q = self.empty() if out is None else self._arr(out, "out")
        self._check(self.lib.mfc_prim_to_cons(self.ctx, _ptr(w), _ptr(q), _stream()), "mfc_prim_to_cons")
        return q

    def cons_to_prim(self, q, out=None):
        q = self._arr(q)
        w = self.empty() if out is None else self._arr(out, "out")
        self._check(self.lib.mfc_cons_to_prim(self.ctx, _ptr(q), _ptr(w), _stream()), "mfc_cons_to_prim")
        return w

    def rhs(self, q, out=None):
        q = self._arr(q)
        r = self.empty() if out is None else self._arr(out, "out")
        self._check(self.lib.mfc_rhs(self.ctx, _ptr(q), _ptr(r), _stream()), "mfc_rhs")
        return r

    def max_signal(self, q):
        """Device scalar tensor holding max_cells sum_d (|u_d| + c)/dx_d."""
        q = self._arr(q)
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        self._check(self.lib.mfc_max_signal(self.ctx, _ptr(q), _ptr(out), _stream()), "mfc_max_signal")
        return out

    def set_grid(self, axis, faces):
        """Non-uniform grid along `axis`: its n + 1 face coordinates (host
        array), or None for uniform spacing again."""
        if faces is None:
            ptr = None
        else:
            self._faces_host = getattr(self, "_faces_host", {})
            a = (ctypes.c_double * len(faces))(*[float(v) for v in faces])
            self._faces_host[axis] = a
            ptr = ctypes.cast(a, ctypes.c_void_p)
        with torch.cuda.device(self.device):
            self._check(self.lib.mfc_set_grid(self.ctx, int(axis), ptr), "mfc_set_grid")

    def step(self, q, cfl=0.0, dt_fixed=0.0, t_remaining=0.0, dt_out=None):
        """Advance q in place by one SSP-RK3 step.  dt_out: optional device double tensor."""
        q = self._arr(q)
        if dt_out is not None and (dt_out.dtype != torch.float64 or dt_out.device != q.device or dt_out.numel() < 1):
            raise ValueError("dt_out must be a float64 tensor with at least one element on the solver's device")
        dp = ctypes.c_void_p(dt_out.data_ptr()) if dt_out is not None else ctypes.c_void_p()
        self._check(self.lib.mfc_step(self.ctx, _ptr(q), float(cfl), float(dt_fixed), float(t_remaining), dp,
                                      _stream()), "mfc_step")
        return q

    def conserved_sums(self, q):
        q = self._arr(q)
        out = torch.empty(self.neq, dtype=torch.float64, device=self.device)
        self._check(self.lib.mfc_conserved_sums(self.ctx, _ptr(q), _ptr(out), _stream()), "mfc_conserved_sums")
        return out

    # -------------------------------------------------------------- adjoint
    def _out(self, out, accumulate):
        if out is None:
            if accumulate:
                raise ValueError("accumulate needs an output tensor")
            return self.empty()
        return self._arr(out, "out")

    def rhs_vjp(self, q, rhs_bar, out=None, accumulate=False):
        """(dL/dq)^T rhs_bar at q."""
        q = self._arr(q)
        rb = self._arr(rhs_bar, "rhs_bar")
        o = self._out(out, accumulate)
        self._check(self.lib.mfc_rhs_vjp(self.ctx, _ptr(q), _ptr(rb), _ptr(o), int(accumulate), _stream()),
                    "mfc_rhs_vjp")
        return o

    def step_vjp(self, q_n, dt, qnp1_bar, out=None):
        """(dq^{n+1}/dq^n)^T qnp1_bar for a fixed-dt step from q_n."""
        q = self._arr(q_n, "q_n")
        b = self._arr(qnp1_bar, "qnp1_bar")
        o = self._out(out, False)
        self._check(self.lib.mfc_step_vjp(self.ctx, _ptr(q), float(dt), _ptr(b), _ptr(o), _stream()),
                    "mfc_step_vjp")
        return o

    def step_save_stages(self, q, dt, q1, q2):
        """Fixed-dt step of q in place; its two stage states are written to q1, q2."""
        qq = self._arr(q, "q")
        a = self._arr(q1, "q1")
        b = self._arr(q2, "q2")
        self._check(self.lib.mfc_step_save_stages(self.ctx, _ptr(qq), float(dt), _ptr(a), _ptr(b), _stream()),
                    "mfc_step_save_stages")
        return qq

    def step_vjp_stages(self, q_n, q1, q2, dt, qnp1_bar, out=None):
        """step_vjp with the step's stage states supplied (from step_save_stages)."""
        q = self._arr(q_n, "q_n")
        a = self._arr(q1, "q1")
        b = self._arr(q2, "q2")
        g = self._arr(qnp1_bar, "qnp1_bar")
        o = self._out(out, False)
        self._check(self.lib.mfc_step_vjp_stages(self.ctx, _ptr(q), _ptr(a), _ptr(b), float(dt), _ptr(g), _ptr(o),
                                                 _stream()), "mfc_step_vjp_stages")
        return o

    def cons_to_prim_vjp(self, q, w_bar, out=None, accumulate=False):
        q = self._arr(q)
        wb = self._arr(w_bar, "w_bar")
        o = self._out(out, accumulate)
        self._check(self.lib.mfc_cons_to_prim_vjp(self.ctx, _ptr(q), _ptr(wb), _ptr(o), int(accumulate),
                                                  _stream()), "mfc_cons_to_prim_vjp")
        return o

    def prim_to_cons_vjp(self, w, q_bar, out=None, accumulate=False):
        w = self._arr(w, "w")
        qb = self._arr(q_bar, "q_bar")
        o = self._out(out, accumulate)
        self._check(self.lib.mfc_prim_to_cons_vjp(self.ctx, _ptr(w), _ptr(qb), _ptr(o), int(accumulate),
                                                  _stream()), "mfc_prim_to_cons_vjp")
        return o

    def check(self):
        """Synchronize and raise MfcError(MFC_ERR_NONFINITE) if a bad state was met."""
        self._check(self.lib.mfc_check(self.ctx, _stream()), "mfc_check")

    def set_timing(self, enable=True):
        self._check(self.lib.mfc_set_timing(self.ctx, int(bool(enable))), "mfc_set_timing")

    def get_timing(self):
        """{kind: (ms_sum, count)} for kinds signal, x, y, z, vjp since the last call."""
        import numpy as np
        ms = np.zeros(5, dtype=np.float64)
        cnt = np.zeros(5, dtype=np.int64)
        self._check(self.lib.mfc_get_timing(self.ctx, ms.ctypes.data_as(ctypes.c_void_p),
                                            cnt.ctypes.data_as(ctypes.c_void_p)), "mfc_get_timing")
        names = ["signal", "pass_x", "pass_y", "pass_z", "vjp"]
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(names)}

    def run(self, q, nsteps, cfl=0.0, dt_fixed=0.0):
        for _ in range(nsteps):
            self.step(q, cfl=cfl, dt_fixed=dt_fixed)
        return q

    def run_to(self, q, t_end, cfl):
        """Advance to t_end with CFL steps clipped at t_end (reads dt back each step)."""
        dt = torch.zeros(1, dtype=torch.float64, device=self.device)
        t, k = 0.0, 0
        while t < t_end:
            self.step(q, cfl=cfl, t_remaining=t_end - t, dt_out=dt)
            t += float(dt.item())
            k += 1
        return k
