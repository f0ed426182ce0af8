"""The allocation-free step (mfc_step_static) against mfc_step, through the C ABI.

Both entry points run the same kernels, so the states after each step must
agree bit for bit.  Two problems in a row, the second smaller than the first,
show that a call depends on nothing the previous call left in the static
scratch.  CFL steps (dt formed on the device) and fixed-dt steps, FP64 and the
FP32 form.
"""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[no-alloc]", *a, flush=True)


def _static_steps(S, q, nsteps, cfl, dt_fixed):
    """Advance the device tensor q in place through mfc_step_static."""
    lib = S.lib
    flag = torch.zeros(1, dtype=torch.int32, device=q.device)
    dts = torch.zeros(nsteps, dtype=torch.float64, device=q.device)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for k in range(nsteps):
        rc = lib.mfc_step_static(ctypes.byref(S.prob), ctypes.c_void_p(q.data_ptr()), float(cfl), float(dt_fixed),
                                 0.0, ctypes.c_void_p(dts[k:].data_ptr()), ctypes.c_void_p(flag.data_ptr()), stream)
        assert rc == 0, rc
    torch.cuda.synchronize()
    return dts.cpu().numpy(), int(flag.item())


def _context_steps(S, q, nsteps, cfl, dt_fixed):
    dts = torch.zeros(nsteps, dtype=torch.float64, device=q.device)
    for k in range(nsteps):
        S.step(q, cfl=cfl, dt_fixed=dt_fixed, dt_out=dts[k:k + 1])
    S.check()
    return dts.cpu().numpy()


CASES = [
    # (case builder, precision, cfl, dt_fixed); each pair runs larger, then smaller
    ("bubble_cloud_48_then_shock_cylinder_40", "fp64"),
    ("bubble_cloud_48_then_shock_cylinder_40", "fp32"),
]


def _pair():
    big = W.bubble_cloud(48, nbub=4)
    small = W.shock_cylinder(40, steps=3)
    return big, small


@pytest.mark.parametrize("name,precision", CASES)
def test_static_step_equals_context_step_twice(name, precision):
    from paper_2503_07953_amd.solver import Solver
    for case, cfl, dt_fixed, nsteps in zip(_pair(), (0.5, 0.0), (0.0, 2e-8), (3, 2)):
        _say(name, precision, case.ncell, "cells", "cfl" if cfl else "fixed dt", nsteps, "steps")
        S = Solver.from_case(case, precision=precision)
        q0 = S.prim_to_cons(S.to_device(case.w))
        qa = q0.clone()
        qb = q0.clone()
        dta, flag = _static_steps(S, qa, nsteps, cfl, dt_fixed)
        dtb = _context_steps(S, qb, nsteps, cfl, dt_fixed)
        assert flag == 0
        assert np.array_equal(dta, dtb), (dta, dtb)
        assert torch.equal(qa, qb), (qa - qb).abs().max().item()
        assert not torch.equal(qa, q0)
