"""The FP32 form (float storage and WENO/HLLC arithmetic, double pressure
inversion, wave speeds, stage update and reductions) against the FP64 oracle.

Error envelope.  Every stage rounds the stored state to float (relative
eps32 = 2^-24), so after S = 3N stages a field that is not formed by
cancellation stays within ~S * eps32 of the FP64 result (bound used: 4 S eps32
of the field maximum).  Momentum is different: rho E of water at 1 bar is ~4e8
J/m^3 of which only Gamma p ~ 2e4 is pressure, so the float rounding of rho E is
a pressure error of eps32 |E| / Gamma_w per stage, which drives the momentum
by dt/dx per axis: bound 4 S D eps32 max|E| (dt/dx) / (Gamma_w max|rho u|) on the
momentum vector.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from helpers import conservative_errors

pytestmark = pytest.mark.gpu
EPS32 = 2.0 ** -24


def _say(*a):
    print("[gpu-fp32]", *a, flush=True)


@pytest.mark.parametrize("kind", ["bubbles", "random", "random-weno-z"])
def test_fp32_form_within_float_envelope(kind):
    from paper_2503_07953_amd.solver import Solver
    if kind == "bubbles":
        c = W.bubble_cloud(64, nbub=6, slab=8)
        nsteps = 20
    else:
        c = W.random_case(3, (40, 36, 30), nf=2, seed=5, bc=(W.EXTRAP, W.SLIPWALL, W.PERIODIC), speed=100.0)
        nsteps = 10
        c.weno_variant = 1 if kind.endswith("weno-z") else 0
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    dts = O.run(q, nsteps, cfl=0.5)
    S = Solver.from_case(c, precision="fp32")
    q32 = S.prim_to_cons(S.to_device(c.w))
    S.run(q32, nsteps, cfl=0.5)
    S.check()
    got = q32.double().cpu().numpy()
    err = conservative_errors(got, q, 2, 3)
    stages = 3 * nsteps
    gam_w = 1.0 / (c.gamma[0] - 1.0)
    mom = np.sqrt((q[2:5] ** 2).sum(axis=0)).max()
    bound_mom = 4 * stages * 3 * EPS32 * np.abs(q[5]).max() * (dts.max() / c.dx[0]) / (gam_w * mom)
    bound = np.full(err.shape, 4 * stages * EPS32)
    bound[2] = max(bound_mom, 4 * stages * EPS32)
    _say(kind, "errors", err, "bounds", bound)
    assert np.all(err <= bound), (err, bound)


def test_fp32_rhs_and_conversions_track_fp64():
    from paper_2503_07953_amd.solver import Solver
    c = W.random_case(2, (70, 50), nf=2, seed=8, bc=(W.EXTRAP, W.SLIPWALL), speed=150.0)
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    ref = O.rhs(q)
    S = Solver.from_case(c, precision="fp32")
    q32 = S.to_device(q)
    r = S.rhs(q32).double().cpu().numpy()
    S.check()
    # float rounding of the state alone moves the pressure of water by
    # eps32 |E| / Gamma, so the RHS is compared on the flux scale
    from helpers import rate_errors
    err = rate_errors(r, ref, q, O.max_signal(q), 2, 2)
    _say("rhs errors", err)
    assert err.max() <= 1e-4
    s64 = O.max_signal(q)
    s32 = S.max_signal(q32).item()
    assert abs(s32 / s64 - 1) <= 1e-6
