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
from helpers import grouped_errors

pytestmark = pytest.mark.gpu
EPS32 = 2.0 ** -24


def _say(*a):
    print("[gpu-fp32]", *a, flush=True)


def _envelope(c, q, dts, nsteps):
    stages = 3 * nsteps
    gam_w = 1.0 / (c.gamma[0] - 1.0)
    mom = np.sqrt((q[2:5] ** 2).sum(axis=0)).max()
    bound_mom = 4 * stages * 3 * EPS32 * np.abs(q[5]).max() * (dts.max() / c.dx[0]) / (gam_w * mom)
    bound = np.full(6, 4 * stages * EPS32)
    bound[2] = max(bound_mom, 4 * stages * EPS32)
    return bound


@pytest.mark.parametrize("kind", ["bubbles", "random", "random-weno-z", "random-weno-m", "random-hll",
                                  "random-low-mach", "random-weno-m-hll-low-mach"])
def test_fp32_form_within_float_envelope(kind):
    from paper_2503_07953_amd.solver import Solver
    if kind == "bubbles":
        c = W.bubble_cloud(64, nbub=6, slab=8)
        nsteps = 20
    else:
        c = W.random_case(3, (40, 36, 30), nf=2, seed=5, bc=(W.EXTRAP, W.SLIPWALL, W.PERIODIC), speed=100.0)
        nsteps = 10
        c.weno_variant = 1 if "weno-z" in kind else 3 if "weno-m" in kind else 0
        c.riemann = 1 if "hll" in kind else 0
        c.low_mach = 1 if "low-mach" in kind else 0
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    dts = O.run(q, nsteps, cfl=0.5)
    S = Solver.from_case(c, precision="fp32")
    q32 = S.prim_to_cons(S.to_device(c.w))
    S.run(q32, nsteps, cfl=0.5)
    S.check()
    got = q32.double().cpu().numpy()
    err = grouped_errors(got, q, 2, 3)
    bound = _envelope(c, q, dts, nsteps)
    _say(kind, "errors", err, "bounds", bound)
    assert np.all(err <= bound), (err, bound)


def test_fp32_teno_bubbles_within_envelope_but_at_flips():
    """TENO5 (Sec. 4.2.2) keeps a candidate stencil when its share of the
    weights is at least C_T: a step function of the data.  Float storage puts a
    pressure noise of eps32 |E| / Gamma_w on water, and where a share lies
    within that noise of C_T the float form keeps a stencil the FP64 oracle
    drops (or the reverse), moving that face flux by a fraction of the local
    variation rather than by rounding.  Such flips are local: every field must
    meet the float envelope outside at most 1% of the cells."""
    from paper_2503_07953_amd.solver import Solver
    c = W.bubble_cloud(64, nbub=6, slab=8)
    c.weno_variant = 2
    nsteps = 20
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    dts = O.run(q, nsteps, cfl=0.5)
    S = Solver.from_case(c, precision="fp32")
    q32 = S.prim_to_cons(S.to_device(c.w))
    S.run(q32, nsteps, cfl=0.5)
    S.check()
    got = q32.double().cpu().numpy()
    bound = _envelope(c, q, dts, nsteps)
    err = grouped_errors(got, q, 2, 3)
    # per-cell errors on each field's scale (momentum as one vector)
    d = np.abs(got - q)
    scale = np.abs(q).reshape(q.shape[0], -1).max(axis=1)
    cell = [d[0] / scale[0], d[1] / scale[1],
            np.sqrt((d[2:5] ** 2).sum(axis=0)) / np.sqrt((q[2:5] ** 2).sum(axis=0)).max(),
            d[5] / scale[5], d[6] / scale[6], d[7] / scale[7]]
    over = np.zeros(q.shape[1:], dtype=bool)
    for f in range(6):
        over |= cell[f] > bound[f]
    _say("bubbles-teno errors", err, "bounds", bound, "cells over", int(over.sum()), "of", over.size)
    assert np.isfinite(got).all()
    assert over.sum() <= 0.01 * over.size


def test_fp32_teno_rhs_on_rough_data():
    """TENO5 keeps a candidate stencil when its share gamma_k / sum(gamma) is
    at least C_T: a step function of the data.  On random data a share can lie
    within float rounding of C_T; there the float form keeps a stencil the
    FP64 oracle drops (or the reverse), and the face flux moves by a fraction
    of the local variation.  Every other face agrees on the flux scale.  A
    float emulation of the cut-off on this state flips 2 of 2.75e6 choices,
    so the test allows flips to spoil at most 0.1% of the cells and requires
    the rest to meet the flux-scale tolerance of the WENO5-JS form."""
    from paper_2503_07953_amd.solver import Solver
    c = W.random_case(3, (40, 36, 30), nf=2, seed=5, bc=(W.EXTRAP, W.SLIPWALL, W.PERIODIC), speed=100.0)
    c.weno_variant = 2
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    ref = O.rhs(q)
    S = Solver.from_case(c, precision="fp32")
    r = S.rhs(S.to_device(q)).double().cpu().numpy()
    S.check()
    assert np.isfinite(r).all()
    smax = O.max_signal(q)
    scale = np.abs(q).reshape(q.shape[0], -1).max(axis=1) * smax
    cell_err = (np.abs(r - ref) / scale[:, None, None, None]).max(axis=0)
    bad = int((cell_err > 1e-4).sum())
    _say("teno rough rhs: cells above 1e-4", bad, "of", cell_err.size, "max", cell_err.max())
    assert bad <= 1e-3 * cell_err.size


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


@pytest.mark.parametrize("variant", [0, 3])
def test_fp32_gigapascal_jump_stays_finite_and_tracks_fp64(variant):
    """A 4.5 GPa pressure jump in water spread over two cells: the squared
    smoothness indicators of the pressure row exceed the float range, so the
    FP32 weights are formed from the ratios s_min / s_k.  The FP32 RHS must be
    finite and agree with the FP64 oracle on the flux scale (1e-4, as for the
    other FP32 RHS checks; the momentum on max p / dx, since the fluid starts
    at rest), and five CFL steps must stay finite and within
    1e-4 of the oracle per field (WENO5-JS and WENO5-M)."""
    from helpers import rate_errors
    from paper_2503_07953_amd.solver import Solver
    n = 128
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    p = np.where(x < 0.5, 1e5, 4.5e9)
    p[n // 2 - 1] = 1e5 + (4.5e9 - 1e5) / 3
    p[n // 2] = 1e5 + 2 * (4.5e9 - 1e5) / 3
    aw = np.full(n, 1.0 - W.ALPHA_FLOOR)
    aw[: n // 4] = W.ALPHA_FLOOR  # an air column as well
    w = W._two_fluid_w(aw, 1000.0, 1.0, [np.zeros(n)], p).reshape(6, 1, 1, n)
    c = W.Case("gpa_jump", 1, (n, 1, 1), 2, (dx, 1.0, 1.0), (6.12, 1.4), (3.43e8, 0.0),
               (W.EXTRAP,) * 3, (W.EXTRAP,) * 3, w)
    c.weno_variant = variant
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    ref = O.rhs(q)
    S = Solver.from_case(c, precision="fp32")
    r = S.rhs(S.to_device(q)).double().cpu().numpy()
    S.check()
    assert np.isfinite(r).all()
    # the fluid starts at rest: the momentum rate is set by the pressure jump
    err = rate_errors(r, ref, q, O.max_signal(q), 2, 1, mom_rate=p.max() / dx)
    _say("GPa jump rhs errors", variant, err)
    assert err.max() <= 1e-4, err
    q32 = S.to_device(q)
    S.run(q32, 5, cfl=0.5)
    S.check()
    O.run(q, 5, cfl=0.5)
    got = q32.double().cpu().numpy()
    assert np.isfinite(got).all()
    e = grouped_errors(got, q, 2, 1)
    _say("GPa jump 5-step errors", variant, e)
    assert e.max() <= 1e-4, e
