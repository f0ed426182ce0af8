"""Non-uniform grids (Sec. 4.2.2) in the HIP library, through the C ABI,
against the CPU FP64 oracle: RHS and 5 CFL steps at the FP64 parity bar,
equally spaced faces against the uniform path, signal speed and conservation
sums with per-cell widths, the FP32 form inside its float envelope, and the
argument checks of mfc_set_grid.
"""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import conservative_errors, grouped_errors
from test_gpu_parity import CASES, _variant_steps_match

pytestmark = pytest.mark.gpu
TOL = 1e-12
EPS32 = 2.0 ** -24


def _say(*a):
    print("[gpu-nonuniform]", *a, flush=True)


def _solver(case, precision="fp64"):
    from paper_2503_07953_amd.solver import Solver
    return Solver.from_case(case, precision=precision)


def _stretch(c, amps, seed=0):
    """Put case c on a stretched grid: per active axis the smooth map of
    workloads.stretched_faces with amplitude amps[d] (None: keep uniform),
    over the axis's own length n dx."""
    faces = []
    for d in range(3):
        a = amps[d] if d < len(amps) else None
        if d >= c.ndim or a is None:
            faces.append(None)
        else:
            faces.append(W.stretched_faces(c.n[d], c.n[d] * c.dx[d], a))
    c.faces = tuple(faces)
    return c


# (CASES index, stretch amplitude per axis)
NU_CASES = [
    (0, (0.5,)),                  # 1D one fluid, extrapolation
    (1, (-0.4,)),                 # 1D two fluids, slip walls
    (2, (0.3,)),                  # 1D two fluids, periodic
    (3, (0.5, -0.3)),             # 2D two fluids, extrapolation x slip wall
    (4, (None, 0.4)),             # 2D one fluid, y stretched only
    (5, (0.4, 0.4)),              # 2D two fluids, periodic
    (6, (0.3, -0.5, 0.4)),        # 3D two fluids, every boundary kind
    (7, (0.5, None, -0.3)),       # 3D one fluid
    (8, (0.2, 0.2, 0.2)),         # 3D, three cells per axis
]


@pytest.mark.parametrize("case,amps", NU_CASES)
def test_nonuniform_rhs_and_steps_match_oracle(case, amps):
    nd, n, nf, bc = CASES[case]
    _say("nonuniform", nd, n, nf, bc, amps)
    c = W.random_case(nd, n, nf=nf, seed=1000 + case, bc=bc, speed=400.0 if nf == 1 else 150.0)
    _stretch(c, amps)
    _variant_steps_match(c, nf, nd)


@pytest.mark.parametrize("n", [(63, 9), (125, 6), (5, 7, 4), (63, 5, 3)])
def test_ragged_x_tiles_match_oracle(n):
    """x extents that leave the last x tile of a row with one output (63 =
    62 + 1, 125 = 2 * 62 + 1) or make a single short tile (5), on grids
    stretched along x and uniform: the lanes past the grid in that tile take
    part in the lane exchange but read nothing outside the grid or the
    stretched-grid tables."""
    nd = len(n)
    bc = (W.EXTRAP, W.SLIPWALL, W.PERIODIC)[:nd]
    for amps in ((0.4,) + (None,) * (nd - 1), None):
        # a uniform mixture with a pressure jump (a bubble does not fit these
        # thin domains); its exact alpha RHS is zero, so the RHS is compared
        # on the flux scale
        c = W.random_case(nd, n, nf=2, seed=1200 + n[0], bc=bc, speed=150.0, pressure_jump=2.0, interface=False)
        if amps is not None:
            _stretch(c, amps)
        _say("ragged x", n, "stretched" if amps else "uniform")
        _variant_steps_match(c, 2, nd, flux_scale=True)


@pytest.mark.parametrize("name", ["shock_cylinder_64", "bubble_cloud_48"])
def test_nonuniform_two_fluid_flows_match_oracle(name):
    """The benchmark flows on centre-clustered grids (width ratio 3 and 2)."""
    if name.startswith("shock"):
        c = _stretch(W.shock_cylinder(64), (-0.5, -0.5))
        zero = (1,)
    else:
        c = _stretch(W.bubble_cloud(48, nbub=4), (-0.33, -0.33, -0.33))
        zero = (1, 2)
    _say("nonuniform flow", name)
    _variant_steps_match(c, 2, c.ndim, flux_scale=True, zero_mom=zero)


def test_equally_spaced_faces_match_the_uniform_path():
    """Face coordinates at equal spacing give the uniform kernels' RHS and
    steps to rounding (different kernels and arithmetic: tabulated
    coefficients instead of constants)."""
    c = W.random_case(3, (40, 36, 30), nf=2, seed=1011, bc=(W.EXTRAP, W.SLIPWALL, W.PERIODIC), speed=150.0)
    Su = _solver(c)
    qu = Su.prim_to_cons(Su.to_device(c.w))
    ru = Su.rhs(qu).cpu().numpy()
    c.faces = tuple(np.arange(c.n[d] + 1) * c.dx[d] for d in range(3))
    Sn = _solver(c)
    qn = Sn.prim_to_cons(Sn.to_device(c.w))
    rn = Sn.rhs(qn).cpu().numpy()
    Su.run(qu, 3, cfl=0.5)
    Sn.run(qn, 3, cfl=0.5)
    Su.check()
    Sn.check()
    e1 = conservative_errors(rn, ru, 2, 3)
    e2 = conservative_errors(qn.cpu().numpy(), qu.cpu().numpy(), 2, 3)
    _say("equal spacing vs uniform", e1, e2)
    assert e1.max() <= 1e-12 and e2.max() <= 1e-12, (e1, e2)
    # and back to uniform spacing: the uniform kernels again, bitwise
    for d in range(3):
        Sn.set_grid(d, None)
    q2 = Sn.prim_to_cons(Sn.to_device(c.w))
    assert np.array_equal(Sn.rhs(q2).cpu().numpy(), ru)


def test_nonuniform_signal_and_sums_match_oracle():
    c = _stretch(W.random_case(3, (40, 36, 30), nf=2, seed=1012, bc=(W.EXTRAP, W.SLIPWALL, W.PERIODIC),
                               speed=300.0), (0.5, -0.4, 0.3))
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    S = _solver(c)
    qd = S.to_device(q)
    s = S.max_signal(qd).item()
    assert abs(s / O.max_signal(q) - 1) <= 1e-13
    sums = S.conserved_sums(qd).cpu().numpy()
    ref = O.conserved_sums(q)
    assert np.all(np.abs(sums - ref) <= 1e-13 * np.abs(ref) + 1e-300), (sums, ref)


@pytest.mark.parametrize("kind", ["random", "bubbles"])
def test_fp32_nonuniform_within_float_envelope(kind):
    """The FP32 form on a stretched grid (float coefficients) against the FP64
    oracle, inside the float envelope of the uniform FP32 tests with the
    smallest width in the momentum bound."""
    if kind == "bubbles":
        c = _stretch(W.bubble_cloud(64, nbub=6, slab=8), (-0.3, -0.3, -0.3))
        nsteps = 20
    else:
        c = _stretch(W.random_case(3, (40, 36, 30), nf=2, seed=5, bc=(W.EXTRAP, W.SLIPWALL, W.PERIODIC),
                                   speed=100.0), (0.4, -0.4, 0.3))
        nsteps = 10
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    dts = O.run(q, nsteps, cfl=0.5)
    S = _solver(c, precision="fp32")
    q32 = S.prim_to_cons(S.to_device(c.w))
    S.run(q32, nsteps, cfl=0.5)
    S.check()
    err = grouped_errors(q32.double().cpu().numpy(), q, 2, 3)
    stages = 3 * nsteps
    hmin = min(np.diff(f).min() for f in c.faces if f is not None)
    gam_w = 1.0 / (c.gamma[0] - 1.0)
    mom = np.sqrt((q[2:5] ** 2).sum(axis=0)).max()
    bound = np.full(6, 4 * stages * EPS32)
    bound[2] = max(4 * stages * 3 * EPS32 * np.abs(q[5]).max() * (dts.max() / hmin) / (gam_w * mom), bound[0])
    _say(kind, "errors", err, "bounds", bound)
    assert np.all(err <= bound), (err, bound)


def test_set_grid_argument_checks():
    from paper_2503_07953_amd import _lib as L
    c = W.random_case(2, (20, 16), nf=2, seed=1013, bc=(W.EXTRAP, W.EXTRAP), speed=100.0)
    S = _solver(c)
    lib = S.lib
    good = (ctypes.c_double * 21)(*np.linspace(0.0, 1.0, 21))
    bad = (ctypes.c_double * 21)(*np.linspace(0.0, 1.0, 21))
    bad[7] = bad[6]
    assert lib.mfc_set_grid(S.ctx, 0, ctypes.cast(bad, ctypes.c_void_p)) == L.MFC_ERR_ARG
    assert lib.mfc_set_grid(S.ctx, 2, ctypes.cast(good, ctypes.c_void_p)) == L.MFC_ERR_ARG
    assert lib.mfc_set_grid(S.ctx, -1, ctypes.cast(good, ctypes.c_void_p)) == L.MFC_ERR_ARG
    assert lib.mfc_set_grid(None, 0, ctypes.cast(good, ctypes.c_void_p)) == L.MFC_ERR_ARG
    assert lib.mfc_set_grid(S.ctx, 0, ctypes.cast(good, ctypes.c_void_p)) == L.MFC_OK
    # other reconstruction weights take no grid
    c.weno_variant = 1
    Sz = _solver(c)
    assert Sz.lib.mfc_set_grid(Sz.ctx, 0, ctypes.cast(good, ctypes.c_void_p)) == L.MFC_ERR_UNSUPPORTED


# ---------------------------------------------------------------------------
# Adjoint on non-uniform grids (no torch reference covers them: checked by the
# dot-product identity against forward differences of the HIP RHS, by equally
# spaced faces against the uniform adjoint, and through a 100-step rollout
# against central differences)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nd,amps", [(2, (0.5, -0.4)), (3, (0.3, -0.3, 0.4)), (1, (0.6,))])
def test_nonuniform_rhs_vjp_dot_product_against_forward_differences(nd, amps):
    """<L(q+hv) - L(q-hv), lam>/2h (Richardson over h, 2h) equals <v, L^T lam>,
    to 1e-5 of |J v|_2: with lam ~ N(0, 1) that is the typical size of the dot
    product, which a draw of lam can cancel to a small fraction of it (where a
    bar relative to the dot product itself measures the cancellation)."""
    import torch
    n = {1: (80,), 2: (48, 40), 3: (24, 20, 18)}[nd]
    bc = {1: (W.SLIPWALL,), 2: (W.EXTRAP, W.SLIPWALL), 3: (W.EXTRAP, W.SLIPWALL, W.PERIODIC)}[nd]
    c = _stretch(W.random_case(nd, n, nf=2, seed=1020 + nd, bc=bc, speed=50.0, pressure_jump=1.0,
                               interface=False), amps)
    S = _solver(c)
    q = S.prim_to_cons(S.to_device(c.w))
    rng = np.random.default_rng(0)
    for _ in range(2):
        v = torch.from_numpy(np.stack([W._smooth_field(rng, q.shape[1:], nd) for _ in range(q.shape[0])])).cuda()
        v = v * q.abs()
        lam = torch.from_numpy(rng.normal(size=q.shape)).cuda()
        lhs = float((S.rhs_vjp(q, lam) * v).sum())
        est = []
        for h in (4e-9, 2e-9):
            fd = (S.rhs((q + h * v).contiguous()) - S.rhs((q - h * v).contiguous())) / (2 * h)
            est.append(float((fd * lam).sum()))
        scale = float(fd.norm())
        rich = (4 * est[1] - est[0]) / 3
        _say("dot product", nd, lhs, rich, "|Jv|", scale, abs(rich - lhs) / scale)
        assert abs(rich - lhs) <= 1e-5 * scale, (lhs, est, scale)


def test_nonuniform_vjp_on_equally_spaced_faces_matches_uniform():
    """Equally spaced faces: the tabulated adjoint equals the uniform one to
    within 10x the uniform adjoint's own spread under one-ulp changes of q
    (the two differ in arithmetic, and WENO weight derivatives amplify
    rounding), and never worse than 1e-7."""
    import torch
    from helpers import field_errors
    c = W.random_case(2, (40, 36), nf=2, seed=1024, bc=(W.EXTRAP, W.SLIPWALL), speed=150.0)
    Su = _solver(c)
    q = Su.prim_to_cons(Su.to_device(c.w))
    lam = torch.from_numpy(np.random.default_rng(1).normal(size=q.shape)).cuda()
    ref = Su.rhs_vjp(q, lam).cpu().numpy()
    rng = np.random.default_rng(5)
    spread = np.zeros(c.neq)
    eps = np.finfo(np.float64).eps
    for _ in range(3):
        qp = q * (1.0 + torch.from_numpy(rng.choice([-1.0, 0.0, 1.0], size=q.shape) * eps).cuda())
        spread = np.maximum(spread, field_errors(Su.rhs_vjp(qp.contiguous(), lam).cpu().numpy(), ref))
    c.faces = tuple(np.arange(c.n[d] + 1) * c.dx[d] for d in range(2)) + (None,)
    Sn = _solver(c)
    got = Sn.rhs_vjp(q, lam).cpu().numpy()
    err = field_errors(got, ref)
    _say("equal spacing vjp", err, "spread", spread)
    assert np.all(err <= np.minimum(np.maximum(10 * spread, 1e-11), 1e-7)), (err, spread)


@pytest.mark.timeout(600)
@pytest.mark.slow
def test_nonuniform_rollout_adjoint_matches_central_differences():
    """The smooth air-water mixture (every indicator far above eps) at 128^2 on
    a grid stretched along x (smooth periodic map, amplitude 0.4), 100
    frozen-dt steps with checkpoints every 20: <grad J, v> of the HIP adjoint
    against central differences of the HIP forward on 8 seeded smooth
    directions, to 1e-6 relative."""
    from test_gpu_adjoint import _fd_projections
    c = W.smooth_mixture(128, steps=100)
    c.faces = (W.stretched_faces(128, 1.0, 0.4), None, None)
    res = _fd_projections(c, 64, 1e-3, 8, seed=33)
    rel = np.abs(res[:, 1] - res[:, 0]) / np.abs(res[:, 0])
    _say("stretched smooth mixture worst relative difference", rel.max())
    assert rel.max() <= 1e-6
