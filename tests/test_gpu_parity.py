"""HIP path (through the C ABI) against the CPU FP64 oracle on the same seeded inputs.

Bar: per conservative field (each partial density, the momentum vector, the
energy, each volume fraction), max|gpu - oracle| / max|oracle| <= 1e-12 (FP64).
Sizes span several tiles with ragged tails on every axis; full-size
configurations are checked on sampled cells or after a full step.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from helpers import EPS, conservative_errors, field_errors, rate_errors

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _solver(case, precision="fp64"):
    from paper_2503_07953_amd.solver import Solver
    return Solver.from_case(case, precision=precision)


def _say(*a):
    print("[gpu-parity]", *a, flush=True)


CASES = [
    # (ndim, n, nf, bc)
    (1, (200,), 1, (W.EXTRAP,)),
    (1, (131,), 2, (W.SLIPWALL,)),
    (1, (64,), 2, (W.PERIODIC,)),
    (2, (150, 70), 2, (W.EXTRAP, W.SLIPWALL)),
    (2, (64, 93), 1, (W.PERIODIC, W.EXTRAP)),
    (2, (37, 41), 2, (W.PERIODIC, W.PERIODIC)),
    (3, (70, 33, 29), 2, (W.SLIPWALL, W.EXTRAP, W.PERIODIC)),
    (3, (40, 40, 40), 1, (W.EXTRAP, W.PERIODIC, W.SLIPWALL)),
    (3, (3, 3, 3), 2, (W.EXTRAP, W.SLIPWALL, W.PERIODIC)),
]


@pytest.mark.parametrize("nd,n,nf,bc", CASES)
def test_rhs_matches_oracle(nd, n, nf, bc):
    _say("rhs", nd, n, nf, bc)
    c = W.random_case(nd, n, nf=nf, seed=100 + nd, bc=bc, speed=400.0 if nf == 1 else 200.0)
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    ref = O.rhs(q)
    S = _solver(c)
    qd = S.to_device(q)
    got = S.rhs(qd).cpu().numpy()
    S.check()
    err = conservative_errors(got, ref, nf, nd)
    assert err.max() <= TOL, err


@pytest.mark.parametrize("nd,n,nf,bc", CASES[:7])
def test_prim_cons_and_signal_match_oracle(nd, n, nf, bc):
    c = W.random_case(nd, n, nf=nf, seed=200 + nd, bc=bc)
    O = oracle.Oracle(c)
    S = _solver(c)
    q_ref = O.prim_to_cons(c.w)
    q = S.prim_to_cons(S.to_device(c.w)).cpu().numpy()
    assert conservative_errors(q, q_ref, nf, nd).max() <= 2 * EPS
    w = S.cons_to_prim(S.to_device(q_ref)).cpu().numpy()
    w_ref = O.cons_to_prim(q_ref)
    # velocities and copied rows: a few ulp; pressure: p = (E - ke - Pi)/Gamma
    # loses the digits that cancel, so its bound is 8 eps (|E| + ke + Pi)/Gamma
    prow = nf + nd
    for v in range(c.neq):
        if v != prow:
            assert np.all(np.abs(w[v] - w_ref[v]) <= 4 * EPS * np.abs(w_ref[v]) + 1e-300)
    rho = w_ref[:nf].sum(axis=0)
    ke = 0.5 * rho * (w_ref[nf:nf + nd] ** 2).sum(axis=0)
    G = [1.0 / (g - 1.0) for g in c.gamma]
    Pc = [g * pi / (g - 1.0) for g, pi in zip(c.gamma, c.pi_inf)]
    if nf == 2:
        Gam = w_ref[prow + 1] * G[0] + w_ref[prow + 2] * G[1]
        Pi = w_ref[prow + 1] * Pc[0] + w_ref[prow + 2] * Pc[1]
    else:
        Gam, Pi = G[0], Pc[0]
    bound = 8 * EPS * (np.abs(q_ref[prow]) + ke + np.abs(Pi)) / Gam
    assert np.all(np.abs(w[prow] - w_ref[prow]) <= bound)
    s = S.max_signal(S.to_device(q_ref)).item()
    assert abs(s / O.max_signal(q_ref) - 1) <= 1e-14
    sums = S.conserved_sums(S.to_device(q_ref)).cpu().numpy()
    sums_ref = O.conserved_sums(q_ref)
    scale = np.abs(q_ref).sum(axis=(1, 2, 3)) * np.prod([c.dx[d] for d in range(nd)])
    assert np.all(np.abs(sums - sums_ref) <= 1e-13 * scale)


@pytest.mark.parametrize("nd,n,nf,bc,nsteps", [
    (2, (96, 80), 2, (W.EXTRAP, W.SLIPWALL), 20),
    (3, (40, 36, 30), 2, (W.PERIODIC, W.EXTRAP, W.SLIPWALL), 5),
    (1, (300,), 1, (W.EXTRAP,), 50),
])
def test_cfl_steps_match_oracle(nd, n, nf, bc, nsteps):
    _say("steps", nd, n, nf, bc, nsteps)
    c = W.random_case(nd, n, nf=nf, seed=300 + nd, bc=bc, speed=150.0)
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    S = _solver(c)
    qd = S.to_device(q)
    dts = O.run(q, nsteps, cfl=0.5)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    gdts = []
    for _ in range(nsteps):
        S.step(qd, cfl=0.5, dt_out=dt)
        gdts.append(dt.item())
    S.check()
    assert np.allclose(gdts, dts, rtol=1e-13, atol=0)
    err = conservative_errors(qd.cpu().numpy(), q, nf, nd)
    assert err.max() <= TOL, err


def _quiet_components(c):
    """Momentum components that stay zero in exact arithmetic over the first
    few steps of the small benchmark flows: the planar shock (or pulse) has not
    reached the air inclusions, which sit at rest in uniform pressure, so no
    momentum arises across the wave (y in 2D, y and z in 3D)."""
    return (1,) if c.ndim == 2 else (1, 2)


def _variant_steps_match(c, nf, nd, flux_scale=False, zero_mom=()):
    """flux_scale: compare the RHS on the flux scale of each field (flows at
    rest in uniform pressure, where the exact alpha RHS is zero and both sides
    return rounding noise), else on the scale of the RHS itself.  zero_mom:
    momentum components that are zero in exact arithmetic over the 5 steps
    (measured on the momentum-vector scale)."""
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    S = _solver(c)
    qd = S.to_device(q)
    r, ref = S.rhs(qd).cpu().numpy(), O.rhs(q)
    if flux_scale:
        err = rate_errors(r, ref, q, O.max_signal(q), nf, nd)
    else:
        err = conservative_errors(r, ref, nf, nd)
    assert err.max() <= TOL, err
    # TENO5 keeps a stencil when its share reaches C_T, a step function of the
    # data: somewhere in a flow a one-ulp change of the state flips a choice,
    # so two correct FP64 runs agree only to the oracle's own spread under such
    # a change (about 1e-15 for WENO5-JS / Z, 4e-11 on the bubble cloud's
    # momentum under TENO5).  The bar is the larger of TOL and 4x that spread.
    rng = np.random.default_rng(17)
    q_ref = q.copy()
    O.run(q_ref, 5, cfl=0.5)
    spread = np.zeros(c.neq)
    for _ in range(2):
        qp = q * (1.0 + rng.choice([-1.0, 0.0, 1.0], size=q.shape) * EPS)
        O.run(qp, 5, cfl=0.5)
        spread = np.maximum(spread, conservative_errors(qp, q_ref, nf, nd, zero_mom))
    bar = np.maximum(TOL, 4 * spread)
    dts = O.run(q, 5, cfl=0.5)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    gdts = []
    for _ in range(5):
        S.step(qd, cfl=0.5, dt_out=dt)
        gdts.append(dt.item())
    S.check()
    assert np.allclose(gdts, dts, rtol=1e-13, atol=0)
    err = conservative_errors(qd.cpu().numpy(), q, nf, nd, zero_mom)
    _say("errors", err, "bar", bar)
    assert np.all(err <= bar), (err, bar)


@pytest.mark.parametrize("nd,n,nf,bc,variant", [CASES[0] + (1,), CASES[3] + (1,), CASES[6] + (1,), CASES[7] + (1,),
                                                CASES[0] + (2,), CASES[7] + (2,),
                                                CASES[0] + (3,), CASES[3] + (3,), CASES[6] + (3,), CASES[7] + (3,)])
def test_weno_variants_rhs_and_steps_match_oracle(nd, n, nf, bc, variant):
    """WENO5-Z (1), TENO5 (2) of Sec. 4.2.2 and WENO5-M (3, the mapped
    weights of Sec. 3.2.1) through the same kernels, on
    white-noise states.  TENO5 is run on the one-fluid ones only: on two-fluid
    white noise its three stencils are equally rough, it keeps all of them and
    the linear five-point scheme makes negative face densities across the
    random density jumps (test_teno_rough_two_fluid_flagged_on_both_sides)."""
    _say("variant", variant, nd, n, nf, bc)
    c = W.random_case(nd, n, nf=nf, seed=500 + nd, bc=bc, speed=400.0 if nf == 1 else 150.0)
    c.weno_variant = variant
    _variant_steps_match(c, nf, nd)


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("name", ["shock-cylinder-96", "bubble-cloud-64"])
def test_weno_variants_two_fluid_flows_match_oracle(name, variant):
    """The variants on the two-fluid flows of the benchmarks at small size."""
    _say("variant", variant, name)
    if name.startswith("shock"):
        c = W.shock_cylinder(96)
    else:
        c = W.bubble_cloud(64, nbub=6, slab=8)
    c.weno_variant = variant
    _variant_steps_match(c, 2, c.ndim, flux_scale=True, zero_mom=_quiet_components(c))


@pytest.mark.parametrize("case", [CASES[0], CASES[1], CASES[3], CASES[5], CASES[6], CASES[7]])
def test_hll_rhs_and_steps_match_oracle(case):
    """The HLL face solver (Sec. 3.2.2) through the same kernels."""
    nd, n, nf, bc = case
    _say("hll", nd, n, nf, bc)
    c = W.random_case(nd, n, nf=nf, seed=600 + nd, bc=bc, speed=400.0 if nf == 1 else 150.0)
    c.riemann = 1
    _variant_steps_match(c, nf, nd)


@pytest.mark.parametrize("name", ["shock-cylinder-96", "bubble-cloud-64"])
def test_hll_two_fluid_flows_match_oracle(name):
    _say("hll", name)
    c = W.shock_cylinder(96) if name.startswith("shock") else W.bubble_cloud(64, nbub=6, slab=8)
    c.riemann = 1
    _variant_steps_match(c, 2, c.ndim, flux_scale=True, zero_mom=_quiet_components(c))


def test_hll_differs_from_hllc():
    c = W.random_case(2, (40, 30), nf=2, seed=9, bc=(W.EXTRAP, W.PERIODIC))
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    S0 = _solver(c)
    r0 = S0.rhs(S0.to_device(q)).cpu().numpy()
    c.riemann = 1
    S1 = _solver(c)
    qd = S1.to_device(q)
    r1 = S1.rhs(qd).cpu().numpy()
    assert not np.array_equal(r0, r1)


@pytest.mark.slow
def test_hll_bubble_cloud_breaks_down_at_the_oracles_step():
    """Under HLL (with its alpha reading) the 100 bar pulse through the 64^3
    bubble cloud reaches a face state with c^2 <= 0 after 67 good CFL steps;
    HLLC passes those steps.  The library must report MFC_ERR_NONFINITE at the
    very step the oracle refuses, and not before."""
    from paper_2503_07953_amd import _lib as L
    c = W.bubble_cloud(64, nbub=6, slab=8)
    c.riemann = 1
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    k_oracle = None
    for k in range(80):
        try:
            O.step(q, cfl=0.5)
        except oracle.OracleError:
            k_oracle = k
            break
    assert k_oracle is not None
    S = _solver(c)
    qd = S.prim_to_cons(S.to_device(c.w))
    k_lib = None
    for k in range(80):
        S.step(qd, cfl=0.5)
        try:
            S.check()
        except L.MfcError as e:
            assert e.code == L.MFC_ERR_NONFINITE
            k_lib = k
            break
    _say("hll breakdown step: oracle", k_oracle, "library", k_lib)
    assert k_lib == k_oracle


@pytest.mark.parametrize("name", ["gresho-32", "random-2d-hllc", "random-3d-hllc", "random-2d-hll"])
def test_low_mach_correction_matches_oracle(name):
    """The low-Mach velocity correction of Thornber et al. (the paper's
    low-Mach section) before the face solver, RHS and 5 CFL steps."""
    _say("low-mach", name)
    if name == "gresho-32":
        c = W.gresho(32, mach=0.01)
        nf, nd = 1, 2
    else:
        nd = 3 if "3d" in name else 2
        nd_, n, nf, bc = (CASES[6] if nd == 3 else CASES[3])
        c = W.random_case(nd, n, nf=nf, seed=700 + nd, bc=bc, speed=150.0)
        c.riemann = 1 if name.endswith("hll") else 0
    c.low_mach = 1
    # the Gresho vortex is a steady state: its RHS is truncation error, small
    # beside fluxes of size p0, so the RHS is compared on the flux scale
    # (one-ulp spread of the oracle there: 4e-14; on the RHS's own scale 9e-11)
    _variant_steps_match(c, nf, nd, flux_scale=name.startswith("gresho"))


@pytest.mark.parametrize("variant,riemann,low_mach,case", [
    (1, 1, 1, 3), (3, 1, 1, 6), (3, 0, 1, 3), (2, 1, 0, 7),
    (2, 1, 1, 0), (1, 0, 1, 7), (3, 1, 0, 5), (2, 0, 1, 4)])
def test_option_combinations_match_oracle(variant, riemann, low_mach, case):
    """The reconstruction weights (Sec. 4.2.2), the face solver (HLLC / HLL)
    and the low-Mach correction are independent options, and every setting of
    the three is a kernel of its own: crossed settings, RHS and 5 CFL steps."""
    nd, n, nf, bc = CASES[case]
    _say("combination", variant, riemann, low_mach, nd, n, nf, bc)
    c = W.random_case(nd, n, nf=nf, seed=800 + 10 * variant + case, bc=bc,
                      speed=400.0 if nf == 1 else 150.0)
    c.weno_variant, c.riemann, c.low_mach = variant, riemann, low_mach
    _variant_steps_match(c, nf, nd)


def test_teno_rough_two_fluid_flagged_on_both_sides():
    """Two-fluid white noise under TENO5 reconstructs a face state with c^2 <= 0;
    the oracle refuses it and the library's check reports MFC_ERR_NONFINITE."""
    from paper_2503_07953_amd import _lib as L
    nd, n, nf, bc = CASES[3]
    c = W.random_case(nd, n, nf=nf, seed=500 + nd, bc=bc, speed=150.0)
    c.weno_variant = 2
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    with pytest.raises(oracle.OracleError):
        O.rhs(q)
    S = _solver(c)
    S.rhs(S.to_device(q))
    with pytest.raises(L.MfcError) as e:
        S.check()
    assert e.value.code == L.MFC_ERR_NONFINITE
    c.weno_variant = 0
    oracle.Oracle(c).rhs(q)
    S0 = _solver(c)
    S0.rhs(S0.to_device(q))
    S0.check()


def test_weno_variants_differ():
    """The four reconstructions are distinct code paths (a non-smooth state)."""
    c = W.random_case(2, (40, 30), nf=2, seed=9, bc=(W.EXTRAP, W.PERIODIC))
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    rs = []
    for variant in (0, 1, 2, 3):
        c.weno_variant = variant
        S = _solver(c)
        rs.append(S.rhs(S.to_device(q)).cpu().numpy())
    for i in range(4):
        for j in range(i + 1, 4):
            assert not np.array_equal(rs[i], rs[j]), (i, j)


def test_sod_full_run_matches_oracle_and_exact():
    from oracle import exact_riemann as er
    c = W.sod(200)
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    n_or = O.run_to(q, 0.2, 0.5)
    S = _solver(c)
    qd = S.prim_to_cons(S.to_device(c.w))
    n_gpu = S.run_to(qd, 0.2, 0.5)
    S.check()
    assert n_gpu == n_or
    got = qd.cpu().numpy()
    assert conservative_errors(got, q, 1, 1).max() <= TOL
    w = S.cons_to_prim(qd).cpu().numpy()[:, 0, 0]
    x = (np.arange(200) + 0.5) / 200
    r, u, p = er.sample((1, 0, 1), (0.125, 0, 0.1), (x - 0.5) / 0.2)
    assert np.mean(np.abs(w[0] - r)) <= 4e-3


def test_uniform_state_gives_zero_rhs_bitwise():
    n = (70, 20, 18)
    w = np.zeros((8,) + n[::-1])
    w[0], w[1], w[2], w[3], w[4], w[5], w[6], w[7] = 300.0, 0.7, 12.0, -5.0, 3.0, 2e5, 0.3, 0.7
    c = W.Case("u", 3, n, 2, (0.1, 0.1, 0.1), (6.12, 1.4), (3.43e8, 0.0), (0,) * 3, (0,) * 3, w)
    S = _solver(c)
    r = S.rhs(S.prim_to_cons(S.to_device(w))).cpu().numpy()
    assert np.all(r == 0.0)


def test_periodic_shift_and_determinism_bitwise():
    c = W.random_case(2, (100, 60), nf=2, seed=7, bc=(W.PERIODIC, W.PERIODIC))
    S = _solver(c)
    q = S.prim_to_cons(S.to_device(c.w))
    r1 = S.rhs(q).cpu().numpy()
    r2 = S.rhs(q).cpu().numpy()
    assert np.array_equal(r1, r2)
    qs = torch.roll(q, shifts=(7, -5), dims=(3, 2)).contiguous()
    rs = S.rhs(qs).cpu().numpy()
    assert np.array_equal(rs, np.roll(r1, (7, -5), axis=(3, 2)))
    a = q.clone()
    b = q.clone()
    S.run(a, 3, cfl=0.5)
    S.run(b, 3, cfl=0.5)
    assert torch.equal(a, b)


def test_nonfinite_state_is_reported():
    from paper_2503_07953_amd import _lib as L
    c = W.random_case(1, (64,), nf=1, seed=1)
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    q[2, 0, 0, 20] = -1e6  # energy below kinetic: negative pressure
    S = _solver(c)
    S.rhs(S.to_device(q))
    with pytest.raises(L.MfcError) as e:
        S.check()
    assert e.value.code == L.MFC_ERR_NONFINITE
    S.check()  # flag is cleared


def test_invalid_arguments_rejected():
    from paper_2503_07953_amd import _lib as L
    c = W.random_case(2, (16, 16), nf=2, seed=1)
    S = _solver(c)
    q = S.prim_to_cons(S.to_device(c.w))
    with pytest.raises(L.MfcError) as e:
        S.step(q, cfl=0.5, dt_fixed=1e-7)
    assert e.value.code == L.MFC_ERR_ARG
    with pytest.raises(L.MfcError) as e:
        S.step(q)
    assert e.value.code == L.MFC_ERR_ARG
    import ctypes
    rc = S.lib.mfc_rhs(S.ctx, ctypes.c_void_p(q.data_ptr() + 4), ctypes.c_void_p(q.data_ptr() + 8), None)
    assert rc == L.MFC_ERR_ARG


# --------------------------------------------------------------------------
# configurations at their full sizes
# --------------------------------------------------------------------------
@pytest.mark.timeout(900)
@pytest.mark.slow
def test_shock_cylinder_512_full_run_matches_oracle():
    """The 2D shock-cylinder configuration, 512^2, 500 CFL steps."""
    c = W.shock_cylinder(512)
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    S = _solver(c)
    qd = S.to_device(q)
    _say("C1 gpu run")
    S.run(qd, c.steps, cfl=0.5)
    S.check()
    _say("C1 oracle run")
    O.run(q, c.steps, cfl=0.5)
    err = conservative_errors(qd.cpu().numpy(), q, 2, 2)
    _say("C1 errors", err)
    assert err.max() <= TOL, err


@pytest.mark.timeout(600)
@pytest.mark.slow
def test_bubble_cloud_256_full_size_step_and_sampled_rhs():
    """The 3D bubble cloud at 256^3: sampled RHS cells, then one full CFL step."""
    c = W.bubble_cloud(256)
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    S = _solver(c)
    qd = S.to_device(q)
    r = S.rhs(qd).cpu().numpy().reshape(c.neq, -1)
    rng = np.random.default_rng(0)
    cells = rng.choice(c.ncell, size=4000, replace=False)
    ref = O.rhs_cells(q, cells).T
    # bubbles at rest in uniform pressure: the exact alpha / air-density RHS is
    # zero there, so errors are measured on the flux scale of each field
    err = rate_errors(r[:, cells], ref, q.reshape(c.neq, -1)[:, cells], O.max_signal(q), 2, 3)
    _say("C2 sampled rhs errors", err)
    assert err.max() <= TOL, err
    _say("C2 step")
    S.step(qd, cfl=0.5)
    S.check()
    O.step(q, cfl=0.5)
    # after one step the pulse is still a planar wave along x and the bubbles
    # sit at rest in uniform pressure (the pulse starts 4 + r cells before the
    # nearest bubble): the y and z momentum are zero in exact arithmetic
    err = conservative_errors(qd.cpu().numpy(), q, 2, 3, zero_mom=(1, 2))
    _say("C2 step errors", err)
    assert err.max() <= TOL, err


@pytest.mark.timeout(900)
@pytest.mark.slow
def test_periodic_slab_512_full_size_rhs_step_and_conservation():
    """The periodic air-water slab at 512^3: sampled RHS cells and one full CFL
    step against the oracle (FP64), conservation of the partial masses,
    momentum and energy over that step to rounding, and the FP32 form's RHS on
    the same cells on the flux scale (bar 1e-4, as for the FP32 form at small
    sizes)."""
    c = W.periodic_slab(512)
    _say("C4 initial condition ready")
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    c.w = None
    S = _solver(c)
    qd = S.to_device(q)
    rng = np.random.default_rng(0)
    cells = rng.choice(c.ncell, size=4000, replace=False)
    cidx = torch.from_numpy(cells).cuda()
    r = S.rhs(qd).reshape(c.neq, -1)[:, cidx].cpu().numpy()
    ref = O.rhs_cells(q, cells).T
    smax = O.max_signal(q)
    qs = q.reshape(c.neq, -1)[:, cells]
    err = rate_errors(r, ref, qs, smax, 2, 3)
    _say("C4 sampled rhs errors", err)
    assert err.max() <= TOL, err
    S32 = _solver(c, "fp32")
    r32 = S32.rhs(S32.to_device(q.astype(np.float32))).reshape(c.neq, -1)[:, cidx].double().cpu().numpy()
    S32.check()
    del S32
    e32 = rate_errors(r32, ref, qs, smax, 2, 3)
    _say("C4 fp32 sampled rhs errors", e32)
    assert e32.max() <= 1e-4, e32
    sums0 = S.conserved_sums(qd).cpu().numpy()
    _say("C4 step")
    S.step(qd, cfl=0.5)
    S.check()
    sums1 = S.conserved_sums(qd).cpu().numpy()
    O.step(q, cfl=0.5)
    err = conservative_errors(qd.cpu().numpy(), q, 2, 3)
    _say("C4 step errors", err)
    assert err.max() <= TOL, err
    # periodic: no boundary flux, so every conservative row except the volume
    # fractions (which carry the non-conservative source) keeps its sum
    scale = np.abs(q).reshape(c.neq, -1).sum(axis=1) * c.dx[0] * c.dx[1] * c.dx[2]
    drift = np.abs(sums1 - sums0)[:6] / scale[:6]
    _say("C4 conservation drift", drift)
    assert np.all(drift <= 1e-13), drift


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("nd", [2, 3])
def test_fused_cfl_dt_equals_the_standalone_signal(nd, precision):
    """In 2D and 3D the first axis pass of a CFL step forms the signal maxima;
    dt must be exactly cfl / mfc_max_signal (both divisions in double), the
    t_remaining clip must apply, and a fixed-dt step with that value must give
    the same state bit for bit."""
    from paper_2503_07953_amd.solver import Solver
    n = (40, 36, 30)[:nd]
    bc = (W.PERIODIC, W.SLIPWALL, W.EXTRAP)[:nd]
    c = W.random_case(nd, n, nf=2, seed=81, bc=bc, speed=150.0)
    S = Solver.from_case(c, precision=precision)
    q = S.prim_to_cons(S.to_device(c.w))
    smax = S.max_signal(q).item()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    q_cfl = q.clone()
    S.step(q_cfl, cfl=0.4, dt_out=dt)
    assert dt.item() == 0.4 / smax
    q_clip = q.clone()
    S.step(q_clip, cfl=0.4, t_remaining=0.25 * (0.4 / smax), dt_out=dt)
    assert dt.item() == 0.25 * (0.4 / smax)
    q_fix = q.clone()
    S.step(q_fix, dt_fixed=0.4 / smax)
    S.check()
    assert torch.equal(q_cfl, q_fix)


@pytest.mark.slow
def test_chunked_x_launch_and_indices_past_2_31():
    """3 x 65535 x 1400 cells, 8 rows, FP32: 2.2e9 elements, so element
    indices pass 2^31, and 2.3e7 x-pass blocks, so that pass runs as two
    launches (chunks of 2^24 blocks).  The state repeats a 3 x 65535 x 14 block
    100 times along a periodic z: every cell sees the stencil values of its
    twin in the small periodic grid, so the RHS and one CFL step must tile the
    small grid's results bit for bit (dt included)."""
    from paper_2503_07953_amd.solver import Solver
    P, reps = 14, 100
    c = W.random_case(3, (3, 65535, P), nf=2, seed=71, bc=(W.PERIODIC, W.EXTRAP, W.PERIODIC), speed=100.0)
    small = Solver.from_case(c, precision="fp32")
    q_small = small.prim_to_cons(small.to_device(c.w))
    kw = dict(c.problem_kwargs())
    kw["n"] = (3, 65535, P * reps)
    _say("large grid", kw["n"])
    big = Solver(**kw, precision="fp32")
    q_big = q_small.repeat(1, reps, 1, 1)
    neq, ny, nx = q_small.shape[0], 65535, 3

    def tiled(a_big, a_small):
        return torch.equal(a_big.view(neq, reps, P, ny, nx), a_small.unsqueeze(1).expand(neq, reps, P, ny, nx))

    r_small = small.rhs(q_small)
    r_big = big.rhs(q_big)
    assert tiled(r_big, r_small)
    del r_big
    dts = torch.zeros(1, dtype=torch.float64, device="cuda")
    dtb = torch.zeros(1, dtype=torch.float64, device="cuda")
    small.step(q_small, cfl=0.5, dt_out=dts)
    big.step(q_big, cfl=0.5, dt_out=dtb)
    small.check()
    big.check()
    assert dts.item() == dtb.item()
    assert tiled(q_big, q_small)
