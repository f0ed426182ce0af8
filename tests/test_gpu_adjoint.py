"""Hand-written HIP adjoint against torch autograd of the FP64 torch reference.

The reference (oracle/torch_ref.py) reproduces the C oracle bit for bit and
its autograd gradient is pinned against finite differences of the C oracle
(tests/test_oracle_pins.py), so it fixes the discrete gradient that the HIP
adjoint must reproduce element by element.

Tolerance.  WENO-JS weight derivatives scale like 1/(eps + beta) and react to
rounding-level data: perturbing q by one ulp moves the reference adjoint by
1e-10 .. 1e-8 (relative, per row).  No float64 implementation can agree with
the reference better than that spread, so each test measures it (helpers.
noise_floor) and requires the HIP adjoint to lie within 10x of it (and never
needs more than 1e-7); a wrong or missing term shows as 1e-3 .. 1.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from helpers import field_errors, noise_floor
from oracle import torch_ref as TR

pytestmark = pytest.mark.gpu
TOL = 1e-11


def _say(*a):
    print("[gpu-adjoint]", *a, flush=True)


def _solver(case):
    from paper_2503_07953_amd.solver import Solver
    return Solver.from_case(case, precision="fp64")


CASES = [
    (1, (70,), 2, (W.SLIPWALL,)),
    (1, (64,), 1, (W.EXTRAP,)),
    (2, (70, 45), 2, (W.EXTRAP, W.SLIPWALL)),
    (2, (33, 40), 2, (W.PERIODIC, W.EXTRAP)),
    (2, (40, 36), 1, (W.PERIODIC, W.PERIODIC)),
    (3, (20, 17, 14), 2, (W.SLIPWALL, W.PERIODIC, W.EXTRAP)),
    (3, (3, 4, 5), 2, (W.EXTRAP, W.SLIPWALL, W.PERIODIC)),
]


@pytest.mark.parametrize("nd,n,nf,bc,variant", [cs + (0,) for cs in CASES]
                         + [CASES[2] + (1,), CASES[5] + (1,), CASES[2] + (2,), CASES[5] + (2,),
                            CASES[2] + (3,), CASES[5] + (3,), CASES[4] + (3,)])
def test_rhs_vjp_matches_reference_autograd(nd, n, nf, bc, variant):
    """variant 0: WENO5-JS, 1: WENO5-Z, 2: TENO5, 3: WENO5-M."""
    _say("rhs_vjp", nd, n, nf, bc, "variant", variant)
    c = W.random_case(nd, n, nf=nf, seed=40 + nd, bc=bc, speed=300.0 if nf == 1 else 150.0)
    c.weno_variant = variant
    _rhs_vjp_vs_autograd(c)


@pytest.mark.parametrize("nd,n,nf,bc", [CASES[0], CASES[2], CASES[4], CASES[5]])
def test_hll_rhs_vjp_matches_reference_autograd(nd, n, nf, bc):
    """The HLL face solver's hand-written adjoint against autograd of the
    torch reference."""
    _say("hll rhs_vjp", nd, n, nf, bc)
    c = W.random_case(nd, n, nf=nf, seed=45 + nd, bc=bc, speed=300.0 if nf == 1 else 150.0)
    c.riemann = 1
    _rhs_vjp_vs_autograd(c)


@pytest.mark.parametrize("nd,n,nf,bc,riemann", [CASES[2] + (0,), CASES[5] + (0,), CASES[4] + (0,), CASES[2] + (1,)])
def test_low_mach_rhs_vjp_matches_reference_autograd(nd, n, nf, bc, riemann):
    """The adjoint through the low-Mach correction and the face solver."""
    _say("low-mach rhs_vjp", nd, n, nf, bc, riemann)
    c = W.random_case(nd, n, nf=nf, seed=75 + nd, bc=bc, speed=300.0 if nf == 1 else 150.0)
    c.riemann = riemann
    c.low_mach = 1
    _rhs_vjp_vs_autograd(c)


@pytest.mark.parametrize("variant,riemann,low_mach,case", [
    (1, 1, 1, 2), (3, 1, 1, 5), (2, 1, 1, 4), (3, 0, 1, 3), (1, 1, 0, 0)])
def test_option_combinations_rhs_vjp_match_reference_autograd(variant, riemann, low_mach, case):
    """The adjoint under crossed settings of the reconstruction weights, the
    face solver and the low-Mach correction."""
    nd, n, nf, bc = CASES[case]
    _say("combination rhs_vjp", variant, riemann, low_mach, nd, n, nf, bc)
    c = W.random_case(nd, n, nf=nf, seed=90 + 10 * variant + case, bc=bc,
                      speed=300.0 if nf == 1 else 150.0)
    c.weno_variant, c.riemann, c.low_mach = variant, riemann, low_mach
    _rhs_vjp_vs_autograd(c)


def _rhs_vjp_vs_autograd(c):
    nd, nf = c.ndim, c.num_fluids
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    P = TR.Problem.from_case(c)
    rng = np.random.default_rng(1)
    lam = rng.normal(size=q.shape)
    def fn(x):
        xt = torch.from_numpy(x.copy()).requires_grad_(True)
        return torch.autograd.grad(TR.rhs(P, xt), xt, torch.from_numpy(lam))[0].numpy()

    ref, spread = noise_floor(fn, q)
    S = _solver(c)
    got = S.rhs_vjp(S.to_device(q), S.to_device(lam)).cpu().numpy()
    err = field_errors(got, ref)
    _say("errors", err, "floor", spread)
    tol = np.minimum(np.maximum(10 * spread, TOL), 1e-7)
    assert np.all(err <= tol), (err, spread)
    # accumulate mode adds onto the output
    base = S.to_device(np.ones_like(q))
    S.rhs_vjp(S.to_device(q), S.to_device(lam), out=base, accumulate=True)
    err2 = field_errors(base.cpu().numpy() - 1.0, ref)
    assert np.all(err2 <= np.maximum(tol, 1e-9))


@pytest.mark.parametrize("nd,n,nf,bc", CASES[:6])
def test_step_vjp_matches_reference_autograd(nd, n, nf, bc):
    _say("step_vjp", nd, n, nf, bc)
    c = W.random_case(nd, n, nf=nf, seed=50 + nd, bc=bc, speed=150.0)
    _step_vjp_vs_autograd(c)


@pytest.mark.parametrize("nd,n,nf,bc", [CASES[2], CASES[5]])
def test_hll_step_vjp_matches_reference_autograd(nd, n, nf, bc):
    """The step adjoint through HLL faces (reading 16)."""
    _say("hll step_vjp", nd, n, nf, bc)
    c = W.random_case(nd, n, nf=nf, seed=55 + nd, bc=bc, speed=150.0)
    c.riemann = 1
    _step_vjp_vs_autograd(c)


@pytest.mark.parametrize("variant,riemann,low_mach,case", [(3, 1, 1, 2), (2, 0, 1, 4), (1, 1, 1, 5)])
def test_option_combinations_step_vjp_match_reference_autograd(variant, riemann, low_mach, case):
    """The SSP-RK3 step adjoint under crossed settings of the reconstruction
    weights, the face solver and the low-Mach correction."""
    nd, n, nf, bc = CASES[case]
    _say("combination step_vjp", variant, riemann, low_mach, nd, n, nf, bc)
    c = W.random_case(nd, n, nf=nf, seed=95 + 10 * variant + case, bc=bc, speed=150.0)
    c.weno_variant, c.riemann, c.low_mach = variant, riemann, low_mach
    _step_vjp_vs_autograd(c)


def _step_vjp_vs_autograd(c):
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    dt = 0.4 / O.max_signal(q)
    P = TR.Problem.from_case(c)
    lam = np.random.default_rng(2).normal(size=q.shape)
    def fn(x):
        xt = torch.from_numpy(x.copy()).requires_grad_(True)
        return torch.autograd.grad(TR.step(P, xt, dt), xt, torch.from_numpy(lam))[0].numpy()

    ref, spread = noise_floor(fn, q)
    S = _solver(c)
    got = S.step_vjp(S.to_device(q), dt, S.to_device(lam)).cpu().numpy()
    err = field_errors(got, ref)
    _say("errors", err, "floor", spread)
    tol = np.minimum(np.maximum(10 * spread, TOL), 1e-7)
    assert np.all(err <= tol), (err, spread)


@pytest.mark.parametrize("nd,n,nf", [(2, (30, 20), 2), (3, (8, 7, 6), 2), (1, (40,), 1)])
def test_conversion_vjps_match_reference(nd, n, nf):
    c = W.random_case(nd, n, nf=nf, seed=7)
    P = TR.Problem.from_case(c)
    S = _solver(c)
    rng = np.random.default_rng(3)
    qb = rng.normal(size=c.w.shape)

    def fw(x):
        xt = torch.from_numpy(x.copy()).requires_grad_(True)
        return torch.autograd.grad(TR.prim_to_cons(P, xt), xt, torch.from_numpy(qb))[0].numpy()

    ref, spread = noise_floor(fw, c.w)
    got = S.prim_to_cons_vjp(S.to_device(c.w), S.to_device(qb)).cpu().numpy()
    assert np.all(field_errors(got, ref) <= np.maximum(10 * spread, 1e-14))
    q = TR.prim_to_cons(P, torch.from_numpy(c.w)).numpy()
    qt = torch.from_numpy(q.copy()).requires_grad_(True)
    wb = rng.normal(size=c.w.shape)

    def fn(x):
        xt = torch.from_numpy(x.copy()).requires_grad_(True)
        return torch.autograd.grad(TR.cons_to_prim(P, xt), xt, torch.from_numpy(wb))[0].numpy()

    ref2, spread = noise_floor(fn, q)
    got = S.cons_to_prim_vjp(S.to_device(q), S.to_device(wb)).cpu().numpy()
    assert np.all(field_errors(got, ref2) <= np.maximum(10 * spread, 1e-14))


def test_rhs_vjp_dot_product_against_gpu_forward_differences():
    """<L(q+hv) - L(q-hv), lam>/2h (GPU forward) equals <v, L^T lam> (GPU adjoint)."""
    c = W.random_case(2, (48, 40), nf=2, seed=11, bc=(W.EXTRAP, W.SLIPWALL), speed=50.0,
                      pressure_jump=1.0, interface=False)
    S = _solver(c)
    q = S.prim_to_cons(S.to_device(c.w))
    rng = np.random.default_rng(0)
    for _ in range(2):
        v = torch.from_numpy(np.stack([W._smooth_field(rng, q.shape[1:], 2) for _ in range(q.shape[0])])).cuda()
        v = v * q.abs()
        lam = torch.from_numpy(rng.normal(size=q.shape)).cuda()
        lhs = float((S.rhs_vjp(q, lam) * v).sum())
        est = []
        for h in (4e-9, 2e-9):
            fd = (S.rhs((q + h * v).contiguous()) - S.rhs((q - h * v).contiguous())) / (2 * h)
            est.append(float((fd * lam).sum()))
        rich = (4 * est[1] - est[0]) / 3
        assert abs(rich / lhs - 1) <= 1e-5, (lhs, est)


def test_autograd_functions_chain():
    from paper_2503_07953_amd import autograd as AG
    c = W.random_case(2, (24, 20), nf=2, seed=3, bc=(W.EXTRAP, W.EXTRAP))
    S = _solver(c)
    P = TR.Problem.from_case(c)
    w = torch.from_numpy(c.w.copy())
    wd = S.to_device(c.w).requires_grad_(True)
    dt = 2e-7
    q = AG.PrimToCons.apply(wd, S)
    q = AG.Step.apply(q, S, dt)
    r = AG.RHS.apply(q, S)
    loss = (r * r).sum() * 1e-20 + AG.ConsToPrim.apply(q, S)[4].sum()
    loss.backward()
    wt = w.clone().requires_grad_(True)
    qt = TR.step(P, TR.prim_to_cons(P, wt), dt)
    rt = TR.rhs(P, qt)
    lt = (rt * rt).sum() * 1e-20 + TR.cons_to_prim(P, qt)[4].sum()
    lt.backward()
    assert field_errors(wd.grad.cpu().numpy(), wt.grad.numpy()).max() <= 1e-10


@pytest.mark.timeout(900)
@pytest.mark.slow
def test_rollout_gradient_matches_reference_at_64():
    """Adjoint problem at 64^2: gradient of the time-integrated wall pressure with
    respect to the initial alpha_1 and p, HIP adjoint vs torch autograd (200 steps,
    frozen dt, checkpoints every 20 steps).

    Bar: 10x the reference's own spread under a one-ulp change of alpha_1.  That
    spread is large here (~1e-4 of max|grad| for alpha_1): in post-shock water
    (7e8 Pa, E ~ 4e9) the pressure carries ~1e-6 Pa of cancellation noise, and
    WENO-JS weight derivatives at such numerically uniform states scale like
    noise^2 / eps, so every float64 evaluation of this gradient moves by that
    much.  A wrong or missing adjoint term moves it by 1e-2 .. 1.
    """
    from paper_2503_07953_amd import autograd as AG
    c = W.adjoint_case(64, steps=200)
    S = _solver(c)
    O = oracle.Oracle(c)
    dt = 0.5 / O.max_signal(O.prim_to_cons(c.w))
    P = TR.Problem.from_case(c)
    ex = c.extra

    def ic(alpha1, p, lib):
        rw = lib(ex["rho_water"])
        ra = lib(ex["rho_air"])
        u, v = lib(ex["u"]), lib(ex["v"])
        rows = [alpha1 * rw, (1 - alpha1) * ra, u, v, p, alpha1, 1 - alpha1]
        return torch.stack(rows).reshape(7, 1, 64, 64).contiguous()

    a0 = c.w[5, 0].copy()
    p0 = c.w[4, 0].copy()
    # HIP adjoint
    ag = torch.from_numpy(a0).cuda().requires_grad_(True)
    pg = torch.from_numpy(p0).cuda().requires_grad_(True)
    q0 = AG.PrimToCons.apply(ic(ag, pg, lambda a: torch.from_numpy(a).cuda()), S)
    J = AG.rollout_objective(q0, S, c.steps, dt, every=20)
    J.backward()
    _say("J gpu", float(J.detach()))
    # reference: torch autograd with per-step checkpointing
    from torch.utils.checkpoint import checkpoint

    def reference(a_init):
        at = torch.from_numpy(a_init.copy()).requires_grad_(True)
        pt = torch.from_numpy(p0.copy()).requires_grad_(True)
        q = TR.prim_to_cons(P, ic(at, pt, torch.from_numpy))
        Jt = torch.zeros((), dtype=torch.float64)
        dy = c.dx[1]
        for _ in range(c.steps):
            q = checkpoint(lambda x: TR.step(P, x, dt), q, use_reentrant=False)
            Jt = Jt + dt * dy * TR.cons_to_prim(P, q)[4, 0, :, 63].sum()
        Jt.backward()
        return float(Jt.detach()), at.grad.numpy(), pt.grad.numpy()

    Jr, ra, rp = reference(a0)
    _say("J ref", Jr)
    # J sums wall pressures p = (E - ke - Pi)/Gamma; in water at 1 bar the
    # cancellation amplifies state rounding by Pi/(Gamma p) ~ 2e4, so J agrees to
    # ~1e-12 * 2e4 at most
    assert abs(float(J.detach()) / Jr - 1) <= 1e-9
    rng = np.random.default_rng(9)
    a1 = a0 * (1.0 + rng.choice([-1.0, 0.0, 1.0], size=a0.shape) * np.finfo(float).eps)
    _, sa, sp = reference(a1)
    fa = np.abs(sa - ra).max() / np.abs(ra).max()
    fp = np.abs(sp - rp).max() / np.abs(rp).max()
    ga, gp = ag.grad.cpu().numpy(), pg.grad.cpu().numpy()
    ea = np.abs(ga - ra).max() / np.abs(ra).max()
    ep = np.abs(gp - rp).max() / np.abs(rp).max()
    _say("grad errors", ea, ep, "reference spread", fa, fp)
    assert ea <= 10 * max(fa, 1e-12)
    assert ep <= 10 * max(fp, 1e-12)


# --------------------------------------------------------------------------
# rollout gradients against central differences of the HIP forward
# --------------------------------------------------------------------------
def _rollout_setup(c, column):
    """J(alpha_1, p): the IC map (phase densities and velocity held), the frozen
    dt of the initial state, and the HIP rollout objective on one x-column."""
    from paper_2503_07953_amd import autograd as AG
    n = c.n[0]
    S = _solver(c)
    ex = c.extra

    def ic(alpha1, p):
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        rows = [alpha1 * t(ex["rho_water"]), (1 - alpha1) * t(ex["rho_air"]), t(ex["u"]), t(ex["v"]), p,
                alpha1, 1 - alpha1]
        return torch.stack(rows).reshape(7, 1, n, n).contiguous()

    a0 = torch.from_numpy(c.w[5, 0].copy()).cuda()
    p0 = torch.from_numpy(c.w[4, 0].copy()).cuda()
    dt = 0.5 / S.max_signal(S.prim_to_cons(ic(a0, p0))).item()   # frozen at its step-0 value

    def J(alpha1, p):
        q = AG.PrimToCons.apply(ic(alpha1, p), S)
        return AG.rollout_objective(q, S, c.steps, dt, every=20, column=column)

    return a0, p0, J


def _smooth_direction(rng, n):
    """Sum of four seeded Fourier modes, wavenumbers 1..3 per axis."""
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    f = np.zeros((n, n))
    for _ in range(4):
        kx, ky = rng.integers(1, 4, size=2)
        f += rng.normal() * np.cos(2 * np.pi * kx * X + rng.uniform(0, 2 * np.pi)) \
            * np.cos(2 * np.pi * ky * Y + rng.uniform(0, 2 * np.pi))
    return f


def _fd_projections(c, column, h, ndir, seed):
    """<grad J, v> from the HIP adjoint and from central differences of the HIP
    forward, on `ndir` seeded smooth directions v = (1e-3 f_a, 1e-3 f_p p0)."""
    a0, p0, J = _rollout_setup(c, column)
    ag = a0.clone().requires_grad_(True)
    pg = p0.clone().requires_grad_(True)
    J(ag, pg).backward()
    rng = np.random.default_rng(seed)
    n = c.n[0]
    out = []
    for k in range(ndir):
        va = torch.from_numpy(_smooth_direction(rng, n) * 1e-3).cuda()
        vp = torch.from_numpy(_smooth_direction(rng, n) * 1e-3).cuda() * p0
        lin = float((ag.grad * va).sum() + (pg.grad * vp).sum())
        with torch.no_grad():
            fd = (float(J(a0 + h * va, p0 + h * vp)) - float(J(a0 - h * va, p0 - h * vp))) / (2 * h)
        _say(c.name, "direction", k, "adjoint", lin, "fd", fd, "rel", abs(fd - lin) / abs(lin))
        out.append((lin, fd))
    return np.array(out)


@pytest.mark.timeout(900)
@pytest.mark.slow
def test_rollout_adjoint_matches_central_differences_on_smooth_mixture_256():
    """256^2 smooth air-water mixture, 200 frozen-dt steps, checkpoints every 20:
    <grad J, v> of the HIP adjoint against central differences of the HIP
    forward on 32 seeded smooth directions, to 1e-6 relative.  Every field
    varies smoothly there, WENO indicators sit well above eps, and J is smooth on
    the step scale (h = 1e-3: FD truncation and rounding both near 1e-7)."""
    c = W.smooth_mixture(256, steps=200)
    res = _fd_projections(c, 128, 1e-3, 32, seed=31)
    rel = np.abs(res[:, 1] - res[:, 0]) / np.abs(res[:, 0])
    _say("smooth mixture worst relative difference", rel.max())
    assert rel.max() <= 1e-6


@pytest.mark.timeout(900)
@pytest.mark.slow
def test_adjoint_256_matches_reference_autograd():
    """The adjoint configuration at its own size: shock-cylinder problem at
    256^2, 200 frozen-dt steps, checkpoints every 20; gradient of the
    time-integrated wall pressure with respect to the initial alpha_1 and p.
    The reference is the torch float64 version of the discretization
    differentiated by autograd (a checkpoint per step), run on the GPU with
    torch's own kernels, so it shares nothing with the HIP library.

    The p gradient is deterministic: per cell (max-relative) and through 32
    seeded N(0, 1) directions (|<g - g_ref, z>| over |g_ref|_2, the standard
    deviation of <g_ref, z>) it must agree to the FP64 bar 1e-12 (measured
    1.2e-15 and 1.7e-15; the reference itself moves by 1.6e-7 and 5e-7 under
    a one-ulp change of alpha_1).  Within 200 steps J does not feel alpha_1: its
    gradient is at most ~2e-12 per cell, in numerically uniform water next to
    the wall, and pure rounding noise -- the reference moves by more than its
    own size under that one-ulp change.  There the HIP gradient only has to be
    noise of the same size: within 10x the reference's spread, per cell and
    through the directions."""
    from torch.utils.checkpoint import checkpoint
    from paper_2503_07953_amd import autograd as AG
    import time
    n = 256
    c = W.adjoint_case(n, steps=200)
    S = _solver(c)
    O = oracle.Oracle(c)
    dt = 0.5 / O.max_signal(O.prim_to_cons(c.w))
    P = TR.Problem.from_case(c)
    ex = c.extra
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()

    def ic(alpha1, p):
        rows = [alpha1 * dev(ex["rho_water"]), (1 - alpha1) * dev(ex["rho_air"]), dev(ex["u"]), dev(ex["v"]), p,
                alpha1, 1 - alpha1]
        return torch.stack(rows).reshape(7, 1, n, n).contiguous()

    a0 = c.w[5, 0].copy()
    p0 = c.w[4, 0].copy()
    t0 = time.time()
    ag = dev(a0).requires_grad_(True)
    pg = dev(p0).requires_grad_(True)
    J = AG.rollout_objective(AG.PrimToCons.apply(ic(ag, pg), S), S, c.steps, dt, every=20)
    J.backward()
    torch.cuda.synchronize()
    _say("C3 HIP adjoint", time.time() - t0, "s; J", float(J.detach()))

    def reference(a_init):
        t1 = time.time()
        at = dev(a_init).requires_grad_(True)
        pt = dev(p0).requires_grad_(True)
        q = TR.prim_to_cons(P, ic(at, pt))
        Jt = torch.zeros((), dtype=torch.float64, device="cuda")
        dy = c.dx[1]
        for _ in range(c.steps):
            q = checkpoint(lambda x: TR.step(P, x, dt), q, use_reentrant=False)
            Jt = Jt + dt * dy * TR.cons_to_prim(P, q)[4, 0, :, n - 1].sum()
        Jt.backward()
        torch.cuda.synchronize()
        _say("C3 reference autograd on the GPU", time.time() - t1, "s")
        return float(Jt.detach()), at.grad.cpu().numpy(), pt.grad.cpu().numpy()

    Jr, ra, rp = reference(a0)
    _say("J", float(J.detach()), "reference", Jr)
    assert abs(float(J.detach()) / Jr - 1) <= 1e-12
    rng = np.random.default_rng(19)
    _, sa, sp = reference(a0 * (1.0 + rng.choice([-1.0, 0.0, 1.0], size=a0.shape) * np.finfo(float).eps))
    ga, gp = ag.grad.cpu().numpy(), pg.grad.cpu().numpy()
    zs = np.random.default_rng(20).standard_normal((32, n, n))
    field = lambda x, y: np.abs(x - y).max() / np.abs(y).max()
    proj = lambda x, y: max(abs((z * (x - y)).sum()) for z in zs) / np.linalg.norm(y)
    ep, ejp, fp = field(gp, rp), proj(gp, rp), field(sp, rp)
    ea, eja, fa, fja = field(ga, ra), proj(ga, ra), field(sa, ra), proj(sa, ra)
    _say("C3 p gradient vs reference: per cell", ep, "directions", ejp, "| reference one-ulp spread", fp)
    _say("C3 alpha_1 gradient: max |g_ref|", np.abs(ra).max(), "vs reference: per cell", ea, "directions", eja,
         "| reference one-ulp spread: per cell", fa, "directions", fja)
    assert ep <= 1e-12 and ejp <= 1e-12
    assert np.abs(ra).max() <= 1e-10 * abs(Jr)
    assert ea <= 10 * fa and eja <= 10 * fja


@pytest.mark.timeout(900)
@pytest.mark.slow
def test_adjoint_256_against_central_differences_at_fd_resolution():
    """Shock-cylinder adjoint problem at 256^2, 200 frozen-dt steps: <grad J, v>
    against central differences on 32 seeded smooth directions.

    Finite differences resolve this gradient only to about 1e-2.  J depends on
    the initial fields mainly through pressure in uniform water next to the
    wall, where WENO-JS indicators vanish and the weights bend on a data scale
    of sqrt(eps) = 1e-3 Pa; a step h moves neighbouring cells apart by ~7 h Pa,
    so h >= 1e-5 leaves the linear regime, while for h <= 1e-6 the change of J
    (~1e-10) approaches its rounding noise.  Measured at h = 1e-6: median
    |fd - adjoint| / max_k |adjoint_k| ~ 0.03, worst ~ 0.26, cosine of the two
    32-vectors ~ 0.98.  The bars below catch a sign error or a dropped term
    (O(1) on every direction); the 1e-6 bar is held on the smooth mixture
    above, through the same kernels, size and step count."""
    c = W.adjoint_case(256, steps=200)
    res = _fd_projections(c, -1, 1e-6, 32, seed=30)
    lin, fd = res[:, 0], res[:, 1]
    err = np.abs(fd - lin) / np.abs(lin).max()
    cos = float(lin @ fd / (np.linalg.norm(lin) * np.linalg.norm(fd)))
    _say("C3 normalized differences: median", np.median(err), "max", err.max(), "cosine", cos)
    assert np.median(err) <= 0.1
    assert err.max() <= 0.5
    assert cos >= 0.95


def test_step_with_saved_stages_matches_step_and_step_vjp_bitwise():
    """mfc_step_save_stages advances exactly as mfc_step (fixed dt) and
    mfc_step_vjp_stages on its stages returns exactly mfc_step_vjp."""
    c = W.random_case(2, (70, 45), nf=2, seed=21, bc=(W.EXTRAP, W.SLIPWALL))
    S = _solver(c)
    q = S.prim_to_cons(S.to_device(c.w))
    dt = 0.4 / S.max_signal(q).item()
    a = q.clone()
    S.step(a, dt_fixed=dt)
    b = q.clone()
    q1, q2 = torch.empty_like(q), torch.empty_like(q)
    S.step_save_stages(b, dt, q1, q2)
    assert torch.equal(a, b)
    lam = torch.from_numpy(np.random.default_rng(4).normal(size=q.shape)).cuda()
    g1 = S.step_vjp(q, dt, lam)
    g2 = S.step_vjp_stages(q, q1, q2, dt, lam)
    S.check()
    assert torch.equal(g1, g2)
    from paper_2503_07953_amd import _lib as L
    with pytest.raises(L.MfcError):
        S.step_save_stages(b, dt, q1, q1)


@pytest.mark.parametrize("nd,n,nf,bc", [CASES[2], CASES[5]])
def test_rhs_vjp_one_axis_at_a_time_matches_all_axes(nd, n, nf, bc, monkeypatch):
    """The adjoint's two schedules: every axis's face pass in one launch with
    one cell pass (default at these sizes), and one axis after the other through
    a shared face buffer (forced by a zero face budget).  Same arithmetic per
    face; only the order in which the axes' cotangents are summed differs."""
    c = W.random_case(nd, n, nf=nf, seed=60 + nd, bc=bc, speed=200.0)
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    lam = np.random.default_rng(3).normal(size=q.shape)
    S_all = _solver(c)
    g_all = S_all.rhs_vjp(S_all.to_device(q), S_all.to_device(lam)).cpu().numpy()
    monkeypatch.setenv("MFC355_ADJOINT_FACE_BUDGET", "0")
    S_seq = _solver(c)
    g_seq = S_seq.rhs_vjp(S_seq.to_device(q), S_seq.to_device(lam)).cpu().numpy()
    S_all.check()
    S_seq.check()
    err = field_errors(g_seq, g_all)
    _say("sequential vs all-axes", err)
    assert err.max() <= 1e-13


def _normal_sweep(c, column, hs, ndir, seed):
    """<grad J, v> of the HIP adjoint and central differences of the HIP
    forward at every step size in hs, on `ndir` seeded directions with N(0, 1)
    entries: v = (1e-3 g_a, 1e-3 g_p p0) (the adjoint configuration's
    directions).  Returns (lin[ndir], fd[len(hs), ndir])."""
    a0, p0, J = _rollout_setup(c, column)
    ag = a0.clone().requires_grad_(True)
    pg = p0.clone().requires_grad_(True)
    J(ag, pg).backward()
    rng = np.random.default_rng(seed)
    n = c.n[0]
    lin, fd = [], np.zeros((len(hs), ndir))
    for k in range(ndir):
        va = torch.from_numpy(rng.standard_normal((n, n)) * 1e-3).cuda()
        vp = torch.from_numpy(rng.standard_normal((n, n)) * 1e-3).cuda() * p0
        lin.append(float((ag.grad * va).sum() + (pg.grad * vp).sum()))
        with torch.no_grad():
            for i, h in enumerate(hs):
                fd[i, k] = (float(J(a0 + h * va, p0 + h * vp)) - float(J(a0 - h * va, p0 - h * vp))) / (2 * h)
    return np.array(lin), fd


@pytest.mark.timeout(900)
@pytest.mark.slow
def test_adjoint_256_second_objective_through_the_cylinder():
    """The second objective of the adjoint configuration: time-integrated
    pressure on the column x = 0.6 L, which crosses the air cylinder and whose
    domain of dependence over the 200 steps takes in the shock and the
    interface.  <grad J2, v> of the HIP adjoint against central differences on
    32 seeded N(0, 1) directions, swept over the step h (printed).  As for the
    wall objective, FD resolves this gradient only to about 1e-2: measured
    median |fd - adjoint| / max_k |adjoint_k| 0.11 at h = 1e-2 falling to 0.014
    at h = 1e-6 (the WENO weights of near-uniform states leave the linear
    regime on the data scale sqrt(eps)), then 0.024 at 1e-7 (rounding);
    cosine of the two 32-vectors 0.9992 at 1e-6.  Bars at the best step:
    median <= 0.03, worst <= 0.1, cosine >= 0.995; a dropped term or sign
    error is O(1) on every direction."""
    c = W.adjoint_case(256, steps=200)
    hs = [1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7]
    lin, fd = _normal_sweep(c, int(0.6 * c.n[0]), hs, 32, seed=32)
    best = None
    for i, h in enumerate(hs):
        err = np.abs(fd[i] - lin) / np.abs(lin).max()
        cos = float(lin @ fd[i] / (np.linalg.norm(lin) * np.linalg.norm(fd[i])))
        _say(f"J2 h={h:g}: median {np.median(err):.3e} worst {err.max():.3e} cosine {cos:.6f}")
        if best is None or np.median(err) < best[0]:
            best = (np.median(err), err.max(), cos, h)
    _say("J2 best step", best)
    assert best[0] <= 0.03 and best[1] <= 0.1 and best[2] >= 0.995, best
