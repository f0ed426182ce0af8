"""Seeded synthetic inputs for the five-equation RHS.

This module builds initial conditions only: primitive state arrays together
with the grid, fluid and boundary parameters that describe a problem.  It holds
none of the method's arithmetic (no equation of state, no reconstruction, no
flux): both the CPU oracle and the HIP library convert the primitive state to
conservative variables with their own code.

Primitive state layout (float64, C order) is ``w[v, k, j, i]`` (x fastest) with
rows, for ``nf`` fluids in ``D`` dimensions:

* ``nf`` partial densities ``alpha_i * rho_i``
* ``D`` velocity components
* pressure
* ``nf`` volume fractions (only when ``nf == 2``; a single fluid carries none)

which is the variable set the method reconstructs (Sec. 3.2.1 of the paper:
reconstruction acts on state variables; Sec. 2.1.1 lists the transported set).

Fluids (stiffened gas, Sec. 2.2): water gamma=6.12, pi_inf=3.43e8 Pa,
rho=1000; air gamma=1.4, pi_inf=0, rho=1.  Fluid 1 is water, fluid 2 is air.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PERIODIC, EXTRAP, SLIPWALL = 0, 1, 2

WATER = dict(gamma=6.12, pi_inf=3.43e8, rho=1000.0)
AIR = dict(gamma=1.4, pi_inf=0.0, rho=1.0)
ALPHA_FLOOR = 1e-6  # volume fractions are kept in [1e-6, 1 - 1e-6]


def num_eqs(ndim: int, nf: int) -> int:
    """Number of transported rows: 2N + D + 1 for two fluids, D + 2 for one."""
    return nf + ndim + 1 + (nf if nf == 2 else 0)


@dataclass
class Case:
    name: str
    ndim: int
    n: tuple            # (nx, ny, nz); unused axes are 1
    num_fluids: int
    dx: tuple           # uniform spacing per axis (unused axes: 1.0)
    gamma: tuple        # per fluid (length 2; second unused for one fluid)
    pi_inf: tuple
    bc_lo: tuple
    bc_hi: tuple
    w: np.ndarray       # primitive state, shape (neq, nz, ny, nx), float64
    steps: int = 0
    cfl: float = 0.5
    t_end: float = 0.0
    weno_eps: float = 1e-6
    weno_variant: int = 0   # 0: WENO5-JS, 1: WENO5-Z, 2: TENO5, 3: WENO5-M
    riemann: int = 0        # 0: HLLC, 1: HLL
    low_mach: int = 0       # 0: none, 1: Thornber et al. velocity correction, 2: Chen et al. APC
    model: int = 0          # 0: Allaire (K = 0), 1: Kapila (K div u on the alpha rows)
    faces: tuple = None     # per axis None (uniform dx) or the n + 1 face coordinates
    extra: dict = field(default_factory=dict)

    @property
    def neq(self) -> int:
        return num_eqs(self.ndim, self.num_fluids)

    @property
    def ncell(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def problem_kwargs(self) -> dict:
        """Plain numbers describing the problem (shared by both sides); the
        face coordinates only for a non-uniform grid."""
        kw = dict(ndim=self.ndim, n=tuple(self.n), num_fluids=self.num_fluids,
                  dx=tuple(self.dx), gamma=tuple(self.gamma),
                  pi_inf=tuple(self.pi_inf), bc_lo=tuple(self.bc_lo),
                  bc_hi=tuple(self.bc_hi), weno_eps=self.weno_eps, weno_variant=self.weno_variant,
                  riemann=self.riemann, low_mach=self.low_mach, model=self.model)
        if self.faces is not None:
            kw["faces"] = self.faces
        return kw


def _pad3(t, fill):
    t = tuple(t)
    return t + (fill,) * (3 - len(t))


def _centres(n, dx):
    return (np.arange(n, dtype=np.float64) + 0.5) * dx


def _tanh_fraction(signed_dist, width):
    """Smoothed indicator of signed_dist < 0, floored to [eps, 1 - eps]."""
    e = ALPHA_FLOOR
    return e + (1.0 - 2.0 * e) * 0.5 * (1.0 - np.tanh(signed_dist / width))


def _two_fluid_w(alpha_water, rho_w, rho_a, vel, p):
    """Assemble the primitive rows from phase quantities (fluid 1 water)."""
    nd = len(vel)
    shape = np.broadcast(alpha_water, rho_w, rho_a, p, *vel).shape
    w = np.empty((5 + nd,) + shape, dtype=np.float64)
    np.multiply(alpha_water, rho_w, out=w[0])
    np.subtract(1.0, alpha_water, out=w[4 + nd])      # alpha_air
    np.multiply(w[4 + nd], rho_a, out=w[1])
    for d, v in enumerate(vel):
        w[2 + d] = v
    w[2 + nd] = p
    w[3 + nd] = alpha_water
    return w


def water_shock_state(mach: float, p0: float = 1e5):
    """Post-shock water state for a shock of Mach `mach` running into water at rest.

    Stiffened-gas Rankine-Hugoniot relations: the ideal-gas relations with
    p replaced by p + pi_inf.  Returns (rho, u, p, shock_speed).
    """
    g, pi, rho0 = WATER["gamma"], WATER["pi_inf"], WATER["rho"]
    c0 = math.sqrt(g * (p0 + pi) / rho0)
    m2 = mach * mach
    rho1 = rho0 * (g + 1.0) * m2 / ((g - 1.0) * m2 + 2.0)
    pt1 = (p0 + pi) * (1.0 + 2.0 * g / (g + 1.0) * (m2 - 1.0))
    s = mach * c0
    u1 = s * (1.0 - rho0 / rho1)
    return rho1, u1, pt1 - pi, s


# ----------------------------------------------------------------------------
# C0: Sod shock tube (single ideal gas)
# ----------------------------------------------------------------------------
def sod(n: int = 200, t_end: float = 0.2, cfl: float = 0.5) -> Case:
    dx = 1.0 / n
    x = _centres(n, dx)
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    u = np.zeros(n)
    p = np.where(left, 1.0, 0.1)
    w = np.stack([rho, u, p]).reshape(3, 1, 1, n).astype(np.float64)
    return Case("sod", 1, (n, 1, 1), 1, (dx, 1.0, 1.0), (1.4, 1.4), (0.0, 0.0),
                (EXTRAP,) * 3, (EXTRAP,) * 3, w, steps=0, cfl=cfl, t_end=t_end)


# ----------------------------------------------------------------------------
# Smooth two-component advection (Sec. 3.5 convergence problem)
# ----------------------------------------------------------------------------
def stretched_faces(n: int, L: float = 1.0, a: float = 0.0) -> np.ndarray:
    """n + 1 face coordinates of a smoothly stretched grid on [0, L]:
    x(xi) = L (xi - a sin(2 pi xi) / (2 pi)) at xi = i/n.  The widths follow
    dx/dxi = L (1 - a cos(2 pi xi)), periodic in xi; |a| < 1, and the largest
    to smallest width ratio is (1 + |a|)/(1 - |a|).  a > 0 clusters cells at
    both ends, a < 0 at the centre; a = 0 is the uniform grid."""
    xi = np.arange(n + 1, dtype=np.float64) / n
    x = L * (xi - a * np.sin(2 * np.pi * xi) / (2 * np.pi))
    x[0], x[-1] = 0.0, L
    return x


def _sin_averages(faces, shift=0.0):
    a = faces[:-1] - shift
    b = faces[1:] - shift
    return (np.cos(2 * np.pi * a) - np.cos(2 * np.pi * b)) / (2 * np.pi * (faces[1:] - faces[:-1]))


def advection_1d(n: int, amplitude: float = 1.0, gamma2: float = 1.4, stretch: float = 0.0) -> Case:
    """alpha_i = alpha_i rho_i = 0.5 + (-1)^i A sin(2 pi x), u = p = 1, periodic.

    Cell averages of sin(2 pi x) over [a, b] are
    (cos 2 pi a - cos 2 pi b) / (2 pi (b - a)).  With A = 1 and both fluids
    ideal with gamma = 1.4 this is the problem as printed (volume fractions
    leave [0, 1] but the mixture stays an ideal gas with Gamma = 2.5, so it is
    pure linear advection); A = 0.25 with gamma2 = 1.6 is a physical variant.
    stretch != 0 puts the problem on the stretched grid of stretched_faces(n,
    1, stretch) (cell averages over the stretched cells).
    """
    dx = 1.0 / n
    faces = stretched_faces(n, 1.0, stretch)
    s = _sin_averages(faces)
    a1 = 0.5 - amplitude * s
    a2 = 0.5 + amplitude * s
    ones = np.ones(n)
    w = np.stack([a1, a2, ones, ones, a1, a2]).reshape(6, 1, 1, n).astype(np.float64)
    return Case(f"advection_{n}", 1, (n, 1, 1), 2, (dx, 1.0, 1.0), (1.4, gamma2), (0.0, 0.0),
                (PERIODIC,) * 3, (PERIODIC,) * 3, w, cfl=0.5,
                faces=(faces, None, None) if stretch != 0.0 else None,
                extra=dict(amplitude=amplitude))


def advection_exact_average(n: int, amplitude: float, t: float, u: float = 1.0, stretch: float = 0.0):
    """Exact cell averages of alpha_1 after advection by u*t (periodic)."""
    return 0.5 - amplitude * _sin_averages(stretched_faces(n, 1.0, stretch), u * t)


# ----------------------------------------------------------------------------
# C1 / C3: planar Mach-1.5 water shock hitting a perturbed air cylinder (2D)
# ----------------------------------------------------------------------------
def shock_cylinder(n: int = 512, seed: int = 1, steps: int = 500, mach: float = 1.5,
                   radius: float = 0.1, shock_x: float = 0.3, p0: float = 1e5) -> Case:
    L = 1.0
    dx = L / n
    rng = np.random.default_rng(seed)
    modes = np.arange(2, 17)
    amp = rng.uniform(-1.0, 1.0, size=modes.size)
    phase = rng.uniform(0.0, 2 * np.pi, size=modes.size)
    th_fine = np.linspace(0.0, 2 * np.pi, 8192, endpoint=False)
    pert_fine = (amp[:, None] * np.cos(modes[:, None] * th_fine[None, :] + phase[:, None])).sum(0)
    norm = np.abs(pert_fine).max()

    x = _centres(n, dx)
    X, Y = np.meshgrid(x, x, indexing="xy")       # shape (ny, nx)
    dxc, dyc = X - 0.5 * L, Y - 0.5 * L
    r = np.hypot(dxc, dyc)
    th = np.arctan2(dyc, dxc)
    pert = (amp[:, None, None] * np.cos(modes[:, None, None] * th[None] + phase[:, None, None])).sum(0)
    r_i = radius * L * (1.0 + 0.01 * pert / norm)
    alpha_air = _tanh_fraction(r - r_i, dx)
    alpha_w = 1.0 - alpha_air

    rho1, u1, p1, s = water_shock_state(mach, p0)
    post = X < shock_x * L
    rho_w = np.where(post, rho1, WATER["rho"])
    rho_a = np.full_like(X, AIR["rho"])
    u = np.where(post, u1, 0.0)
    v = np.zeros_like(X)
    p = np.where(post, p1, p0)
    w = _two_fluid_w(alpha_w, rho_w, rho_a, [u, v], p).reshape(7, 1, n, n)
    return Case(f"shock_cylinder_{n}", 2, (n, n, 1), 2, (dx, dx, 1.0),
                (WATER["gamma"], AIR["gamma"]), (WATER["pi_inf"], AIR["pi_inf"]),
                (EXTRAP, EXTRAP, EXTRAP), (SLIPWALL, EXTRAP, EXTRAP), w,
                steps=steps, cfl=0.5,
                extra=dict(seed=seed, shock_speed=s, post_shock=(rho1, u1, p1),
                           rho_water=rho_w, rho_air=rho_a, u=u, v=v))


def adjoint_case(n: int = 256, seed: int = 3, steps: int = 200) -> Case:
    """Adjoint problem: the shock-cylinder physics at n x n with frozen dt."""
    c = shock_cylinder(n=n, seed=seed, steps=steps)
    c.name = f"adjoint_{n}"
    return c


def smooth_mixture(n: int = 256, seed: int = 11, steps: int = 200, p0: float = 1e6) -> Case:
    """Smooth air-water mixture on a periodic square.

    Every field varies smoothly everywhere (no uniform patch, no jump): water
    fraction 0.5 +- 0.3, phase densities within 2 % (water) and 25 % (air),
    velocity up to 30 m/s, pressure p0 (1 +- 0.3).  WENO smoothness
    indicators then sit well above epsilon in every cell, so the discrete
    map is smooth on finite-difference step scales: the problem on which a
    rollout gradient can be checked against central differences closely.
    """
    L = 1.0
    dx = L / n
    rng = np.random.default_rng(seed)
    shape = (1, n, n)
    f = [_smooth_field(rng, shape, 2, nmodes=4, kmax=3)[0] for _ in range(6)]
    alpha_w = 0.5 + 0.3 * f[0]
    rho_w = WATER["rho"] * (1.0 + 0.02 * f[1])
    rho_a = AIR["rho"] * (1.0 + 0.25 * f[2])
    u, v = 30.0 * f[3], 30.0 * f[4]
    p = p0 * (1.0 + 0.3 * f[5])
    w = _two_fluid_w(alpha_w, rho_w, rho_a, [u, v], p).reshape(7, 1, n, n)
    return Case(f"smooth_mixture_{n}", 2, (n, n, 1), 2, (dx, dx, 1.0),
                (WATER["gamma"], AIR["gamma"]), (WATER["pi_inf"], AIR["pi_inf"]),
                (PERIODIC, PERIODIC, EXTRAP), (PERIODIC, PERIODIC, EXTRAP), w,
                steps=steps, cfl=0.5,
                extra=dict(seed=seed, rho_water=rho_w, rho_air=rho_a, u=u, v=v))


# ----------------------------------------------------------------------------
# C2: 3D bubble cloud in water with an entering pressure pulse
# ----------------------------------------------------------------------------
def bubble_positions(n: int, nbub: int, seed: int, slab: int = 16, rmin=4.0, rmax=12.0):
    rng = np.random.default_rng(seed)
    out = []
    tries = 0
    while len(out) < nbub:
        tries += 1
        if tries > 200000:
            raise RuntimeError("bubble rejection sampling did not converge")
        r = rng.uniform(rmin, rmax)
        lo = np.array([max(r + 2.0, slab + r + 4.0), r + 2.0, r + 2.0])
        hi = np.full(3, n - r - 2.0)
        if np.any(hi <= lo):
            continue
        c = lo + (hi - lo) * rng.uniform(0.0, 1.0, size=3)
        if all(np.linalg.norm(c - c2) >= r + r2 + 2.0 for c2, r2 in out):
            out.append((c, r))
    return out


def bubble_cloud(n: int = 256, seed: int = 2, nbub: int = 64, steps: int = 200,
                 p0: float = 1e5, p_pulse: float = 1e7, slab: int = 16) -> Case:
    L = 1.0
    dx = L / n
    bubbles = bubble_positions(n, nbub, seed, slab=slab)
    alpha_air = np.full((n, n, n), ALPHA_FLOOR)       # (z, y, x)
    ci = np.arange(n, dtype=np.float64) + 0.5            # cell centres in cell units
    for c, r in bubbles:
        lo = np.maximum(np.floor(c - r - 8).astype(int), 0)
        hi = np.minimum(np.ceil(c + r + 8).astype(int), n)
        xs, ys, zs = ci[lo[0]:hi[0]], ci[lo[1]:hi[1]], ci[lo[2]:hi[2]]
        d = np.sqrt((xs[None, None, :] - c[0]) ** 2 + (ys[None, :, None] - c[1]) ** 2
                    + (zs[:, None, None] - c[2]) ** 2)
        a = _tanh_fraction((d - r) * dx, dx)
        sub = alpha_air[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        np.maximum(sub, a, out=sub)
    alpha_w = 1.0 - alpha_air
    cw = math.sqrt(WATER["gamma"] * (p0 + WATER["pi_inf"]) / WATER["rho"])
    u_pulse = (p_pulse - p0) / (WATER["rho"] * cw)
    xi = np.arange(n)
    pulse = (xi < slab)[None, None, :]
    p = np.where(pulse, p_pulse, p0) * np.ones((n, n, n))
    u = np.where(pulse, u_pulse, 0.0) * np.ones((n, n, n))
    z = np.zeros((n, n, n))
    w = _two_fluid_w(alpha_w, WATER["rho"], AIR["rho"], [u, z, z], p)
    return Case(f"bubble_cloud_{n}", 3, (n, n, n), 2, (dx, dx, dx),
                (WATER["gamma"], AIR["gamma"]), (WATER["pi_inf"], AIR["pi_inf"]),
                (EXTRAP,) * 3, (EXTRAP,) * 3, w, steps=steps, cfl=0.5,
                extra=dict(seed=seed, bubbles=bubbles, u_pulse=u_pulse))


# ----------------------------------------------------------------------------
# C4: periodic air-water slab advected by a random solenoidal velocity field
# ----------------------------------------------------------------------------
def _interface_height(n, seed_rng, amplitude):
    k = np.arange(-16, 17)
    KX, KY = np.meshgrid(k, k, indexing="xy")
    kk = np.hypot(KX, KY)
    sel = (kk >= 2) & (kk <= 16)
    kx, ky = KX[sel], KY[sel]
    a = seed_rng.normal(size=kx.size)
    ph = seed_rng.uniform(0, 2 * np.pi, size=kx.size)
    x = (np.arange(n) + 0.5) / n
    # separable evaluation: cos(2pi(kx x + ky y) + ph) = Re(e^{i ph} e^{2pi i kx x} e^{2pi i ky y})
    ex = np.exp(2j * np.pi * np.outer(kx, x))          # (m, nx)
    ey = np.exp(2j * np.pi * np.outer(ky, x))          # (m, ny)
    eta = np.real((ey.T * (a * np.exp(1j * ph))[None, :]) @ ex)
    return amplitude * eta / np.abs(eta).max()


def periodic_slab(n: int = 512, seed: int = 4, steps: int = 100, mach_rms: float = 0.3,
                  kmax: int = 32, dtype=np.float64) -> Case:
    """Water slab z in [L/4 + eta1, 3L/4 + eta2] in air, random k^-2 solenoidal velocity."""
    import scipy.fft as sfft
    L = 1.0
    dx = L / n
    rng = np.random.default_rng(seed)
    eta1 = _interface_height(n, rng, 0.01 * L)
    eta2 = _interface_height(n, rng, 0.01 * L)
    z = _centres(n, dx)[:, None, None]
    zlo = 0.25 * L + eta1[None]
    zhi = 0.75 * L + eta2[None]
    e = ALPHA_FLOOR
    alpha_w = e + (1 - 2 * e) * 0.5 * (np.tanh((z - zlo) / dx) - np.tanh((z - zhi) / dx))
    alpha_w = np.clip(alpha_w, e, 1 - e)

    # Gaussian random velocity field with E(k) ~ k^-2 on 1 <= |k| <= kmax,
    # solenoidal.  Coefficients are drawn only inside the |k_i| <= kmax box and
    # zero-padded to the n^3 spectrum before the inverse FFT.
    m = 2 * kmax + 1
    kb = np.concatenate([np.arange(0, kmax + 1), np.arange(-kmax, 0)]).astype(np.float32)
    KZ = kb[:, None, None]
    KY = kb[None, :, None]
    KX = np.arange(0, kmax + 1, dtype=np.float32)[None, None, :]
    kk = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    shell = (kk >= 1) & (kk <= kmax)
    amp = np.zeros_like(kk)
    amp[shell] = kk[shell] ** -2.0       # |u_hat| ~ sqrt(E(k) / k^2) ~ k^-2
    comps = []
    for _ in range(3):
        re = rng.standard_normal(kk.shape, dtype=np.float32)
        im = rng.standard_normal(kk.shape, dtype=np.float32)
        comps.append((re + 1j * im).astype(np.complex64) * amp)
    k2 = np.where(kk > 0, kk * kk, 1.0).astype(np.float32)
    dot = (KX * comps[0] + KY * comps[1] + KZ * comps[2]) / k2
    comps[0] -= KX * dot
    comps[1] -= KY * dot
    comps[2] -= KZ * dot
    zidx = np.concatenate([np.arange(0, kmax + 1), np.arange(n - kmax, n)])
    vel = []
    for cb in comps:
        full = np.zeros((n, n, n // 2 + 1), dtype=np.complex64)
        full[np.ix_(zidx, zidx, np.arange(kmax + 1))] = cb
        vel.append(sfft.irfftn(full, s=(n, n, n), axes=(0, 1, 2), workers=-1))
        del full
    assert m == zidx.size
    rms = math.sqrt(sum(float(np.mean(v * v)) for v in vel) / 3.0)
    c_air = math.sqrt(AIR["gamma"] * 1e5 / AIR["rho"])
    scale = mach_rms * c_air / rms
    for v in vel:
        v *= np.float32(scale)
    p = 1e5
    w = _two_fluid_w(alpha_w, WATER["rho"], AIR["rho"], vel, p)
    if dtype != np.float64:
        w = w.astype(dtype)
    return Case(f"periodic_slab_{n}", 3, (n, n, n), 2, (dx, dx, dx),
                (WATER["gamma"], AIR["gamma"]), (WATER["pi_inf"], AIR["pi_inf"]),
                (PERIODIC,) * 3, (PERIODIC,) * 3, w, steps=steps, cfl=0.5,
                extra=dict(seed=seed, u_rms=mach_rms * c_air))


# ----------------------------------------------------------------------------
# Generic randomized states for parity tests
# ----------------------------------------------------------------------------
def _smooth_field(rng, shape_zyx, ndim, nmodes=4, kmax=3):
    nz, ny, nx = shape_zyx
    axes = [(np.arange(nx) + 0.5) / nx, (np.arange(ny) + 0.5) / ny, (np.arange(nz) + 0.5) / nz]
    f = np.zeros(shape_zyx)
    for _ in range(nmodes):
        k = rng.integers(0, kmax + 1, size=3)
        k[ndim:] = 0
        ph = rng.uniform(0, 2 * np.pi, size=3)
        a = rng.uniform(-1, 1)
        fx = np.cos(2 * np.pi * k[0] * axes[0] + ph[0])[None, None, :]
        fy = np.cos(2 * np.pi * k[1] * axes[1] + ph[1])[None, :, None]
        fz = np.cos(2 * np.pi * k[2] * axes[2] + ph[2])[:, None, None]
        f += a * fx * fy * fz
    m = np.abs(f).max()
    return f / m if m > 0 else f


def random_case(ndim: int, n, nf: int = 2, seed: int = 0, bc=None, speed: float = 200.0,
                pressure_jump: float = 10.0, interface: bool = True) -> Case:
    """Randomized state that exercises every branch of the face solver.

    Two fluids: air bubble(s)/planes in water, smooth velocity of amplitude
    `speed`, a pressure jump of ratio `pressure_jump` across a random plane.
    One fluid: an ideal gas with density and pressure jumps; `speed` above
    the sound speed (~374 m/s) makes some faces supersonic.
    """
    rng = np.random.default_rng(seed)
    n3 = _pad3(tuple(int(v) for v in n), 1)
    nx, ny, nz = n3
    shape = (nz, ny, nx)
    dx = 1.0 / nx
    dx3 = (dx, dx if ndim > 1 else 1.0, dx if ndim > 2 else 1.0)
    axes = np.meshgrid((np.arange(nz) + 0.5) / nz, (np.arange(ny) + 0.5) / ny,
                       (np.arange(nx) + 0.5) / nx, indexing="ij")
    Z, Y, X = axes
    if ndim < 3:
        Z = np.zeros_like(Z)
    if ndim < 2:
        Y = np.zeros_like(Y)
    nrm = rng.normal(size=3)
    nrm[ndim:] = 0
    nrm /= np.linalg.norm(nrm)
    plane = nrm[0] * (X - 0.5) + nrm[1] * (Y - 0.5) + nrm[2] * (Z - 0.5) - rng.uniform(-0.2, 0.2)
    bc_tuple = _pad3(bc if bc is not None else (EXTRAP,) * 3, EXTRAP)
    if any(bc_tuple[d] == PERIODIC for d in range(ndim)):
        # a plane wrapped by a periodic axis leaves slots a few cells wide; use
        # a ball that stays clear of the boundaries instead
        cj = rng.uniform(0.4, 0.6, size=3)
        cj[ndim:] = 0
        plane = np.sqrt((X - cj[0]) ** 2 + (Y - cj[1]) ** 2 + (Z - cj[2]) ** 2) - 0.25
    jump = np.where(plane < 0, pressure_jump, 1.0)
    vel = [speed * _smooth_field(rng, shape, ndim) for _ in range(ndim)]
    if bc is None:
        bc = (EXTRAP, EXTRAP, EXTRAP)
    bc = _pad3(bc, EXTRAP)
    if nf == 2:
        c = rng.uniform(0.3, 0.7, size=3)
        c[ndim:] = 0
        R = rng.uniform(0.12, 0.25)
        dist = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) - R
        alpha_air = _tanh_fraction(dist, 1.5 * dx) if interface else np.full(shape, 0.3)
        alpha_w = 1.0 - alpha_air
        rho_w = WATER["rho"] * (1.0 + 0.05 * _smooth_field(rng, shape, ndim))
        rho_a = AIR["rho"] * (1.0 + 0.2 * _smooth_field(rng, shape, ndim))
        p = 1e5 * (1.0 + 0.3 * _smooth_field(rng, shape, ndim)) * jump
        w = _two_fluid_w(alpha_w, rho_w, rho_a, vel, p)
        gam, pi = (WATER["gamma"], AIR["gamma"]), (WATER["pi_inf"], AIR["pi_inf"])
    else:
        rho = 1.0 + 0.3 * _smooth_field(rng, shape, ndim) + np.where(plane < 0, 1.0, 0.0)
        p = 1e5 * (1.0 + 0.3 * _smooth_field(rng, shape, ndim)) * jump
        w = np.ascontiguousarray(np.stack([rho] + vel + [p]).astype(np.float64))
        gam, pi = (1.4, 1.4), (0.0, 0.0)
    return Case(f"random_{ndim}d_nf{nf}_s{seed}", ndim, n3, nf, dx3, gam, pi,
                bc, bc, w, cfl=0.5, extra=dict(seed=seed))


CONFIGS = {
    "C0": "1D Sod shock tube, 200 cells, to t=0.2",
    "C1": "2D shock-cylinder, 512x512, 500 steps, FP64",
    "C2": "3D bubble cloud, 256^3, 200 steps, FP64 and FP32 form",
    "C3": "adjoint on the shock-cylinder physics at 256x256, 200 steps",
    "C4": "3D periodic slab, 512^3, 100 steps, FP32 form vs FP64",
}


def gresho(n: int = 32, mach: float = 0.01, gamma: float = 1.4) -> Case:
    """Gresho vortex (the paper's low-Mach validation case): a stationary
    vortex of the incompressible Euler equations, u_theta = 5r (r < 0.2),
    2 - 5r (0.2 <= r < 0.4), 0 outside, with the pressure that balances it;
    rho = 1, ideal gas, background pressure p0 = 1/(gamma M^2) so that the
    peak speed 1 has Mach M.  Periodic unit square, n x n cells."""
    dx = 1.0 / n
    x = _centres(n, dx)
    X, Y = np.meshgrid(x, x, indexing="xy")
    dxc, dyc = X - 0.5, Y - 0.5
    r = np.hypot(dxc, dyc)
    ut = np.where(r < 0.2, 5.0 * r, np.where(r < 0.4, 2.0 - 5.0 * r, 0.0))
    p0 = 1.0 / (gamma * mach * mach)
    with np.errstate(divide="ignore"):
        p = np.where(r < 0.2, p0 + 12.5 * r * r,
                     np.where(r < 0.4, p0 + 12.5 * r * r + 4.0 - 20.0 * r + 4.0 * np.log(np.maximum(5.0 * r, 1e-300)),
                              p0 - 2.0 + 4.0 * np.log(2.0)))
    rs = np.where(r > 0, r, 1.0)
    u = -ut * dyc / rs
    v = ut * dxc / rs
    w = np.stack([np.ones_like(X), u, v, p]).reshape(4, 1, n, n)
    return Case("gresho", 2, (n, n, 1), 1, (dx, dx, 1.0), (gamma, gamma), (0.0, 0.0),
                (PERIODIC,) * 3, (PERIODIC,) * 3, w)
