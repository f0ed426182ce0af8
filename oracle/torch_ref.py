"""Plain PyTorch float64 version of the five-equation RHS -- TEST ONLY.

It runs on the CPU; the adjoint test at the configuration's full size runs it
on a GPU with torch's own kernels (nothing here depends on the device).

The same discretization as ``oracle.c`` (same readings, same expression
order) written with whole-array torch operations so that autograd yields
reference gradients: the vector-Jacobian product of the RHS, of an SSP-RK3
step and of a whole rollout.  Branches (wave-speed min/max, HLLC regions) are
``torch.where`` selections, so a derivative follows the branch the forward
pass takes; min/max ties go to the first argument as in the oracle.

Layout: q[v, k, j, i] (x fastest); rows as in ``oracle.c``.
"""
from __future__ import annotations

import numpy as np
import torch

PERIODIC, EXTRAP, SLIPWALL = 0, 1, 2


class _Sqrt(torch.autograd.Function):
    """Correctly rounded square root (numpy's) with its derivative.

    torch's CPU sqrt kernel may differ from the correctly rounded result by
    one unit in the last place; the C oracle uses the correctly rounded one.
    """

    @staticmethod
    def forward(ctx, x):
        y = torch.from_numpy(np.asarray(np.sqrt(x.detach().cpu().numpy()))).to(x.device)
        ctx.save_for_backward(y)
        return y

    @staticmethod
    def backward(ctx, g):
        (y,) = ctx.saved_tensors
        return g / (2.0 * y)


def sqrt(x):
    return _Sqrt.apply(x)


class Problem:
    def __init__(self, ndim, n, num_fluids, dx, gamma, pi_inf, bc_lo, bc_hi, weno_eps=1e-6, weno_variant=0,
                 riemann=0, low_mach=0, model=0, faces=None):
        if faces is not None and any(f is not None for f in faces):
            raise NotImplementedError("the torch reference covers uniform grids only")
        self.ndim = ndim
        self.n = tuple(n) + (1,) * (3 - len(n))
        self.nf = num_fluids
        self.dx = tuple(dx) + (1.0,) * (3 - len(dx))
        self.gamma = tuple(gamma)
        self.pi_inf = tuple(pi_inf)
        self.bc_lo = tuple(bc_lo) + (EXTRAP,) * (3 - len(bc_lo))
        self.bc_hi = tuple(bc_hi) + (EXTRAP,) * (3 - len(bc_hi))
        self.eps = weno_eps
        self.weno_variant = int(weno_variant)
        self.riemann = int(riemann)
        self.low_mach = int(low_mach)
        self.model = int(model)
        self.neq = self.nf + ndim + 1 + (2 if self.nf == 2 else 0)
        self.G = [1.0 / (g - 1.0) for g in self.gamma]
        self.P = [g * p / (g - 1.0) for g, p in zip(self.gamma, self.pi_inf)]

    @classmethod
    def from_case(cls, case):
        return cls(**case.problem_kwargs())

    def row_mom(self, d):
        return self.nf + d

    @property
    def row_E(self):
        return self.nf + self.ndim

    def row_alpha(self, i):
        return self.nf + self.ndim + 1 + i


# tensor axis of the grid direction d in q[v, z, y, x]
def _axis(d):
    return 3 - d


def mixture(P: Problem, alpha):
    if P.nf == 1:
        return P.G[0], P.P[0]
    Gam = alpha[0] * P.G[0] + alpha[1] * P.G[1]
    Pi = alpha[0] * P.P[0] + alpha[1] * P.P[1]
    return Gam, Pi


def cons_to_prim(P: Problem, q):
    nf, D = P.nf, P.ndim
    rho = q[0] if nf == 1 else q[0] + q[1]
    if nf == 1:
        rho = 0.0 + q[0]
    vel = [q[P.row_mom(d)] / rho for d in range(D)]
    usq = 0.0
    for u in vel:
        usq = usq + u * u
    alpha = [q[P.row_alpha(i)] for i in range(2)] if nf == 2 else None
    Gam, Pi = mixture(P, alpha)
    ke = 0.5 * rho * usq
    p = (q[P.row_E] - ke - Pi) / Gam
    rows = [q[i] for i in range(nf)] + vel + [p] + (alpha if nf == 2 else [])
    return torch.stack(rows)


def prim_to_cons(P: Problem, w):
    nf, D = P.nf, P.ndim
    rho = 0.0 + w[0] if nf == 1 else w[0] + w[1]
    usq = 0.0
    mom = []
    for d in range(D):
        u = w[P.row_mom(d)]
        mom.append(rho * u)
        usq = usq + u * u
    alpha = [w[P.row_alpha(i)] for i in range(2)] if nf == 2 else None
    Gam, Pi = mixture(P, alpha)
    ke = 0.5 * rho * usq
    E = Gam * w[P.row_E] + Pi + ke
    rows = [w[i] for i in range(nf)] + mom + [E] + (alpha if nf == 2 else [])
    return torch.stack(rows)


def pad_axis(P: Problem, q, d):
    """Three ghost layers on both sides of grid axis d (Sec. 3.3)."""
    n = P.n[d]
    ax = _axis(d)
    idx = torch.arange(-3, n + 3)
    flip = torch.zeros(n + 6, dtype=torch.bool)
    lo, hi = P.bc_lo[d], P.bc_hi[d]
    m = idx.clone()
    low, high = idx < 0, idx >= n
    if lo == PERIODIC:
        m[low] = idx[low] + n
    elif lo == EXTRAP:
        m[low] = 0
    else:
        m[low] = -1 - idx[low]
        flip[low] = True
    if hi == PERIODIC:
        m[high] = idx[high] - n
    elif hi == EXTRAP:
        m[high] = n - 1
    else:
        m[high] = 2 * n - 1 - idx[high]
        flip[high] = True
    qp = torch.index_select(q, ax, m.to(q.device))
    if flip.any():
        shape = [1, 1, 1, 1]
        shape[ax] = n + 6
        sign = torch.where(flip, -1.0, 1.0).to(dtype=q.dtype, device=q.device).reshape(shape)
        r = P.row_mom(d)
        qp = torch.cat([qp[:r], qp[r:r + 1] * sign, qp[r + 1:]], dim=0)
    return qp


def _sl(t, ax, start, length):
    return t.narrow(ax, start, length)


def weno5_js_left(a, b, c, d, e, eps):
    q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0
    q1 = (-b + 5.0 * c + 2.0 * d) / 6.0
    q2 = (2.0 * c + 5.0 * d - e) / 6.0
    b0 = 13.0 / 12.0 * ((a + c) - 2.0 * b) ** 2 + 0.25 * ((a + 3.0 * c) - 4.0 * b) ** 2
    b1 = 13.0 / 12.0 * ((b + d) - 2.0 * c) ** 2 + 0.25 * (b - d) ** 2
    b2 = 13.0 / 12.0 * ((c + e) - 2.0 * d) ** 2 + 0.25 * ((3.0 * c + e) - 4.0 * d) ** 2
    # scalar / tensor in torch multiplies by a reciprocal; divide tensor by tensor
    a0 = torch.full_like(b0, 0.1) / (eps + b0) ** 2
    a1 = torch.full_like(b1, 0.6) / (eps + b1) ** 2
    a2 = torch.full_like(b2, 0.3) / (eps + b2) ** 2
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2)


def weno5_z_left(a, b, c, d, e, eps):
    """WENO5-Z (Sec. 4.2.2): tau = |beta_0 - beta_2|, a_k = d_k (1 + tau/(beta_k + eps)), q = 1."""
    q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0
    q1 = (-b + 5.0 * c + 2.0 * d) / 6.0
    q2 = (2.0 * c + 5.0 * d - e) / 6.0
    b0 = 13.0 / 12.0 * ((a + c) - 2.0 * b) ** 2 + 0.25 * ((a + 3.0 * c) - 4.0 * b) ** 2
    b1 = 13.0 / 12.0 * ((b + d) - 2.0 * c) ** 2 + 0.25 * (b - d) ** 2
    b2 = 13.0 / 12.0 * ((c + e) - 2.0 * d) ** 2 + 0.25 * ((3.0 * c + e) - 4.0 * d) ** 2
    tau = torch.abs(b0 - b2)
    a0 = 0.1 * (1.0 + tau / (b0 + eps))
    a1 = 0.6 * (1.0 + tau / (b1 + eps))
    a2 = 0.3 * (1.0 + tau / (b2 + eps))
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2)


TENO_CT = 1e-5


def teno5_left(a, b, c, d, e, eps, ct=TENO_CT):
    """TENO5 (Sec. 4.2.2): stencils whose share of gamma_r = d_r (1 + tau/(beta_r + eps))^6
    reaches ct combine with their linear weights; the weights are piecewise constant."""
    q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0
    q1 = (-b + 5.0 * c + 2.0 * d) / 6.0
    q2 = (2.0 * c + 5.0 * d - e) / 6.0
    b0 = 13.0 / 12.0 * ((a + c) - 2.0 * b) ** 2 + 0.25 * ((a + 3.0 * c) - 4.0 * b) ** 2
    b1 = 13.0 / 12.0 * ((b + d) - 2.0 * c) ** 2 + 0.25 * (b - d) ** 2
    b2 = 13.0 / 12.0 * ((c + e) - 2.0 * d) ** 2 + 0.25 * ((3.0 * c + e) - 4.0 * d) ** 2
    tau = torch.abs(b0 - b2)
    p6 = lambda x: (x * x) * (x * x) * (x * x)
    g0 = 0.1 * p6(1.0 + tau / (b0 + eps))
    g1 = 0.6 * p6(1.0 + tau / (b1 + eps))
    g2 = 0.3 * p6(1.0 + tau / (b2 + eps))
    gs = g0 + g1 + g2
    zero = torch.zeros_like(b0)
    w0 = torch.where(g0 / gs >= ct, zero + 0.1, zero).detach()
    w1 = torch.where(g1 / gs >= ct, zero + 0.6, zero).detach()
    w2 = torch.where(g2 / gs >= ct, zero + 0.3, zero).detach()
    return (w0 * q0 + w1 * q1 + w2 * q2) / (w0 + w1 + w2)


def weno5_m_left(a, b, c, d, e, eps):
    """WENO5-M (Sec. 3.2.1, Henrick-Aslam-Powers mapping of the JS weights)."""
    q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0
    q1 = (-b + 5.0 * c + 2.0 * d) / 6.0
    q2 = (2.0 * c + 5.0 * d - e) / 6.0
    b0 = 13.0 / 12.0 * ((a + c) - 2.0 * b) ** 2 + 0.25 * ((a + 3.0 * c) - 4.0 * b) ** 2
    b1 = 13.0 / 12.0 * ((b + d) - 2.0 * c) ** 2 + 0.25 * (b - d) ** 2
    b2 = 13.0 / 12.0 * ((c + e) - 2.0 * d) ** 2 + 0.25 * ((3.0 * c + e) - 4.0 * d) ** 2
    a0 = torch.full_like(b0, 0.1) / (eps + b0) ** 2
    a1 = torch.full_like(b1, 0.6) / (eps + b1) ** 2
    a2 = torch.full_like(b2, 0.3) / (eps + b2) ** 2
    s = a0 + a1 + a2

    def g(w, dk):
        return w * (dk + dk * dk - 3.0 * dk * w + w * w) / (dk * dk + w * (1.0 - 2.0 * dk))

    m0, m1, m2 = g(a0 / s, 0.1), g(a1 / s, 0.6), g(a2 / s, 0.3)
    return (m0 * q0 + m1 * q1 + m2 * q2) / (m0 + m1 + m2)


def _min_first(a, b):
    return torch.where(a <= b, a, b)


def _max_first(a, b):
    return torch.where(a >= b, a, b)


def _face_side(P: Problem, d, W):
    """Face-side quantities of a reconstructed state: rho, u_n, p, E, c, U, F."""
    nf, D = P.nf, P.ndim
    rho = 0.0 + W[0] if nf == 1 else W[0] + W[1]
    usq = 0.0
    for e in range(D):
        usq = usq + W[P.row_mom(e)] * W[P.row_mom(e)]
    alpha = [W[P.row_alpha(i)] for i in range(2)] if nf == 2 else None
    Gam, Pi = mixture(P, alpha)
    p = W[P.row_E]
    un = W[P.row_mom(d)]
    E = Gam * p + Pi + 0.5 * rho * usq
    c2 = ((Gam + 1.0) * p + Pi) / (Gam * rho)
    c = sqrt(c2)
    U, F = [], []
    for i in range(nf):
        U.append(W[i])
        F.append(W[i] * un)
    for e in range(D):
        m = rho * W[P.row_mom(e)]
        U.append(m)
        F.append(m * un + p if e == d else m * un + 0.0)
    U.append(E)
    F.append((E + p) * un)
    return dict(rho=rho, un=un, p=p, E=E, c=c, c2=c2, U=U, F=F)


def hllc(P: Problem, d, WL, WR):
    """HLLC flux of every row and the face velocity, arrays over faces."""
    nf, D = P.nf, P.ndim
    L, R = _face_side(P, d, WL), _face_side(P, d, WR)
    SL = _min_first(L["un"] - L["c"], R["un"] - R["c"])
    SR = _max_first(L["un"] + L["c"], R["un"] + R["c"])
    Sstar = (R["p"] - L["p"] + L["rho"] * L["un"] * (SL - L["un"]) - R["rho"] * R["un"] * (SR - R["un"])) / (
        L["rho"] * (SL - L["un"]) - R["rho"] * (SR - R["un"]))

    def star_flux(W, s, SK):
        chi = (SK - s["un"]) / (SK - Sstar)
        Us = [chi * W[i] for i in range(nf)]
        for e in range(D):
            Us.append(chi * s["rho"] * Sstar if e == d else chi * s["rho"] * W[P.row_mom(e)])
        Us.append(chi * (s["E"] + (Sstar - s["un"]) * (s["rho"] * Sstar + s["p"] / (SK - s["un"]))))
        return [s["F"][v] + SK * (Us[v] - s["U"][v]) for v in range(len(Us))]

    FLs = star_flux(WL, L, SL)
    FRs = star_flux(WR, R, SR)
    if P.low_mach == 2:
        # anti-dissipation pressure correction of Chen et al. (Sec. 4.2.4) on
        # both star-region fluxes
        mL = torch.abs(L["un"]) / L["c"]
        mR = torch.abs(R["un"]) / R["c"]
        z = torch.where(mL >= mR, mL, mR)
        z = torch.where(z > 1.0, torch.ones_like(z), z)
        pd = L["rho"] * R["rho"] * (SL - L["un"]) * (SR - R["un"]) * (R["un"] - L["un"]) / (
            R["rho"] * (SR - R["un"]) - L["rho"] * (SL - L["un"]))
        apc_mom = (z - 1.0) * pd
        apc_E = (z - 1.0) * pd * Sstar
        m, e = P.row_mom(d), P.row_E
        FLs[m], FRs[m] = FLs[m] + apc_mom, FRs[m] + apc_mom
        FLs[e], FRs[e] = FLs[e] + apc_E, FRs[e] + apc_E
    c1 = SL >= 0.0
    c2 = Sstar >= 0.0
    c3 = SR > 0.0
    F = []
    for v in range(nf + D + 1):
        F.append(torch.where(c1, L["F"][v], torch.where(c2, FLs[v], torch.where(c3, FRs[v], R["F"][v]))))
    uf = torch.where(c1, L["un"], torch.where(c2 | c3, Sstar, R["un"]))
    if nf == 2:
        left_side = c1 | c2
        for i in range(2):
            a = P.row_alpha(i)
            F.append(torch.where(left_side, WL[a], WR[a]) * uf)
    return torch.stack(F), uf, (L["c2"], R["c2"])


def thornber(P: Problem, d, WL, WR):
    """Thornber et al. low-Mach correction of the face-normal velocities (the
    form printed in the paper's low-Mach section), sound speeds of the
    uncorrected states."""
    L, R = _face_side(P, d, WL), _face_side(P, d, WR)
    mL = torch.abs(L["un"]) / L["c"]
    mR = torch.abs(R["un"]) / R["c"]
    z = torch.where(mL >= mR, mL, mR)
    z = torch.where(z > 1.0, torch.ones_like(z), z)
    r = P.row_mom(d)
    uL, uR = WL[r], WR[r]
    uLs = 0.5 * (uL + uR) + z * (0.5 * (uL - uR))
    uRs = 0.5 * (uL + uR) + z * (0.5 * (uR - uL))
    WL = torch.cat([WL[:r], uLs.unsqueeze(0), WL[r + 1:]], dim=0)
    WR = torch.cat([WR[:r], uRs.unsqueeze(0), WR[r + 1:]], dim=0)
    return WL, WR


def hll(P: Problem, d, WL, WR):
    """HLL flux (Sec. 3.2.2): two waves, one averaged state; the volume
    fractions take the same formula on alpha u_n and the face velocity is the
    matching average (S_R u_L - S_L u_R)/(S_R - S_L)."""
    nf, D = P.nf, P.ndim
    L, R = _face_side(P, d, WL), _face_side(P, d, WR)
    SL = _min_first(L["un"] - L["c"], R["un"] - R["c"])
    SR = _max_first(L["un"] + L["c"], R["un"] + R["c"])
    den = SR - SL
    c1 = SL >= 0.0
    c4 = SR <= 0.0
    F = []
    for v in range(nf + D + 1):
        Fm = (SR * L["F"][v] - SL * R["F"][v] + SL * SR * (R["U"][v] - L["U"][v])) / den
        F.append(torch.where(c1, L["F"][v], torch.where(c4, R["F"][v], Fm)))
    um = (SR * L["un"] - SL * R["un"]) / den
    uf = torch.where(c1, L["un"], torch.where(c4, R["un"], um))
    if nf == 2:
        for i in range(2):
            a = P.row_alpha(i)
            aL, aR = WL[a], WR[a]
            Fm = (SR * aL * L["un"] - SL * aR * R["un"] + SL * SR * (aR - aL)) / den
            F.append(torch.where(c1, aL * L["un"], torch.where(c4, aR * R["un"], Fm)))
    return torch.stack(F), uf, (L["c2"], R["c2"])


def axis_contribution(P: Problem, q, d):
    """D_d of eq. eqn:rhs for every cell (see oracle.c)."""
    n = P.n[d]
    ax = _axis(d)
    qp = pad_axis(P, q, d)
    wp = cons_to_prim(P, qp)
    # faces m - 1/2, m = 0..n; padded index of cell g is g + 3
    fl = [_sl(wp, ax, s, n + 1) for s in range(5)]       # centre m-1: cells m-3..m+1
    fr = [_sl(wp, ax, s + 1, n + 1) for s in range(5)]   # centre m: cells m-2..m+2
    weno = {0: weno5_js_left, 1: weno5_z_left, 2: teno5_left, 3: weno5_m_left}[P.weno_variant]
    WL = weno(fl[0], fl[1], fl[2], fl[3], fl[4], P.eps)
    WR = weno(fr[4], fr[3], fr[2], fr[1], fr[0], P.eps)
    if P.low_mach == 1:
        WL, WR = thornber(P, d, WL, WR)
    F, uf, _ = (hll if P.riemann == 1 else hllc)(P, d, WL, WR)
    inv_dx = 1.0 / P.dx[d]
    Flo, Fhi = _sl(F, ax, 0, n), _sl(F, ax, 1, n)
    Dv = inv_dx * (Flo - Fhi)
    if P.nf == 2:
        ulo, uhi = _sl(uf, ax - 1, 0, n), _sl(uf, ax - 1, 1, n)
        K = kapila_K(P, cons_to_prim(P, q)) if P.model == 1 else None
        rows = []
        for v in range(P.neq):
            if v >= P.row_alpha(0):
                if K is None:
                    rows.append(Dv[v] + q[v] * (inv_dx * (uhi - ulo)))
                else:
                    Ki = K if v == P.row_alpha(0) else -K
                    rows.append(Dv[v] + (q[v] + Ki) * (inv_dx * (uhi - ulo)))
            else:
                rows.append(Dv[v])
        Dv = torch.stack(rows)
    return Dv


def kapila_K(P: Problem, w):
    """Kapila's K of the alpha_1 equation (Sec. 2.1.1, difference in the
    numerator) from primitive cell states w; alpha_2 takes -K."""
    p = w[P.row_E]
    rc2 = []
    for i in range(2):
        rho_i = w[i] / w[P.row_alpha(i)]
        c2_i = P.gamma[i] * (p + P.pi_inf[i]) / rho_i
        rc2.append(rho_i * c2_i)
    return (rc2[1] - rc2[0]) / (rc2[0] / w[P.row_alpha(0)] + rc2[1] / w[P.row_alpha(1)])


def rhs(P: Problem, q):
    out = None
    for d in range(P.ndim):
        Dv = axis_contribution(P, q, d)
        out = Dv if out is None else out + Dv
    return out


def max_signal(P: Problem, q):
    w = cons_to_prim(P, q)
    rho = 0.0 + q[0] if P.nf == 1 else q[0] + q[1]
    alpha = [q[P.row_alpha(i)] for i in range(2)] if P.nf == 2 else None
    Gam, Pi = mixture(P, alpha)
    c = sqrt(((Gam + 1.0) * w[P.row_E] + Pi) / (Gam * rho))
    s = 0.0
    for d in range(P.ndim):
        s = s + (torch.abs(w[P.row_mom(d)]) + c) * (1.0 / P.dx[d])
    return s.max()


def step(P: Problem, q, dt):
    L0 = rhs(P, q)
    q1 = q + dt * L0
    L1 = rhs(P, q1)
    q2 = 0.75 * q + 0.25 * (q1 + dt * L1)
    L2 = rhs(P, q2)
    return (1.0 / 3.0) * q + (2.0 / 3.0) * (q2 + dt * L2)
