"""Shared test helpers (no method arithmetic here)."""
import numpy as np

EPS = np.finfo(np.float64).eps


def field_errors(a, b):
    """Per-row max-relative L-infinity error: max|a - b| / max|b| for every row."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = []
    for v in range(b.shape[0]):
        den = np.abs(b[v]).max()
        num = np.abs(a[v] - b[v]).max()
        out.append(0.0 if num == 0 else (num / den if den > 0 else np.inf))
    return np.array(out)


def conservative_errors(a, b, nf, ndim, zero_mom=()):
    """Max-relative L-infinity error per conservative row, max|a - b| / max|b|.

    One entry per row: each partial density, each momentum component, the
    energy, each volume fraction.  Every momentum component is measured on its
    own scale, except the components listed in ``zero_mom``: those are zero in
    exact arithmetic for the flow at hand (a planar wave, or a fluid at rest in
    uniform pressure, has no momentum across it), so both sides carry only
    rounding noise there, and such a component is measured on the scale of the
    whole momentum vector, max over cells of |rho u|.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = field_errors(a, b)
    m = slice(nf, nf + ndim)
    vec = np.sqrt((b[m] ** 2).sum(axis=0)).max()
    for d in zero_mom:
        num = np.abs(a[nf + d] - b[nf + d]).max()
        out[nf + d] = 0.0 if num == 0 else (num / vec if vec > 0 else np.inf)
    return out


def grouped_errors(a, b, nf, ndim):
    """Max-relative L-infinity error per conservative field with the momentum
    taken as one vector (|d(rho u)| over cells divided by the largest
    |rho u|): the grouping of the FP32 error envelopes, whose momentum bound is
    derived for the vector."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = []
    for i in range(nf):
        out.append(field_errors(a[i:i + 1], b[i:i + 1])[0])
    m = slice(nf, nf + ndim)
    den = np.sqrt((b[m] ** 2).sum(axis=0)).max()
    num = np.sqrt(((a[m] - b[m]) ** 2).sum(axis=0)).max()
    out.append(0.0 if num == 0 else (num / den if den > 0 else np.inf))
    for r in range(nf + ndim, b.shape[0]):
        out.append(field_errors(a[r:r + 1], b[r:r + 1])[0])
    return np.array(out)


def field_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = []
    for v in range(b.shape[0]):
        den = np.linalg.norm(b[v].ravel())
        num = np.linalg.norm((a[v] - b[v]).ravel())
        out.append(0.0 if num == 0 else (num / den if den > 0 else np.inf))
    return np.array(out)


def noise_floor(fn, q, trials=3, seed=5):
    """Per-row spread of fn when q is perturbed by one unit in the last place.

    Two correct float64 evaluations of an ill-conditioned map (here: WENO-JS
    derivatives, whose weights react strongly to rounding-level data) cannot
    agree better than this spread; adjoint parity is measured against it.
    """
    base = fn(q)
    rng = np.random.default_rng(seed)
    spread = np.zeros(base.shape[0])
    for _ in range(trials):
        qp = q * (1.0 + rng.choice([-1.0, 0.0, 1.0], size=q.shape) * EPS)
        spread = np.maximum(spread, field_errors(fn(qp), base))
    return base, spread


def rate_errors(a, b, q, smax, nf, ndim, mom_rate=None):
    """RHS error per conservative field on the scale of the field's fastest rate.

    A right-hand side is a difference of face fluxes; its rounding error is
    relative to the fluxes, |F_v| <= |q_v| (|u| + c), not to the difference,
    which is pure rounding noise wherever the exact RHS vanishes (fluid at rest
    in uniform pressure).  Scale: max|q_v| * s_max with s_max = max over cells
    of sum_d (|u_d| + c)/dx_d.  Momentum is one vector field; its flux also
    carries the pressure, so for a state at rest (zero momentum) the caller
    passes the momentum scale, e.g. max p / dx, as ``mom_rate``.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    out = []
    for i in range(nf):
        out.append(np.abs(a[i] - b[i]).max() / (np.abs(q[i]).max() * smax))
    m = slice(nf, nf + ndim)
    num = np.sqrt(((a[m] - b[m]) ** 2).sum(axis=0)).max()
    den = np.sqrt((q[m] ** 2).sum(axis=0)).max() * smax if mom_rate is None else mom_rate
    out.append(num / den)
    for r in range(nf + ndim, b.shape[0]):
        out.append(np.abs(a[r] - b[r]).max() / (np.abs(q[r]).max() * smax))
    return np.array(out)
