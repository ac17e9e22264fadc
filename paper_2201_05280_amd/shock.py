"""Normal-shock set-up on the lattice: the model's own jump conditions.

Far from a steady shock the populations are the equilibrium of the local
state, so the fluxes that cross a plane per step are moments of that
equilibrium: mass sum F c_x, x momentum sum F c_x^2 and energy
sum F c_x c^2/2 plus the rotational part (delta/2) rho u theta carried by the
theta_R transport.  The first two equal rho u and rho (u^2 + theta) for F3 and
E2 alike; the energy flux is a third moment, which E2 (exact only up to the
second moments) carries with an error that grows with the Mach number.
`discrete_rankine_hugoniot` therefore solves the three flux balances with the
library's own equilibrium (Newton's method with a finite-difference Jacobian)
instead of the ideal-gas formulas, so that Dirichlet faces holding the two
states admit a stationary shock.
"""
import numpy as np

from . import _lib
from .inputs import THETA0, positions, rankine_hugoniot, uniform


_LATTICE = {}


def equilibrium_fluxes(rho, u, theta, delta, kind=_lib.E2, theta0=0.0):
    """(mass, x momentum, energy) fluxes of the equilibrium at (rho, u e_x, theta)."""
    if theta0 not in _LATTICE:
        _LATTICE[theta0] = _lib.lattice(theta0)
    c, _ = _LATTICE[theta0]
    F = _lib.equilibrium(kind, rho, (u, 0.0, 0.0), (theta, theta, theta, 0.0, 0.0, 0.0), theta0)
    cx, c2 = c[:, 0], (c ** 2).sum(1)
    return np.array([F @ cx, F @ cx ** 2, 0.5 * F @ (cx * c2) + 0.5 * delta * rho * u * theta])


def discrete_rankine_hugoniot(Ma, delta, theta1=THETA0, kind=_lib.E2, tol=1e-13, maxit=50):
    """Upstream state (rho 1, Ma c_s, theta1) and the downstream state with equal
    equilibrium fluxes, started from the ideal-gas jump of gamma = (5+delta)/(3+delta)."""
    gamma = (5.0 + delta) / (3.0 + delta)
    up, down = rankine_hugoniot(Ma, gamma, theta1)
    target = equilibrium_fluxes(*up, delta, kind)
    x = np.array(down, dtype=np.float64)
    for _ in range(maxit):
        r = equilibrium_fluxes(*x, delta, kind) - target
        if np.abs(r).max() <= tol * np.abs(target).max():
            return up, tuple(float(v) for v in x)
        J = np.empty((3, 3))
        for j in range(3):
            h = 1e-7 * max(abs(x[j]), 1e-3)
            xp = x.copy()
            xp[j] += h
            J[:, j] = (equilibrium_fluxes(*xp, delta, kind) - target - r) / h
        x = x - np.linalg.solve(J, r)
    raise ValueError("no downstream state found for Ma %g" % Ma)


def tanh_profile(L, up, down, width=4.0, x0=None):
    """Line of L cells blending the two states with a tanh of the given width."""
    x = positions(L, 1, 1)[0]
    x0 = L / 2 if x0 is None else x0
    sm = 0.5 * (1 + np.tanh((x - x0) / width))
    f = uniform(L, 1, 1)
    f["rho"] = up[0] + (down[0] - up[0]) * sm
    f["u"][0] = up[1] + (down[1] - up[1]) * sm
    f["thT"] = up[2] + (down[2] - up[2]) * sm
    f["thR"] = f["thT"].copy()
    return f


def profile_metrics(x, rho, up, down):
    """Shock position (where rho crosses the mean of the two densities) and
    maximum-slope thickness (rho2 - rho1) / max |d rho / dx|, in cells."""
    o = np.argsort(x)
    xs, rs = x[o], rho[o]
    mid = 0.5 * (up[0] + down[0])
    k = int(np.argmax(rs > mid))
    pos = xs[k - 1] + (mid - rs[k - 1]) / (rs[k] - rs[k - 1]) * (xs[k] - xs[k - 1]) if k > 0 else float("nan")
    slope = np.abs(np.diff(rs) / np.diff(xs)).max()
    return float(pos), float((down[0] - up[0]) / slope)
