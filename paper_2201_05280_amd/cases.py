"""Seeded 1D case generator for the batched sweep and the learned warm start.

Two kinds of case: Couette layers (F3) and normal-shock lines (E2).

Couette layers between two diffuse walls (Sec. 6 runs start-up and thermal
Couette flows): the low wall at rest, the high wall moving tangentially (y)
at Ma_w c_s, both at theta0.  Knudsen number Kn = nu/(c_s L) (the reading
under which the Landau formula of Sec. 6 matches the sound-diffusion law),
so nu = Kn c_s L.  Draws: L ~ U{Lmin..Lmax}, Ma_w ~ U[Ma range],
Kn ~ logU[Kn range], delta ~ {2, 3}, and the pair Pr ~ U[Pr range],
mu_b/mu ~ U[mub range] redrawn together while it is out of the model's reach
(mu_b/mu at or below 1.02 times the floor 2 delta/(3(3+delta)), or no
feasible (b, k_r) for it).

Shock lines: upstream (rho 1, Ma c_s, theta1) at the low face, the model's
own downstream state (equal equilibrium fluxes) at the high face, flow along
+x; Ma ~ U[shock Ma range], Kn = lambda1 / L with the upstream mean free path
lambda1 = nu sqrt(pi / (2 theta1)), Kn ~ logU[shock Kn range]; same Pr,
mu_b/mu and delta draws.  The upstream temperature theta1 is theta0 when the
E2 equilibrium has both jump states there; above about Mach 2.65 the upstream
speed Ma sqrt(gamma theta0) is beyond the lattice, and theta1 is the warmest
temperature on a grid from 0.12 down to 0.04 (steps of 0.005) at which both
states exist (a colder gas crosses the lattice at a lower speed).  A draw
with no such temperature is infeasible: it is counted and drawn again.
Their cold start is the tanh blend of the two states (width 4 cells) centred
at L/2.

Network features (all O(1)): x/L, 2 ln(Ma/0.3), (Pr - 0.835)/0.165,
(mu_b/mu - 1), log10 Kn + 2, (delta - 2.5)/0.5.  Targets, Couette:
(rho - 1)/U^2, u_y/U, (theta_T - theta0)/U^2, (theta_R - theta0)/U^2 with U the
wall speed; shock: each field scaled to run from 0 upstream to 1 downstream,
(phi - phi1)/(phi2 - phi1) for rho, u_x, theta_T, theta_R.
"""
import math

import numpy as np

from . import _lib
from .inputs import THETA0, positions

COUETTE = "couette"
SHOCK = "shock"


_THETA1 = {}


def shock_upstream_theta(Ma, delta):
    """(theta1, upstream, downstream) for a shock of Mach Ma: theta1 = theta0
    when both jump states have an E2 equilibrium there, else the warmest
    theta1 from 0.12 down to 0.04 (steps of 0.005) that has them; None when
    none has."""
    from .shock import discrete_rankine_hugoniot
    key = (round(Ma, 12), delta)
    if key not in _THETA1:
        found = None
        for th1 in [THETA0] + [0.12 - 0.005 * i for i in range(17)]:
            try:
                up, down = discrete_rankine_hugoniot(Ma, delta, th1)
                # both faces need an E2 state of their own temperature
                _lib.equilibrium(_lib.E2, up[0], (up[1], 0, 0), (up[2],) * 3 + (0, 0, 0))
                _lib.equilibrium(_lib.E2, down[0], (down[1], 0, 0), (down[2],) * 3 + (0, 0, 0))
                found = (th1, up, down)
                break
            except (ValueError, np.linalg.LinAlgError):
                continue
        _THETA1[key] = found
    return _THETA1[key]


def sweep_cases(n, seed, L_range=(256, 1024), Ma_range=(0.1, 0.5), Kn_range=(3e-3, 3e-2),
                Pr_range=(0.67, 1.0), mub_range=(0.0, 2.0), deltas=(2.0, 3.0), shock_fraction=0.0,
                shock_Ma_range=(1.1, 2.0), shock_Kn_range=(2e-3, 1e-2), counts=None):
    """n seeded cases (a shock with probability shock_fraction) and the number
    of infeasible (Pr, mu_b/mu) draws that were redrawn.  `counts` (a dict,
    optional) receives the shock draws with no jump states on the lattice
    (redrawn) and those that needed an upstream temperature below theta0."""
    rng = np.random.default_rng(seed)
    out = []
    redraws = 0
    if counts is not None:
        counts.update(shock_no_states=0, shock_cold_upstream=0)
    for _ in range(n):
        kind = SHOCK if rng.uniform() < shock_fraction else COUETTE
        L = int(rng.integers(L_range[0], L_range[1] + 1))
        ma_r, kn_r = (shock_Ma_range, shock_Kn_range) if kind == SHOCK else (Ma_range, Kn_range)
        delta = float(deltas[int(rng.integers(0, len(deltas)))])
        th1, states = THETA0, None
        while True:
            Ma = float(rng.uniform(*ma_r))
            if kind == COUETTE:
                break
            states = shock_upstream_theta(Ma, delta)
            if states is not None:
                th1 = states[0]
                if counts is not None and th1 != THETA0:
                    counts["shock_cold_upstream"] += 1
                break
            if counts is not None:
                counts["shock_no_states"] += 1
        Kn = float(10 ** rng.uniform(math.log10(kn_r[0]), math.log10(kn_r[1])))
        floor = 2 * delta / (3 * (3 + delta)) * 1.02
        gamma = (5 + delta) / (3 + delta)
        cs = math.sqrt(gamma * THETA0)
        nu = Kn * cs * L if kind == COUETTE else Kn * L / math.sqrt(math.pi / (2 * th1))
        while True:
            # (Pr, mu_b/mu) pairs outside the model's reach (bulk viscosity at
            # or below the floor, or no b in [-1/2, 1) with k_r >= 0) are redrawn
            Pr = float(rng.uniform(*Pr_range))
            mub = float(rng.uniform(*mub_range))
            if mub > floor:
                try:
                    # the map takes nu at theta0; the shock's nu is the upstream one,
                    # and nu grows like theta at fixed relaxation times
                    p = _lib.resolve(nu * THETA0 / th1, Pr, mub, delta)
                    break
                except ValueError:
                    pass
            redraws += 1
        c = dict(kind=kind, L=L, Ma=Ma, Kn=Kn, Pr=Pr, mub=mub, delta=delta, nu=nu, U=Ma * cs, params=p)
        if kind == SHOCK:
            c["theta1"], c["up"], c["down"] = states
        out.append(c)
    return out, redraws


def to_batch_cases(cases, variant=0):
    from .batch import make_case
    res = []
    for c in cases:
        p = c["params"]
        pp = (p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
        if c["kind"] == SHOCK:
            up, dn = c["up"], c["down"]
            res.append(make_case(c["L"], _lib.DIRICHLET, pp, rho=(up[0], dn[0]), u=((up[1], 0, 0), (dn[1], 0, 0)),
                                 theta=(up[2], dn[2]), vel_axis=0, variant=variant, equilibrium=_lib.E2))
        else:
            res.append(make_case(c["L"], _lib.WALL, pp, u=((0, 0, 0), (0, c["U"], 0)), theta=(THETA0, THETA0),
                                 vel_axis=1, variant=variant))
    return res


def cold_fields(cases):
    """Cold starts concatenated over sites: Couette, uniform gas at rest at
    theta0; shock, the tanh blend of its two states."""
    from .shock import tanh_profile
    parts = []
    for c in cases:
        if c["kind"] == SHOCK:
            parts.append(tanh_profile(c["L"], c["up"], c["down"]))
        else:
            ns = 2 * c["L"]
            parts.append(dict(rho=np.ones(ns), u=np.zeros((3, ns)), thT=np.full(ns, THETA0), thR=np.full(ns, THETA0)))
    return {k: np.concatenate([f[k] for f in parts], axis=-1) for k in ("rho", "u", "thT", "thR")}


def features(cases):
    """[ns_total][6] float32 network inputs, site order of the batch."""
    rows = []
    for c in cases:
        x = positions(c["L"], 1, 1)[0]
        # walls at -1/4 and L - 1/4
        xl = (x + 0.25) / c["L"]
        f = np.empty((x.size, 6), dtype=np.float32)
        f[:, 0] = xl
        f[:, 1] = 2.0 * math.log(c["Ma"] / 0.3)
        f[:, 2] = (c["Pr"] - 0.835) / 0.165
        f[:, 3] = c["mub"] - 1.0
        f[:, 4] = math.log10(c["Kn"]) + 2.0
        f[:, 5] = (c["delta"] - 2.5) / 0.5
        rows.append(f)
    return np.concatenate(rows)


def targets(cases, m):
    """Normalised moments of converged states, [ns_total][4] float32."""
    out, o = [], 0
    for c in cases:
        ns = 2 * c["L"]
        U = c["U"]
        sl = slice(o, o + ns)
        t = np.empty((ns, 4), dtype=np.float32)
        if c["kind"] == SHOCK:
            (r1, u1, t1), (r2, u2, t2) = c["up"], c["down"]
            t[:, 0] = (m["rho"][sl] - r1) / (r2 - r1)
            t[:, 1] = (m["u"][0][sl] - u1) / (u2 - u1)
            t[:, 2] = (m["thT"][sl] - t1) / (t2 - t1)
            t[:, 3] = (m["thR"][sl] - t1) / (t2 - t1)
        else:
            t[:, 0] = (m["rho"][sl] - 1.0) / U ** 2
            t[:, 1] = m["u"][1][sl] / U
            t[:, 2] = (m["thT"][sl] - THETA0) / U ** 2
            t[:, 3] = (m["thR"][sl] - THETA0) / U ** 2
        out.append(t)
        o += ns
    return np.concatenate(out)


def recentre_shock(L, ys):
    """A predicted shock profile (normalised outputs of one line's sites)
    shifted along x so that its density crosses the mean of the two states at
    L/2, where the cold start puts its shock; the end plateaus extend."""
    x = positions(L, 1, 1)[0]
    o = np.argsort(x)
    xs, f = x[o], ys[o, 0]
    k = int(np.argmax(f > 0.5))
    if k == 0 or not (f[k] > 0.5):
        return ys
    pos = xs[k - 1] + (0.5 - f[k - 1]) / (f[k] - f[k - 1]) * (xs[k] - xs[k - 1])
    out = np.empty_like(ys)
    for j in range(ys.shape[1]):
        out[:, j] = np.interp(x + (pos - 0.5 * L), xs, ys[o, j])
    return out


def fields_from_prediction(cases, y, recentre_shocks=False):
    """Moment fields (for pgk_batch_init) from normalised network outputs;
    recentre_shocks: each shock profile moved to the cold start's position."""
    ns = y.shape[0]
    rho, u, thT, thR = np.empty(ns), np.zeros((3, ns)), np.empty(ns), np.empty(ns)
    o = 0
    for c in cases:
        n = 2 * c["L"]
        U = c["U"]
        sl = slice(o, o + n)
        if c["kind"] == SHOCK:
            (r1, u1, t1), (r2, u2, t2) = c["up"], c["down"]
            ys = recentre_shock(c["L"], y[sl]) if recentre_shocks else y[sl]
            rho[sl] = r1 + (r2 - r1) * ys[:, 0]
            u[0, sl] = u1 + (u2 - u1) * ys[:, 1]
            thT[sl] = t1 + (t2 - t1) * ys[:, 2]
            thR[sl] = t1 + (t2 - t1) * ys[:, 3]
        else:
            rho[sl] = 1.0 + U ** 2 * y[sl, 0]
            u[1, sl] = U * y[sl, 1]
            thT[sl] = THETA0 + U ** 2 * y[sl, 2]
            thR[sl] = THETA0 + U ** 2 * y[sl, 3]
        o += n
    return dict(rho=rho, u=u, thT=thT, thR=thR)
