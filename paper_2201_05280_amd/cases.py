"""Seeded 1D case generator for the batched sweep and the learned warm start.

Couette layers between two diffuse walls (Sec. 6 runs start-up and thermal
Couette flows): the low wall at rest, the high wall moving tangentially (y)
at Ma_w c_s, both at theta0.  Knudsen number Kn = nu/(c_s L) (the reading
under which the Landau formula of Sec. 6 matches the sound-diffusion law),
so nu = Kn c_s L.  Draws: L ~ U{Lmin..Lmax}, Ma_w ~ U[Ma range],
Kn ~ logU[Kn range], delta ~ {2, 3}, and the pair Pr ~ U[Pr range],
mu_b/mu ~ U[mub range] redrawn together while it is out of the model's reach
(mu_b/mu at or below 1.02 times the floor 2 delta/(3(3+delta)), or no
feasible (b, k_r) for it).

Network features (all O(1)): x/L, (Ma - 0.3)/0.2, (Pr - 0.835)/0.165,
(mu_b/mu - 1), log10 Kn + 2, (delta - 2.5)/0.5; targets: (rho - 1)/U^2,
u_y/U, (theta_T - theta0)/U^2, (theta_R - theta0)/U^2 with U the wall speed.
"""
import math

import numpy as np

from . import _lib
from .inputs import THETA0, positions

COUETTE = "couette"


def sweep_cases(n, seed, L_range=(256, 1024), Ma_range=(0.1, 0.5), Kn_range=(3e-3, 3e-2),
                Pr_range=(0.67, 1.0), mub_range=(0.0, 2.0), deltas=(2.0, 3.0)):
    rng = np.random.default_rng(seed)
    out = []
    redraws = 0
    for _ in range(n):
        L = int(rng.integers(L_range[0], L_range[1] + 1))
        Ma = float(rng.uniform(*Ma_range))
        Kn = float(10 ** rng.uniform(math.log10(Kn_range[0]), math.log10(Kn_range[1])))
        delta = float(deltas[int(rng.integers(0, len(deltas)))])
        floor = 2 * delta / (3 * (3 + delta)) * 1.02
        gamma = (5 + delta) / (3 + delta)
        cs = math.sqrt(gamma * THETA0)
        nu = Kn * cs * L
        while True:
            # (Pr, mu_b/mu) pairs outside the model's reach (bulk viscosity at
            # or below the floor, or no b in [-1/2, 1) with k_r >= 0) are redrawn
            Pr = float(rng.uniform(*Pr_range))
            mub = float(rng.uniform(*mub_range))
            if mub > floor:
                try:
                    p = _lib.resolve(nu, Pr, mub, delta)
                    break
                except ValueError:
                    pass
            redraws += 1
        out.append(dict(kind=COUETTE, L=L, Ma=Ma, Kn=Kn, Pr=Pr, mub=mub, delta=delta, nu=nu,
                        U=Ma * cs, params=p))
    return out, redraws


def to_batch_cases(cases, variant=0):
    from .batch import make_case
    res = []
    for c in cases:
        p = c["params"]
        res.append(make_case(c["L"], _lib.WALL, (p["tau"], p["tau1"], p["b"], p["kr"], p["delta"]),
                             u=((0, 0, 0), (0, c["U"], 0)), theta=(THETA0, THETA0), vel_axis=1, variant=variant))
    return res


def cold_fields(cases):
    """Uniform gas at rest at theta0 for every case, concatenated over sites."""
    ns = sum(2 * c["L"] for c in cases)
    return dict(rho=np.ones(ns), u=np.zeros((3, ns)), thT=np.full(ns, THETA0), thR=np.full(ns, THETA0))


def features(cases):
    """[ns_total][6] float32 network inputs, site order of the batch."""
    rows = []
    for c in cases:
        x = positions(c["L"], 1, 1)[0]
        # walls at -1/4 and L - 1/4
        xl = (x + 0.25) / c["L"]
        f = np.empty((x.size, 6), dtype=np.float32)
        f[:, 0] = xl
        f[:, 1] = (c["Ma"] - 0.3) / 0.2
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
        t[:, 0] = (m["rho"][sl] - 1.0) / U ** 2
        t[:, 1] = m["u"][1][sl] / U
        t[:, 2] = (m["thT"][sl] - THETA0) / U ** 2
        t[:, 3] = (m["thR"][sl] - THETA0) / U ** 2
        out.append(t)
        o += ns
    return np.concatenate(out)


def fields_from_prediction(cases, y):
    """Moment fields (for pgk_batch_init) from normalised network outputs."""
    ns = y.shape[0]
    rho, u, thT, thR = np.empty(ns), np.zeros((3, ns)), np.empty(ns), np.empty(ns)
    o = 0
    for c in cases:
        n = 2 * c["L"]
        U = c["U"]
        sl = slice(o, o + n)
        rho[sl] = 1.0 + U ** 2 * y[sl, 0]
        u[1, sl] = U * y[sl, 1]
        thT[sl] = THETA0 + U ** 2 * y[sl, 2]
        thR[sl] = THETA0 + U ** 2 * y[sl, 3]
        o += n
    return dict(rho=rho, u=u, thT=thT, thR=thR)
