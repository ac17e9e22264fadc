"""Normal-shock lines with the E2 equilibrium on the GPU (full 4096-cell size).

The faces hold the model's own jump states (equal equilibrium fluxes of mass,
momentum and energy), at Mach 1.5 with the upstream at the lattice
temperature and at Mach 3 with a cold upstream gas (theta1 = 0.08, the warm
upstream state at Mach 3 being beyond the lattice).  Parity with the FP64
oracle: element by element on the whole line after the first steps from the
seeded tanh profile, and after 2000 steps on a 512-cell line.  At full size the steady state is checked through
properties: the residual falls below 1e-10, the far fields equal the jump
states and the shock stays put.
"""
import numpy as np
import pytest

import oracle
from oracle.params import resolve

pytestmark = pytest.mark.gpu

CASES = {1.5: oracle.THETA0, 3.0: 0.08}
FLOOR = dict(rho=0.0, u=1e-2, thT=0.0, thR=0.0, P=0.0)
_ORACLE = {}


def _setup(Ma, L):
    from paper_2201_05280_amd.shock import discrete_rankine_hugoniot, tanh_profile
    th1 = CASES[Ma]
    up, down = discrete_rankine_hugoniot(Ma, 2.0, th1)
    p = resolve(2.0 * np.sqrt(1.4 * th1), 0.71, 0.8, 2.0)
    return up, down, p, tanh_profile(L, up, down)


def _solver(L, prec, up, down, p, f):
    import paper_2201_05280_amd as pgk
    s = pgk.Solver(L, 1, 1, precision=prec, bc_x=(pgk.DIRICHLET, pgk.DIRICHLET), equilibrium=pgk.E2)
    s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
    s.set_bc_x(0, up[0], (up[1], 0, 0), up[2])
    s.set_bc_x(1, down[0], (down[1], 0, 0), down[2])
    s.init(f["rho"], f["u"], f["thT"], f["thR"])
    return s


def _oracle(L, up, down, p, f):
    o = oracle.Oracle(L, 1, 1, equilibrium=oracle.E2)
    o.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
    o.set_bc_x(0, oracle.DIRICHLET, up[0], (up[1], 0, 0), up[2])
    o.set_bc_x(1, oracle.DIRICHLET, down[0], (down[1], 0, 0), down[2])
    o.init(f["rho"], f["u"], f["thT"], f["thR"])
    return o


def _rel(g, o):
    return {k: float(np.abs(g[k] - o[k]).max() / max(np.abs(o[k]).max(), FLOOR[k])) for k in FLOOR}


def _resid(a, b):
    r = 0.0
    for k, v in (("rho", None), ("u", 0), ("thT", None), ("thR", None)):
        x0 = a[k] if v is None else a[k][v]
        x1 = b[k] if v is None else b[k][v]
        d = float(np.linalg.norm(x1 - x0) / np.linalg.norm(x1))
        r = max(r, d) if d == d else d   # a NaN stays NaN
    return r


@pytest.mark.parametrize("Ma", [1.5, 3.0])
@pytest.mark.parametrize("precision,bar", [(0, 1e-12), (1, 1e-5)])
def test_full_line_matches_oracle(Ma, precision, bar):
    L, steps = 4096, 40
    up, down, p, f = _setup(Ma, L)
    if Ma not in _ORACLE:
        o = _oracle(L, up, down, p, f)
        o.step(steps)
        _ORACLE[Ma] = o.moments()
    s = _solver(L, precision, up, down, p, f)
    s.step(steps)
    e = _rel(s.moments(), _ORACLE[Ma])
    s.close()
    print("shock parity", Ma, precision, e)
    for k, v in e.items():
        assert v <= bar, (k, v, e)


@pytest.mark.parametrize("precision", [0, 1])
def test_long_run_matches_oracle(precision):
    # 2000 steps of a 512-cell line: the shock forms from the tanh blend and the
    # start-up waves cross the line and leave through the faces.  FP64: the
    # whole line element by element at 1e-12.  FP32 storage: between two
    # Dirichlet faces the shock's position is a neutral mode fixed only by the
    # mass held between the faces, and the FP32 run ends the start-up
    # transient with 2.4e-6 less mass than the FP64 one (the deficit grows
    # while the waves leave and stops at steady state), which places its shock
    # 7e-4 cells downstream.  The profiles are therefore compared with the two
    # positions aligned, at the 1e-5 bar on every moment; the unaligned error
    # (1.0e-5 measured) is held at 3e-5, the mass deficit at 5e-6 and the
    # shift at 2e-3 cells.
    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd import inputs
    from paper_2201_05280_amd.shock import profile_metrics
    L, steps = 512, 2000
    up, down, p, f = _setup(1.5, L)
    key = ("long", L, steps)
    if key not in _ORACLE:
        o = _oracle(L, up, down, p, f)
        o.step(steps)
        _ORACLE[key] = (o.moments(), o.conserved())
    ref, ref_c = _ORACLE[key]
    s = _solver(L, precision, up, down, p, f)
    s.step(steps)
    m = s.moments()
    c = s.conserved()
    s.close()
    e = _rel(m, ref)
    x = inputs.positions(L, 1, 1)[0]
    pg, tg = profile_metrics(x, m["rho"], up, down)
    po, to = profile_metrics(x, ref["rho"], up, down)
    dm = (c[0] - ref_c[0]) / ref_c[0]
    print("long shock parity", precision, e, "position", pg, po, "thickness", tg, to, "mass", dm)
    if precision == pgk.FP64:
        for k, v in e.items():
            assert v <= 1e-12, (k, v, e)
        assert abs(pg - po) < 1e-9 and abs(dm) < 1e-13
        return
    # aligned: the FP32 fields sampled at x + (pg - po) against the oracle at x
    order = np.argsort(x)
    xs = x[order]
    inside = (xs + (pg - po) >= xs[0]) & (xs + (pg - po) <= xs[-1])
    al = {}
    for k in ("rho", "u", "thT", "thR", "P"):
        g, o = m[k], ref[k]
        rows = [(g[i], o[i]) for i in range(g.shape[0])] if g.ndim == 2 else [(g, o)]
        err = 0.0
        for gi, oi in rows:
            gs = np.interp(xs[inside] + (pg - po), xs, gi[order])
            err = max(err, float(np.abs(gs - oi[order][inside]).max()))
        al[k] = err / max(np.abs(o).max(), FLOOR[k])
    print("aligned FP32 parity", al)
    for k, v in al.items():
        assert v <= 1e-5, (k, v, al)
    for k, v in e.items():
        assert v <= 3e-5, (k, v, e)
    assert abs(dm) < 5e-6 and abs(pg - po) < 2e-3 and abs(tg / to - 1) < 1e-4


def test_full_size_shock_reaches_its_steady_state():
    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd import inputs
    from paper_2201_05280_amd.shock import profile_metrics
    L = 4096
    up, down, p, f = _setup(1.5, L)
    s = _solver(L, pgk.FP64, up, down, p, f)
    x = inputs.positions(L, 1, 1)[0]
    done, r, pos = 0, 1.0, []
    while r > 1e-10 and done < 80000:
        s.step(4999)
        a = s.moments()
        s.step(1)
        b = s.moments()
        done += 5000
        r = _resid(a, b)
        pos.append(profile_metrics(x, b["rho"], up, down)[0])
    s.close()
    assert r <= 1e-10, (done, r)
    o = np.argsort(x)
    for i, st in ((o[4], up), (o[-5], down)):
        assert abs(b["rho"][i] / st[0] - 1) < 1e-6 and abs(b["u"][0][i] / st[1] - 1) < 1e-6
        assert abs(b["thT"][i] / st[2] - 1) < 1e-6 and abs(b["thR"][i] / st[2] - 1) < 1e-6
    assert abs(pos[-1] - pos[-2]) < 1e-3   # cells moved over the last 5000 steps
    _, thick = profile_metrics(x, b["rho"], up, down)
    print("steady shock", done, r, pos[-1], thick)


def test_fast_inflow_line_stays_on_the_oracle():
    """A Mach 2.31 line with its upstream at theta0 (inflow speed 1.49, near the
    end of what E2 reaches at theta0; nu 2.71, Pr 0.71, mu_b/mu 1.75, 2621
    cells, 24 diffusion sub-steps) from the tanh start: after 576 FP64 steps the
    line is finite and on the oracle.  A lane-pair kernel that summed each
    lane's populations first and added the two sums (other last bits in the
    moments) turned this line NaN between steps 512 and 576; the lane pair
    sums the moments as one lane does."""
    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd.shock import discrete_rankine_hugoniot, tanh_profile
    L, Ma, steps = 2621, 2.312666544905132, 576
    up, down = discrete_rankine_hugoniot(Ma, 2.0, oracle.THETA0)
    p = resolve(2.713688893895381, 0.7100164850878086, 1.7524045176004193, 2.0)
    f = tanh_profile(L, up, down)
    s = _solver(L, pgk.FP64, up, down, p, f)
    s.step(steps)
    g = s.moments()
    s.close()
    for k in ("rho", "thT", "thR"):
        assert np.isfinite(g[k]).all(), k
    o = _oracle(L, up, down, p, f)
    o.step(steps)
    e = _rel(g, o.moments())
    print("Mach 2.31 line after", steps, "steps:", e)
    for k, v in e.items():
        assert v <= 1e-12, (k, v)
