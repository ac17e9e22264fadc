"""pgk_step's replayed K-step graphs against steps launched one by one (GPU only).

With K graph steps set, a call records K steps once per starting buffer and
replays them, the rest launched directly; calls shorter than K and timed runs
launch each kernel directly.  Both must give identical bits: the same kernels
with the same arguments run in the same order.  The cases cover step counts
below, at and above multiples of K, the untouched first step, diffuse walls
and Dirichlet faces (the ghost refresh), the sub-cycled diffusion, FP32
storage, the E2 equilibrium, a parameter change and a new K between calls
(the recorded chunks must be rebuilt) and a caller's own stream.
"""
import numpy as np
import pytest

import oracle
from oracle.params import resolve
from paper_2201_05280_amd import inputs

pytestmark = pytest.mark.gpu


def _pair(nx, ny, nz, f, p, precision=0, bc=None, equilibrium=0, stream=None, K=2):
    import paper_2201_05280_amd as pgk
    kinds = (pgk.PERIODIC, pgk.PERIODIC) if bc is None else (bc[0][0], bc[1][0])
    out = []
    for _ in range(2):
        s = pgk.Solver(nx, ny, nz, precision=precision, bc_x=kinds, equilibrium=equilibrium, stream=stream)
        s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
        if bc is not None:
            for side in (0, 1):
                _, rho, u, th = bc[side]
                s.set_bc_x(side, rho, u, th)
        s.init(f["rho"], f["u"], f["thT"], f["thR"])
        out.append(s)
    out[0].set_graph_steps(K)
    return out


def _same(a, b, label):
    ma, mb = a.moments(), b.moments()
    for k in ma:
        assert np.array_equal(ma[k], mb[k]), (label, k, float(np.abs(ma[k] - mb[k]).max()))
    assert a.steps_done() == b.steps_done(), label


def _run(a, b, calls, label):
    """a: each call in one pgk_step; b: the same number of single steps."""
    for n in calls:
        a.step(n)
        for _ in range(n):
            b.step(1)
        _same(a, b, (label, n))


@pytest.mark.parametrize("precision,K", [(0, 2), (1, 2), (0, 6), (1, 16)])
def test_periodic_odd_and_even_calls(precision, K):
    f = inputs.random_smooth(12, 10, 6, seed=31)
    p = resolve(0.02, 0.71, 0.6, 2.0)
    a, b = _pair(12, 10, 6, f, p, precision, K=K)
    _run(a, b, [5, 8, 7, 3, 12, 2 * K + 1, K], "periodic")
    a.close(); b.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_walls_and_subcycled_diffusion(precision):
    import paper_2201_05280_amd as pgk
    th0 = oracle.THETA0
    bc = [(pgk.WALL, 1.0, (0.0, 0.0, 0.0), th0), (pgk.WALL, 1.0, (0.0, 0.04, 0.0), th0 * 1.05)]
    p = resolve(0.5, 0.71, 0.8, 2.0)   # several FTCS sub-steps per step
    a, b = _pair(20, 3, 1, inputs.uniform(20, 3, 1), p, precision, bc=bc)
    _run(a, b, [4, 9, 6], "walls")
    a.close(); b.close()


def test_dirichlet_e2_shock():
    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd.shock import discrete_rankine_hugoniot, tanh_profile
    up, down = discrete_rankine_hugoniot(1.5, 2.0, oracle.THETA0)
    p = resolve(2.0 * np.sqrt(1.4 * oracle.THETA0), 0.71, 0.8, 2.0)
    bc = [(pgk.DIRICHLET, up[0], (up[1], 0, 0), up[2]), (pgk.DIRICHLET, down[0], (down[1], 0, 0), down[2])]
    a, b = _pair(48, 1, 1, tanh_profile(48, up, down), p, 0, bc=bc, equilibrium=pgk.E2)
    _run(a, b, [6, 5], "e2 shock")
    a.close(); b.close()


def test_parameter_change_rebuilds_the_pair():
    f = inputs.random_smooth(9, 8, 5, seed=32)
    p1 = resolve(0.02, 0.71, 0.6, 2.0)
    p2 = resolve(0.05, 0.9, 0.8, 2.0)
    a, b = _pair(9, 8, 5, f, p1)
    _run(a, b, [6], "before")
    for s in (a, b):
        s.set_params(p2["tau"], p2["tau1"], p2["b"], p2["kr"], p2["delta"])
    _run(a, b, [6, 7], "after")
    a.set_graph_steps(4)
    _run(a, b, [9, 4], "new K")
    a.set_graph_steps(0)
    _run(a, b, [5], "direct")
    a.close(); b.close()


def test_callers_stream_and_timing():
    import torch
    f = inputs.random_smooth(10, 6, 4, seed=33)
    p = resolve(0.02, 0.71, 0.6, 2.0)
    st = torch.cuda.Stream()
    a, b = _pair(10, 6, 4, f, p, stream=st, K=4)
    b.set_graph_steps(4)
    b.set_timing(True)   # timed runs launch kernel by kernel
    a.step(10)
    b.step(10)
    _same(a, b, "stream")
    a.close(); b.close()


@pytest.mark.parametrize("kind", ["wall", "dirichlet"])
def test_face_changes_and_reinitialisation_between_calls(kind):
    # the ghost bookkeeping across replays: face states changed between calls
    # (the pending pull keeps the old state), moments read in between, and a
    # second initialisation of the same grid
    import paper_2201_05280_amd as pgk
    th0 = oracle.THETA0
    K = pgk.WALL if kind == "wall" else pgk.DIRICHLET
    bc = [(K, 1.0, (0.0, 0.0, 0.0) if kind == "wall" else (0.03, 0.0, 0.0), th0),
          (K, 1.0, (0.0, 0.04, 0.0) if kind == "wall" else (0.03, 0.0, 0.0), th0 * 1.05)]
    p = resolve(0.05, 0.71, 0.8, 2.0)
    f = inputs.uniform(24, 2, 1, u=(0.0, 0, 0) if kind == "wall" else (0.03, 0, 0))
    a, b = _pair(24, 2, 1, f, p, 0, bc=bc, K=4)
    _run(a, b, [9, 5], "start")
    new = (1.0, (0.0, -0.03, 0.0), th0 * 0.9) if kind == "wall" else (1.04, (0.0, 0.0, 0.0), th0 * 1.1)
    for s in (a, b):
        s.set_bc_x(0, *new)
    _run(a, b, [1, 8, 13], "changed")
    for s in (a, b):
        s.init(f["rho"], f["u"], f["thT"], f["thR"])
    _run(a, b, [12, 3], "again")
    a.close(); b.close()
