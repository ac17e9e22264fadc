"""Checkpoints on the GPU: a state copied out between steps and copied back
(into the same grid, or into a fresh grid from a file) continues bit for bit,
on periodic grids in FP32 storage, between walls in FP64, with E2 Dirichlet
faces (whose Newton warm starts are part of the state), and for a batch under
a fixed config."""
import numpy as np
import pytest

import oracle
from oracle.params import resolve
from paper_2201_05280_amd import inputs

pytestmark = pytest.mark.gpu


def _grid(kind, precision):
    import paper_2201_05280_amd as pgk
    th0 = oracle.THETA0
    if kind == "periodic":
        s = pgk.Solver(10, 8, 6, precision=precision)
        p = resolve(0.02, 0.71, 0.6, 2.0)
        f = inputs.random_smooth(10, 8, 6, seed=51)
        faces = None
    elif kind == "walls":
        s = pgk.Solver(24, 3, 1, precision=precision, bc_x=(pgk.WALL, pgk.WALL))
        p = resolve(0.3, 0.71, 0.8, 2.0)
        f = inputs.uniform(24, 3, 1)
        faces = [(1.0, (0.0, 0.0, 0.0), th0), (1.0, (0.0, 0.05, 0.0), 1.1 * th0)]
    else:
        from paper_2201_05280_amd.shock import discrete_rankine_hugoniot, tanh_profile
        up, down = discrete_rankine_hugoniot(1.5, 2.0, th0)
        s = pgk.Solver(48, 1, 1, precision=precision, bc_x=(pgk.DIRICHLET, pgk.DIRICHLET), equilibrium=pgk.E2)
        p = resolve(2.0 * np.sqrt(1.4 * th0), 0.71, 0.8, 2.0)
        f = tanh_profile(48, up, down)
        faces = [(up[0], (up[1], 0, 0), up[2]), (down[0], (down[1], 0, 0), down[2])]
    s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
    if faces:
        for side in (0, 1):
            s.set_bc_x(side, *faces[side])
    return s, f


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("kind,precision", [("periodic", 1), ("walls", 0), ("e2", 0), ("e2", 1)])
def test_checkpoint_resumes_bit_for_bit(kind, precision, tmp_path):
    s, f = _grid(kind, precision)
    s.init(f["rho"], f["u"], f["thT"], f["thR"])
    s.step(37)
    ck = s.checkpoint()
    s.save(str(tmp_path / "ck.npz"))
    s.step(45)
    ref, n_ref = s.moments(), s.steps_done()
    s.restore(ck)                       # same grid, in memory
    s.step(45)
    _same(ref, s.moments())
    assert s.steps_done() == n_ref
    s.close()
    t, _ = _grid(kind, precision)       # fresh grid, from the file
    t.load(str(tmp_path / "ck.npz"))
    t.step(45)
    _same(ref, t.moments())
    assert t.steps_done() == n_ref
    t.close()


def test_checkpoint_before_the_first_step():
    s, f = _grid("walls", 1)
    s.init(f["rho"], f["u"], f["thT"], f["thR"])
    ck = s.checkpoint()
    s.step(40)
    ref = s.moments()
    s.restore(ck)
    s.step(40)
    _same(ref, s.moments())
    s.close()


def test_batch_checkpoint_resumes_bit_for_bit():
    from paper_2201_05280_amd import cases as C
    from paper_2201_05280_amd.batch import Batch
    cs, _ = C.sweep_cases(6, 7, L_range=(40, 90), Kn_range=(0.02, 0.08), shock_fraction=0.5,
                          shock_Ma_range=(1.1, 1.3), shock_Kn_range=(0.01, 0.02))
    fields = C.cold_fields(cs)
    b = Batch(C.to_batch_cases(cs))
    b.init(fields["rho"], fields["u"], fields["thT"], fields["thR"])
    b.config(256, 16)
    b.run(64, 0.0)
    ck = b.checkpoint()
    st1, rs1, _ = b.run(160, 0.0)
    ref = b.moments()
    b.restore(ck)
    st2, rs2, _ = b.run(160, 0.0)
    _same(ref, b.moments())
    assert (st1 == st2).all() and np.array_equal(rs1, rs2)
    b.close()
