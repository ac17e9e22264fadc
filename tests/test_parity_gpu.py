"""Parity of the HIP path with the FP64 oracle (GPU only).

Both sides start from the same seeded fields and the same resolved
parameters; the comparison is element by element on the f-moments
rho, u, theta_T, theta_R and the pressure tensor.  Error measure per field:
max |gpu - oracle| / max(max |oracle|, floor), floor = 1e-2 for u (the
perturbation scale) and the field's own magnitude otherwise.
Bars: FP64 storage 1e-12, FP32 deviation storage 1e-5.
"""
import numpy as np
import pytest

import oracle
from oracle.params import resolve
from paper_2201_05280_amd import inputs

pytestmark = pytest.mark.gpu

FLOOR = dict(rho=0.0, u=1e-2, thT=0.0, thR=0.0, P=0.0)


def _solver(*a, **kw):
    import paper_2201_05280_amd as pgk
    return pgk.Solver(*a, **kw)


def rel_err(g, o):
    out = {}
    for k in ("rho", "u", "thT", "thR", "P"):
        den = max(np.abs(o[k]).max(), FLOOR[k])
        out[k] = float(np.abs(g[k] - o[k]).max() / den)
    return out


def run_pair(nx, ny, nz, fields, p, steps, precision, variant=0, bc=None, checkpoints=None):
    import paper_2201_05280_amd as pgk
    bc_kind = (pgk.PERIODIC, pgk.PERIODIC) if bc is None else (bc[0][0], bc[1][0])
    s = _solver(nx, ny, nz, precision=precision, variant=variant, bc_x=bc_kind)
    s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
    o = oracle.Oracle(nx, ny, nz, variant=variant)
    o.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
    if bc is not None:
        for side in (0, 1):
            kind, rho, u, th = bc[side]
            s.set_bc_x(side, rho, u, th)
            o.set_bc_x(side, kind, rho, u, th)
    s.init(fields["rho"], fields["u"], fields["thT"], fields["thR"])
    o.init(fields["rho"], fields["u"], fields["thT"], fields["thR"])
    errs = []
    done = 0
    for n in (checkpoints or [steps]):
        s.step(n - done)
        o.step(n - done)
        done = n
        errs.append(rel_err(s.moments(), o.moments()))
    cons = (s.conserved(), o.conserved())
    s.close()
    return errs, cons


def _assert_bar(errs, bar, label=""):
    for e in errs:
        for k, v in e.items():
            assert v <= bar, (label, k, v, e)


P_SHEAR = resolve(0.01, 0.71, 0.6, 2.0)


@pytest.mark.parametrize("precision,bar", [(0, 1e-12), (1, 1e-5)])
def test_shear_wave_64x64_2000_steps(precision, bar):
    # the 2D shear-wave workload at full size: 64x64 cells, 8192 sites
    f = inputs.shear_wave(64, 64, 1, amp=0.01)
    errs, (cg, co) = run_pair(64, 64, 1, f, P_SHEAR, 2000, precision, checkpoints=[1, 10, 500, 2000])
    print("shear parity", precision, errs)
    _assert_bar(errs, bar, "shear")
    assert abs(cg[0] - co[0]) <= bar * co[0]
    assert abs(cg[4] - co[4]) <= bar * co[4]


@pytest.mark.parametrize("precision,bar", [(0, 1e-12), (1, 1e-5)])
@pytest.mark.parametrize("dims", [(7, 5, 3), (13, 1, 1), (1, 9, 4), (2, 2, 2), (33, 17, 1)])
def test_random_fields_ragged_grids(precision, bar, dims):
    # grids whose site counts are not multiples of the 256-thread block, with
    # axes of length 1 and 2 (wrap-around onto the same cell)
    nx, ny, nz = dims
    p = resolve(0.02, 0.8, 0.7, 3.0)
    f = inputs.random_smooth(nx, ny, nz, seed=sum(dims))
    errs, _ = run_pair(nx, ny, nz, f, p, 60, precision, checkpoints=[1, 7, 60])
    print("random parity", dims, precision, errs)
    _assert_bar(errs, bar, dims)


@pytest.mark.parametrize("precision,bar", [(0, 1e-12), (1, 1e-5)])
def test_printed_variant(precision, bar):
    f = inputs.random_smooth(12, 10, 3, seed=5)
    errs, _ = run_pair(12, 10, 3, f, P_SHEAR, 100, precision, variant=1, checkpoints=[1, 100])
    _assert_bar(errs, bar, "LIT")


@pytest.mark.parametrize("precision,bar", [(0, 1e-12), (1, 1e-5)])
def test_taylor_green_small(precision, bar):
    # the 3D Taylor-Green workload at reduced size (same Mach, same Reynolds scaling)
    n = 16
    U = 0.1 * np.sqrt(1.4 * oracle.THETA0)
    nu = U * (n / (2 * np.pi)) / 1600.0
    p = resolve(nu, 0.71, 0.6, 2.0)
    f = inputs.taylor_green(n, U)
    errs, (cg, co) = run_pair(n, n, n, f, p, 200, precision, checkpoints=[1, 50, 200])
    print("tgv parity", precision, errs)
    _assert_bar(errs, bar, "tgv")


@pytest.mark.parametrize("precision,bar", [(0, 1e-12), (1, 1e-5)])
def test_diffuse_walls_couette(precision, bar):
    import paper_2201_05280_amd as pgk
    th0 = oracle.THETA0
    U = 0.05
    bc = [(pgk.WALL, 1.0, (0.0, 0.0, 0.0), th0), (pgk.WALL, 1.0, (0.0, U, 0.0), th0 * 1.02)]
    f = inputs.uniform(24, 1, 1)
    p = resolve(0.05, 0.71, 0.8, 2.0)
    errs, _ = run_pair(24, 1, 1, f, p, 300, precision, bc=bc, checkpoints=[1, 2, 30, 300])
    print("couette parity", precision, errs)
    _assert_bar(errs, bar, "couette")


@pytest.mark.parametrize("precision,bar", [(0, 1e-12), (1, 1e-5)])
def test_diffuse_walls_3d_columns(precision, bar):
    import paper_2201_05280_amd as pgk
    th0 = oracle.THETA0
    bc = [(pgk.WALL, 1.0, (0.0, 0.02, 0.01), th0), (pgk.WALL, 1.0, (0.0, -0.02, 0.0), th0)]
    f = inputs.random_smooth(6, 5, 3, seed=9)
    p = resolve(0.03, 0.9, 0.9, 2.0)
    errs, _ = run_pair(6, 5, 3, f, p, 40, precision, bc=bc, checkpoints=[1, 3, 40])
    _assert_bar(errs, bar, "walls3d")


@pytest.mark.parametrize("precision,bar", [(0, 1e-12), (1, 1e-5)])
def test_dirichlet_faces(precision, bar):
    import paper_2201_05280_amd as pgk
    th0 = oracle.THETA0
    bc = [(pgk.DIRICHLET, 1.02, (0.03, 0.0, 0.0), th0 * 1.01), (pgk.DIRICHLET, 0.99, (0.03, 0.0, 0.0), th0)]
    f = inputs.uniform(32, 1, 1, u=(0.03, 0, 0))
    p = resolve(0.05, 0.71, 0.8, 2.0)
    errs, _ = run_pair(32, 1, 1, f, p, 200, precision, bc=bc, checkpoints=[1, 2, 200])
    _assert_bar(errs, bar, "dirichlet")


def test_conservation_on_gpu_fp64():
    # mass and momentum exact to round-off through the GPU reductions
    f = inputs.random_smooth(10, 9, 8, seed=3)
    p = resolve(0.02, 0.71, 0.6, 2.0)
    s = _solver(10, 9, 8, precision=0)
    s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
    s.init(f["rho"], f["u"], f["thT"], f["thR"])
    c0 = s.conserved()
    s.step(200)
    c1 = s.conserved()
    eps = np.finfo(float).eps
    assert (np.abs(c1[:4] - c0[:4]) <= 4 * eps * 200 * c0[0]).all(), c1 - c0
    s.close()


def test_bitwise_determinism_fp64():
    f = inputs.random_smooth(9, 8, 7, seed=4)
    p = resolve(0.02, 0.71, 0.6, 2.0)
    outs = []
    for _ in range(2):
        s = _solver(9, 8, 7, precision=0)
        s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
        s.init(f["rho"], f["u"], f["thT"], f["thR"])
        s.step(50)
        outs.append(s.moments())
        s.close()
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


@pytest.mark.parametrize("precision", [0, 1])
def test_bitwise_determinism_e2_shock_line(precision):
    # a 2100-cell E2 line between Dirichlet faces (warm-started Newton
    # multipliers, the one-launch line transport), run twice from the same
    # state: the same bits in FP64 and in FP32 storage
    import paper_2201_05280_amd as pgk
    th0 = oracle.THETA0
    p = resolve(0.3, 0.71, 0.8, 2.0)
    f = inputs.uniform(2100, 1, 1, u=(0.2, 0, 0))
    outs = []
    for _ in range(2):
        s = _solver(2100, 1, 1, precision=precision, bc_x=(pgk.DIRICHLET, pgk.DIRICHLET), equilibrium=pgk.E2)
        s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
        s.set_bc_x(0, 1.0, (0.2, 0.0, 0.0), th0)
        s.set_bc_x(1, 1.05, (0.19, 0.0, 0.0), 1.02 * th0)
        s.init(f["rho"], f["u"], f["thT"], f["thR"])
        s.step(300)
        outs.append(s.moments())
        s.close()
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), (precision, k)


@pytest.mark.parametrize("precision,bar", [(0, 1e-12), (1, 1e-5)])
def test_subcycled_diffusion_paths(precision, bar):
    # large viscosity: several FTCS sub-steps per step, both for a periodic
    # grid (the unfused transport path) and for diffuse walls
    import paper_2201_05280_amd as pgk
    p = resolve(0.5, 0.71, 0.8, 2.0)
    f = inputs.random_smooth(10, 6, 1, seed=21)
    errs, _ = run_pair(10, 6, 1, f, p, 40, precision, checkpoints=[1, 40])
    _assert_bar(errs, bar, "subcycled periodic")
    th0 = oracle.THETA0
    bc = [(pgk.WALL, 1.0, (0.0, 0.0, 0.0), th0), (pgk.WALL, 1.0, (0.0, 0.04, 0.0), th0 * 1.05)]
    errs, _ = run_pair(20, 1, 1, inputs.uniform(20, 1, 1), p, 60, precision, bc=bc, checkpoints=[1, 60])
    _assert_bar(errs, bar, "subcycled walls")


@pytest.mark.parametrize("precision,bar", [(0, 1e-12), (1, 1e-5)])
@pytest.mark.parametrize("nx", [2049, 2100])
def test_long_lines_transport_in_one_launch(precision, bar, nx):
    # lines of more than 4096 sites, bounded or sub-cycled: the theta_R
    # transport runs in work-groups of 1024 cells with a halo of nsub + 1
    # (2049 cells: a last chunk of one cell; 2100: of 52); walls with a
    # temperature step, Dirichlet faces with inflow, and a periodic line, each
    # with 1, 3 and 11 diffusion sub-steps
    import paper_2201_05280_amd as pgk
    th0 = oracle.THETA0
    f = inputs.random_smooth(nx, 1, 1, seed=nx, amp_u=0.02, amp_th=0.05)
    for nu, steps in ((0.05, 12), (0.5, 12), (2.0, 8)):
        p = resolve(nu, 0.71, 0.8, 2.0)
        bc = [(pgk.WALL, 1.0, (0.0, 0.0, 0.0), 0.95 * th0), (pgk.WALL, 1.0, (0.0, 0.03, 0.0), 1.05 * th0)]
        errs, _ = run_pair(nx, 1, 1, f, p, steps, precision, bc=bc, checkpoints=[1, 2, steps])
        _assert_bar(errs, bar, ("walls", nu))
        bc = [(pgk.DIRICHLET, 1.01, (0.02, 0.0, 0.0), 1.02 * th0), (pgk.DIRICHLET, 0.99, (0.02, 0.0, 0.0), th0)]
        errs, _ = run_pair(nx, 1, 1, f, p, steps, precision, bc=bc, checkpoints=[1, steps])
        _assert_bar(errs, bar, ("dirichlet", nu))
        if nu > 0.1:
            errs, _ = run_pair(nx, 1, 1, f, p, steps, precision, checkpoints=[1, steps])
            _assert_bar(errs, bar, ("periodic", nu))
    # the printed (LIT) variant on the same path, and 78 sub-steps: beyond the
    # halo the work-groups hold, so the transport falls back to 1 + n_sub launches
    p = resolve(0.5, 0.71, 0.8, 2.0)
    bc = [(pgk.WALL, 1.0, (0.0, 0.0, 0.0), 0.95 * th0), (pgk.WALL, 1.0, (0.0, 0.03, 0.0), 1.05 * th0)]
    errs, _ = run_pair(nx, 1, 1, f, p, 10, precision, variant=1, bc=bc, checkpoints=[1, 10])
    _assert_bar(errs, bar, "walls, printed variant")
    p = resolve(15.0, 0.71, 0.8, 2.0)
    errs, _ = run_pair(nx, 1, 1, f, p, 4, precision, checkpoints=[1, 4])
    _assert_bar(errs, bar, "periodic, 78 sub-steps")


@pytest.mark.parametrize("precision,bar", [(0, 1e-12), (1, 1e-5)])
def test_dirichlet_face_state_changed_mid_run(precision, bar):
    # Dirichlet ghosts are written once per face state: a new state given
    # between calls must reach the next step (graph-replayed and direct)
    import paper_2201_05280_amd as pgk
    th0 = oracle.THETA0
    bc = [(pgk.DIRICHLET, 1.02, (0.03, 0.0, 0.0), th0 * 1.01), (pgk.DIRICHLET, 0.99, (0.03, 0.0, 0.0), th0)]
    f = inputs.uniform(32, 1, 1, u=(0.03, 0, 0))
    p = resolve(0.05, 0.71, 0.8, 2.0)
    s = _solver(32, 1, 1, precision=precision, bc_x=(pgk.DIRICHLET, pgk.DIRICHLET))
    o = oracle.Oracle(32, 1, 1)
    for r in (s, o):
        r.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
    for side in (0, 1):
        kind, rho, u, th = bc[side]
        s.set_bc_x(side, rho, u, th)
        o.set_bc_x(side, kind, rho, u, th)
    s.init(f["rho"], f["u"], f["thT"], f["thR"])
    o.init(f["rho"], f["u"], f["thT"], f["thR"])
    errs = []
    for n, new in ((70, (1.05, (0.0, 0.0, 0.0), th0 * 1.1)), (3, (0.97, (0.05, 0.0, 0.0), th0 * 0.95)), (40, None)):
        s.step(n)
        o.step(n)
        errs.append(rel_err(s.moments(), o.moments()))
        if new is not None:
            s.set_bc_x(0, *new)
            o.set_bc_x(0, oracle.DIRICHLET, *new)
    s.close()
    _assert_bar(errs, bar, "dirichlet change")


@pytest.mark.parametrize("precision,bar", [(0, 1e-12), (1, 1e-5)])
@pytest.mark.parametrize("nx", [2, 3])
def test_thinnest_bounded_grids(precision, bar, nx):
    # the fewest cells between two faces: populations with |c_x| = 2 reach
    # past the opposite face's first cell, every pull near a face reads ghosts
    import paper_2201_05280_amd as pgk
    th0 = oracle.THETA0
    p = resolve(0.05, 0.71, 0.8, 2.0)
    walls = [(pgk.WALL, 1.0, (0.0, 0.0, 0.0), th0), (pgk.WALL, 1.0, (0.0, 0.03, 0.0), th0 * 1.05)]
    errs, _ = run_pair(nx, 3, 2, inputs.uniform(nx, 3, 2), p, 50, precision, bc=walls, checkpoints=[1, 2, 50])
    _assert_bar(errs, bar, ("walls", nx))
    dirichlet = [(pgk.DIRICHLET, 1.01, (0.02, 0.0, 0.0), th0), (pgk.DIRICHLET, 0.99, (0.02, 0.0, 0.0), th0 * 0.98)]
    errs, _ = run_pair(nx, 1, 1, inputs.uniform(nx, 1, 1, u=(0.02, 0, 0)), p, 50, precision, bc=dirichlet,
                       checkpoints=[1, 2, 50])
    _assert_bar(errs, bar, ("dirichlet", nx))
