"""The theta_R transport (Sec. 5, steps 2-4) by its LDS kernels against its
plain global-memory kernels (`pgk_set_transport_reference`), on the grid
shapes that select each LDS kernel: the fused periodic kernel (tiles of
64 x 8 x 128 with ragged edges and several z-chunks), the one-work-group
kernel of small bounded or sub-cycled grids, and the line kernel of long lines
(halo of n_sub + 1 cells).  The one-work-group kernel runs the reference
kernels' per-site code, so every moment must agree bit for bit after many
steps; the fused periodic and line kernels evaluate the same formulas in the
same order, but the compiler fuses their multiply-adds differently (a last
bit differs here and there), so they agree to round-off (FP64 storage 1e-13
after 25 steps, FP32 storage 1e-6, where a last-bit flip of a population can
follow).  A missing barrier or a halo indexing slip in an LDS kernel shows as
a difference far above those bars (GPU only)."""
import numpy as np
import pytest

import oracle
from oracle.params import resolve
from paper_2201_05280_amd import inputs

pytestmark = pytest.mark.gpu


def _run(dims, p, f, precision, bc, reference, steps):
    import paper_2201_05280_amd as pgk
    kinds = (pgk.PERIODIC, pgk.PERIODIC) if bc is None else (bc[0][0], bc[1][0])
    s = pgk.Solver(*dims, precision=precision, bc_x=kinds)
    s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
    if bc is not None:
        for side in (0, 1):
            kind, rho, u, th = bc[side]
            s.set_bc_x(side, rho, u, th)
    s.set_transport_reference(reference)
    s.init(f["rho"], f["u"], f["thT"], f["thR"])
    s.step(steps)
    m = s.moments()
    s.close()
    return m


def _cases():
    import paper_2201_05280_amd as pgk
    th0 = oracle.THETA0
    walls = [(pgk.WALL, 1.0, (0.0, 0.0, 0.0), 0.95 * th0), (pgk.WALL, 1.0, (0.0, 0.03, 0.0), 1.05 * th0)]
    low, high = resolve(0.02, 0.71, 0.8, 2.0), resolve(0.5, 0.71, 0.8, 2.0)
    return [
        ("fused periodic, ragged tiles", (70, 20, 9), low, None, False),
        ("fused periodic, three z-chunks", (16, 9, 260), low, None, False),
        ("line, walls, 24 cells", (24, 1, 1), low, walls, False),
        ("one work-group, walls, 3D columns", (6, 5, 3), high, walls, True),
        ("one work-group, periodic sub-cycled", (10, 6, 1), high, None, True),
        ("line, walls, 3 sub-steps", (2100, 1, 1), high, walls, False),
        ("line, periodic, 3 sub-steps", (2049, 1, 1), high, None, False),
    ]


FLOOR = dict(rho=0.0, u=1e-2, thT=0.0, thR=0.0, P=0.0)


@pytest.mark.parametrize("precision", [0, 1])
def test_lds_transport_kernels_match_the_reference_kernels(precision):
    bar = 1e-13 if precision == 0 else 1e-6
    for label, dims, p, bc, bitwise in _cases():
        f = inputs.random_smooth(*dims, seed=sum(dims), amp_u=0.03, amp_th=0.05)
        a = _run(dims, p, f, precision, bc, False, 25)
        b = _run(dims, p, f, precision, bc, True, 25)
        for k in FLOOR:
            diff = float(np.abs(a[k] - b[k]).max())
            if bitwise:
                assert np.array_equal(a[k], b[k]), (label, precision, k, diff)
            else:
                err = diff / max(float(np.abs(b[k]).max()), FLOOR[k])
                assert err <= bar, (label, precision, k, err)


def _line_substeps(p, th_max):
    """FTCS sub-steps per step of the theta_R diffusion on a line: the host
    rule n = ceil(3 D_R), D_R = 5 k_r theta tau / (B delta), B = 1 + tau/tau1,
    theta the largest of theta0 and the face temperatures."""
    B = 1.0 + p["tau"] / p["tau1"]
    return int(np.ceil(3.0 * 5.0 * p["kr"] * th_max * p["tau"] / (B * p["delta"])))


def _nu_for_substeps(n, th_max):
    """A viscosity in the middle of the range whose line diffusion takes
    exactly n sub-steps (clear of the rounding at either end)."""
    def first_nu_with(m):
        lo, hi = 1e-3, 100.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if _line_substeps(resolve(mid, 0.71, 0.8, 2.0), th_max) < m:
                lo = mid
            else:
                hi = mid
        return hi
    nu = 0.5 * (first_nu_with(n) + first_nu_with(n + 1))
    assert _line_substeps(resolve(nu, 0.71, 0.8, 2.0), th_max) == n
    return nu


@pytest.mark.parametrize("precision", [0, 1])
def test_line_kernel_at_its_sub_step_limit(precision):
    """Lines between walls at 15 and 16 sub-steps (the last count with
    one-wavefront windows, each producing 64 - 32 = 32 cells, and the first
    with 256-thread windows), at 63 (the line kernel's limit: each work-group
    then produces 256 - 128 = 128 cells, so a 2100-cell line takes 17
    work-groups per sublattice) and at 64 (beyond it; with 4200 sites, more
    than the one-work-group kernel takes, the reference kernels run): the
    timing records show which path ran, and the line kernel matches the
    reference kernels to round-off."""
    import paper_2201_05280_amd as pgk
    th0 = oracle.THETA0
    walls = [(pgk.WALL, 1.0, (0.0, 0.0, 0.0), 0.95 * th0), (pgk.WALL, 1.0, (0.0, 0.03, 0.0), 1.05 * th0)]
    bar = 1e-13 if precision == 0 else 1e-6
    dims, steps = (2100, 1, 1), 12
    for n in (15, 16, 63, 64):
        p = resolve(_nu_for_substeps(n, 1.05 * th0), 0.71, 0.8, 2.0)
        f = inputs.random_smooth(*dims, seed=n, amp_u=0.03, amp_th=0.05)
        s = pgk.Solver(*dims, precision=precision, bc_x=(pgk.WALL, pgk.WALL))
        s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
        for side in (0, 1):
            _, rho, u, th = walls[side]
            s.set_bc_x(side, rho, u, th)
        s.init(f["rho"], f["u"], f["thT"], f["thR"])
        s.set_timing(True)
        s.step(steps)
        kt = s.kernel_times()
        a = s.moments()
        s.close()
        # the line kernel is one record per step under the diffusion entry; the
        # reference path records its MacCormack launch and then its sub-steps
        assert kt["k_dif"][1] == steps, kt
        assert kt["k_mc"][1] == (0 if n <= 63 else steps), kt
        b = _run(dims, p, f, precision, walls, True, steps)
        for k in FLOOR:
            err = float(np.abs(a[k] - b[k]).max()) / max(float(np.abs(b[k]).max()), FLOOR[k])
            assert err <= bar, (n, precision, k, err)
