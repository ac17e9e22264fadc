"""Host-side equilibria of the library (pgk_equilibrium, pgk_lattice) against
the oracle's, and the discrete jump conditions built on them (no GPU)."""
import numpy as np
import pytest

import oracle
from paper_2201_05280_amd import _lib
from paper_2201_05280_amd.shock import discrete_rankine_hugoniot, equilibrium_fluxes


def _order():
    c, w = _lib.lattice()
    co, wo = oracle.lattice()
    idx = [int(np.flatnonzero((np.abs(co - ci) < 1e-12).all(1))[0]) for ci in c]
    assert sorted(idx) == list(range(41))
    assert np.allclose(w, wo[idx], rtol=1e-15, atol=0)
    return idx


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_library_equilibria_equal_the_oracles(seed):
    idx = _order()
    rng = np.random.default_rng(seed)
    for _ in range(10):
        rho = 1 + 0.2 * rng.uniform(-1, 1)
        u = 0.35 * rng.uniform(-1, 1, 3)
        lam = np.array([0.3, 0.27, 0.32, 0.01, -0.015, 0.004]) * (1 + 0.1 * rng.uniform(-1, 1))
        Fo, it = oracle.feq_e2(rho, u, lam)
        assert it > 0
        F = _lib.equilibrium(_lib.E2, rho, u, lam)
        assert np.abs(F - Fo[idx]).max() <= 1e-13 * np.abs(Fo).max()
        F3o = oracle.feq_f3(rho, u, lam)
        F3 = _lib.equilibrium(_lib.F3, rho, u, lam)
        assert np.abs(F3 - F3o[idx]).max() <= 1e-13 * np.abs(F3o).max()
        F4o = oracle.feq_f4(rho, u, lam)
        F4 = _lib.equilibrium(_lib.F4, rho, u, lam)
        assert np.abs(F4 - F4o[idx]).max() <= 1e-13 * np.abs(F4o).max()


def test_e2_refuses_a_state_off_the_lattice():
    with pytest.raises(ValueError):
        _lib.equilibrium(_lib.E2, 1.0, (0.4, 0.0, 0.0), (0.05, 0.05, 0.05, 0, 0, 0))


def test_mach_3_upstream_state_needs_a_cold_or_warm_gas():
    # with the upstream at the lattice temperature, u = 3 c_s lies beyond what a
    # positive distribution on the 41 velocities can carry; theta1 = 0.08 works
    from paper_2201_05280_amd.inputs import rankine_hugoniot
    (r1, u1, t1), _ = rankine_hugoniot(3.0, 1.4, oracle.THETA0)
    with pytest.raises(ValueError):
        _lib.equilibrium(_lib.E2, r1, (u1, 0, 0), (t1, t1, t1, 0, 0, 0))
    (r1, u1, t1), _ = rankine_hugoniot(3.0, 1.4, 0.08)
    _lib.equilibrium(_lib.E2, r1, (u1, 0, 0), (t1, t1, t1, 0, 0, 0))


@pytest.mark.parametrize("Ma,theta1", [(1.5, oracle.THETA0), (3.0, 0.08)])
def test_discrete_jump_conditions(Ma, theta1):
    up, down = discrete_rankine_hugoniot(Ma, 2.0, theta1)
    fu, fd = equilibrium_fluxes(*up, 2.0), equilibrium_fluxes(*down, 2.0)
    assert np.abs(fu - fd).max() <= 1e-12 * np.abs(fu).max()
    # mass and momentum fluxes are the exact second-order moments
    assert abs(fu[0] - up[0] * up[1]) < 1e-14
    assert abs(fu[1] - up[0] * (up[1] ** 2 + up[2])) < 1e-13
    # the same jump from the oracle's E2 (an independent implementation)
    co, _ = oracle.lattice()
    cx, c2 = co[:, 0], (co ** 2).sum(1)

    def flux_o(r, u, t):
        F, it = oracle.feq_e2(r, np.array([u, 0, 0.]), np.array([t, t, t, 0, 0, 0.]))
        return np.array([F @ cx, F @ cx ** 2, 0.5 * F @ (cx * c2) + r * u * t])

    assert np.abs(flux_o(*down) - flux_o(*up)).max() <= 1e-11 * np.abs(fu).max()
    # close to the ideal-gas jump (within the E2 energy-flux error at this Mach number)
    from paper_2201_05280_amd.inputs import rankine_hugoniot
    _, ideal = rankine_hugoniot(Ma, 1.4, theta1)
    assert np.abs(np.array(down) / np.array(ideal) - 1).max() < 0.02
