"""FP64 CPU oracle for the reduced polyatomic ES-BGK lattice-Boltzmann step.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product (the HIP library under
``paper_2201_05280_amd``) never imports this package and shares no code with it.

The arithmetic lives in ``pgk_oracle.c`` (plain C, double precision, loops over
sites and velocities in the paper's order); this module only marshals numpy
arrays through ctypes.  ``params.py`` holds the oracle's own copy of the
paper's transport-coefficient formulas (Sec. 4, hydrodynamics).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libpgk_oracle.so")
_SRC = os.path.join(_HERE, "pgk_oracle.c")

PERIODIC, WALL, DIRICHLET = 0, 1, 2
CN, LIT = 0, 1
F3, E2, F4 = 0, 1, 2
THETA0 = 0.2948964908710633  # lattice reference temperature, Table of weights

_lib = None


def build(verbose=False):
    """Compile the oracle with gcc (-O2, OpenMP)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99", "-Wall",
           "-o", _LIB, _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.pgko_create.restype = vp
        L.pgko_create.argtypes = [ctypes.c_int] * 5
        L.pgko_destroy.argtypes = [vp]
        L.pgko_sites.argtypes = [vp]
        L.pgko_threads.restype = ctypes.c_int
        L.pgko_set_params.argtypes = [vp] + [ctypes.c_double] * 6
        L.pgko_set_bc_x.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, ctypes.c_double]
        L.pgko_set_bc.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, ctypes.c_double]
        L.pgko_init.argtypes = [vp, dp, dp, dp, dp]
        L.pgko_step.argtypes = [vp, ctypes.c_long]
        L.pgko_moments.argtypes = [vp, dp, dp, dp, dp, dp]
        L.pgko_conserved.argtypes = [vp, dp]
        L.pgko_lattice.argtypes = [ctypes.c_double, dp, dp]
        L.pgko_feq_f3.argtypes = [ctypes.c_double, dp, dp, ctypes.c_double, dp, dp, dp]
        L.pgko_feq_e2.argtypes = [ctypes.c_double, dp, dp, ctypes.c_double, dp, dp, dp]
        L.pgko_feq_f4.argtypes = [ctypes.c_double, dp, dp, ctypes.c_double, dp, dp, dp]
        L.pgko_feq_e2.restype = ctypes.c_int
        L.pgko_collide_site.argtypes = [vp, dp, ctypes.c_double, dp, dp]
        L.pgko_get_state.argtypes = [vp, dp, dp]
        L.pgko_set_state.argtypes = [vp, dp, dp]
        L.pgko_substeps.argtypes = [vp]
        L.pgko_substeps.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def threads():
    return int(lib().pgko_threads())


def lattice(theta0=THETA0):
    """RD3Q41 velocities (41x3) and weights (41) from the Table of weights."""
    c = np.zeros((41, 3))
    w = np.zeros(41)
    lib().pgko_lattice(theta0, _p(c), _p(w))
    return c, w


def feq_f3(rho, u, lam6, theta0=THETA0):
    c, w = lattice(theta0)
    F = np.zeros(41)
    lib().pgko_feq_f3(theta0, _p(w), _p(c), float(rho), _p(np.ascontiguousarray(u, dtype=np.float64)),
                      _p(np.ascontiguousarray(lam6, dtype=np.float64)), _p(F))
    return F


def feq_f4(rho, u, lam6, theta0=THETA0):
    """F3 plus the contracted fourth-order Hermite terms (exact contracted fourth moment)."""
    c, w = lattice(theta0)
    F = np.zeros(41)
    lib().pgko_feq_f4(theta0, _p(w), _p(c), float(rho), _p(np.ascontiguousarray(u, dtype=np.float64)),
                      _p(np.ascontiguousarray(lam6, dtype=np.float64)), _p(F))
    return F


def feq_e2(rho, u, lam6, theta0=THETA0):
    """Discrete quasi-equilibrium; returns (F, iterations) with iterations < 0 on failure."""
    c, w = lattice(theta0)
    F = np.zeros(41)
    it = lib().pgko_feq_e2(theta0, _p(w), _p(c), float(rho), _p(np.ascontiguousarray(u, dtype=np.float64)),
                           _p(np.ascontiguousarray(lam6, dtype=np.float64)), _p(F))
    return F, int(it)


class Oracle:
    """One periodic (or x-bounded) bcc grid of nx*ny*nz cells = 2*nx*ny*nz sites.

    Site order of every field: [sub][z][y][x] (sub 0 = corner sites at integer
    positions, sub 1 = body-centre sites offset by (1/2,1/2,1/2)).
    """

    def __init__(self, nx, ny, nz, variant=CN, equilibrium=F3):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.ns = 2 * nx * ny * nz
        self.variant = variant
        self._h = lib().pgko_create(nx, ny, nz, variant, equilibrium)
        if not self._h:
            raise ValueError("bad grid")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().pgko_destroy(h)
            self._h = None

    def set_params(self, tau, tau1, b, kr, delta, theta0=THETA0):
        rc = lib().pgko_set_params(self._h, tau, tau1, b, kr, delta, theta0)
        if rc != 0:
            raise ValueError("bad parameters")

    def set_bc(self, axis, side, kind, rho=1.0, u=(0.0, 0.0, 0.0), theta=THETA0):
        """Face `side` (0 low, 1 high) of axis `axis` (0 x, 1 y; z is periodic)."""
        uu = np.ascontiguousarray(u, dtype=np.float64)
        if lib().pgko_set_bc(self._h, int(axis), int(side), int(kind), float(rho), _p(uu), float(theta)) != 0:
            raise ValueError("bad face")

    def set_bc_x(self, side, kind, rho=1.0, u=(0.0, 0.0, 0.0), theta=THETA0):
        self.set_bc(0, side, kind, rho, u, theta)

    def init(self, rho, u, thT, thR):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, -1)
        thT = np.ascontiguousarray(thT, dtype=np.float64).reshape(-1)
        thR = np.ascontiguousarray(thR, dtype=np.float64).reshape(-1)
        assert rho.size == self.ns and u.shape[1] == self.ns
        rc = lib().pgko_init(self._h, _p(rho), _p(u), _p(thT), _p(thR))
        if rc != 0:
            raise RuntimeError("equilibrium failed at initialisation")

    def step(self, n=1):
        rc = lib().pgko_step(self._h, int(n))
        if rc != 0:
            raise RuntimeError("oracle step failed (%d)" % rc)

    def moments(self):
        ns = self.ns
        rho = np.zeros(ns)
        u = np.zeros((3, ns))
        thT = np.zeros(ns)
        thR = np.zeros(ns)
        P = np.zeros((6, ns))
        lib().pgko_moments(self._h, _p(rho), _p(u), _p(thT), _p(thR), _p(P))
        return dict(rho=rho, u=u, thT=thT, thR=thR, P=P)

    def conserved(self):
        out = np.zeros(5)
        lib().pgko_conserved(self._h, _p(out))
        return out

    def substeps(self):
        """FTCS sub-steps the theta_R diffusion takes per time step."""
        return int(lib().pgko_substeps(self._h))

    def collide_site(self, g, er):
        g = np.ascontiguousarray(g, dtype=np.float64)
        go = np.zeros(41)
        info = np.zeros(5)
        rc = lib().pgko_collide_site(self._h, _p(g), float(er), _p(go), _p(info))
        if rc != 0:
            raise RuntimeError("collision failed")
        return go, dict(rho=info[0], T=info[1], R=info[2], theta=info[3], a=info[4])

    def get_state(self):
        g = np.zeros((41, self.ns))
        er = np.zeros(self.ns)
        lib().pgko_get_state(self._h, _p(g), _p(er))
        return g, er

    def set_state(self, g, er):
        g = np.ascontiguousarray(g, dtype=np.float64)
        er = np.ascontiguousarray(er, dtype=np.float64)
        assert g.shape == (41, self.ns) and er.shape == (self.ns,)
        lib().pgko_set_state(self._h, _p(g), _p(er))
