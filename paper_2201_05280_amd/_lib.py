"""ctypes binding of libpgk.so (the C ABI declared in include/pgk.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  Importing this module does not need a GPU; loading the
library does need the built libpgk.so, and creating a solver needs a HIP
device.  There is no fallback: a missing library or device raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpgk.so")

PGK_OK = 0
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EINFEASIBLE", -6: "ENOTBOUND", -7: "ETOOBIG"}
MLP_STATIC_NMAX = 4096
FP64, FP32DEV = 0, 1
CN, LIT = 0, 1
F3 = 0
E2 = 1
F4 = 2
PERIODIC, WALL, DIRICHLET = 0, 1, 2
NBUF = 4

# every symbol include/pgk.h declares
EXPORTS = ["pgk_resolve", "pgk_lattice", "pgk_equilibrium", "pgk_buffer_sizes", "pgk_create", "pgk_bind", "pgk_set_params",
           "pgk_set_bc", "pgk_set_bc_x", "pgk_init_fields", "pgk_step", "pgk_read_moments", "pgk_conserved",
           "pgk_set_graph_steps", "pgk_set_transport_reference", "pgk_set_timing", "pgk_kernel_times", "pgk_get_clock", "pgk_set_clock", "pgk_steps_done", "pgk_last_error", "pgk_destroy",
           "pgk_batch_bytes", "pgk_batch_create", "pgk_batch_offsets", "pgk_batch_init", "pgk_batch_config",
           "pgk_batch_run", "pgk_batch_stall", "pgk_batch_tuned", "pgk_batch_read_moments", "pgk_batch_last_error",
           "pgk_batch_destroy", "pgk_mlp_bytes", "pgk_mlp_create", "pgk_mlp_set_params", "pgk_mlp_get_params",
           "pgk_mlp_forward", "pgk_mlp_loss_grad", "pgk_mlp_adam_step", "pgk_mlp_train", "pgk_mlp_get_state",
           "pgk_mlp_set_state", "pgk_mlp_save", "pgk_mlp_load", "pgk_mlp_last_error", "pgk_mlp_destroy",
           "pgk_mlp_forward_static"]
MLP_NPARAM = 50948
CASE_RUNNING, CASE_CONVERGED, CASE_DIVERGED, CASE_MAXSTEPS, CASE_STALLED = 0, 1, 2, 3, 4
NKERNEL = 4
KERNEL_NAMES = ["k_lb", "k_mc", "k_dif", "k_bc"]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("precision", ctypes.c_int), ("variant", ctypes.c_int), ("equilibrium", ctypes.c_int),
                ("bc_x", ctypes.c_int * 2), ("bc_y", ctypes.c_int * 2)]


class Clock(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("cur", ctypes.c_int), ("ghosts_ok", ctypes.c_int),
                ("face_changed", ctypes.c_int)]


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("tau", "tau1", "b", "kr", "delta", "theta0")]


class Targets(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("nu", "Pr", "mub_over_mu", "delta", "b", "kr", "theta0")]


class Resolved(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "tau", "tau1", "b", "kr", "delta", "theta0", "tau_star", "beta", "X", "Y", "s_sigma", "B",
        "nu", "mub_over_mu", "Pr", "gamma", "D_R")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Case(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int), ("bc", ctypes.c_int), ("vel_axis", ctypes.c_int), ("variant", ctypes.c_int),
                ("p", Params), ("rho", ctypes.c_double * 2), ("u", (ctypes.c_double * 3) * 2),
                ("theta", ctypes.c_double * 2), ("equilibrium", ctypes.c_int)]


_lib = None


def load():
    """Load libpgk.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpgk.so is not built: run `python -m paper_2201_05280_amd.build` "
                           "(or __graft_entry__.build()) first")
    # torch ships its own HIP runtime under the same soname as /opt/rocm's;
    # let torch load and initialise it first so that one runtime serves both
    import torch
    if torch.cuda.is_available():
        torch.cuda.init()
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64
    sz = ctypes.c_size_t
    L.pgk_resolve.argtypes = [ctypes.POINTER(Targets), ctypes.POINTER(Resolved)]
    L.pgk_buffer_sizes.argtypes = [ctypes.POINTER(Grid), sz * NBUF]
    L.pgk_create.argtypes = [ctypes.POINTER(Grid), vp, ctypes.POINTER(vp)]
    L.pgk_bind.argtypes = [vp, vp * NBUF, sz * NBUF]
    L.pgk_set_params.argtypes = [vp, ctypes.POINTER(Params), ctypes.POINTER(Resolved)]
    L.pgk_set_bc.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, ctypes.c_double]
    L.pgk_set_bc_x.argtypes = [vp, ctypes.c_int, ctypes.c_double, dp, ctypes.c_double]
    L.pgk_init_fields.argtypes = [vp, vp, vp, vp, vp]
    L.pgk_step.argtypes = [vp, i64]
    L.pgk_read_moments.argtypes = [vp, vp, vp, vp, vp, vp]
    L.pgk_conserved.argtypes = [vp, dp]
    L.pgk_set_graph_steps.argtypes = [vp, ctypes.c_int]
    L.pgk_set_transport_reference.argtypes = [vp, ctypes.c_int]
    L.pgk_set_timing.argtypes = [vp, ctypes.c_int]
    L.pgk_kernel_times.argtypes = [vp, ctypes.c_double * NKERNEL, ctypes.c_int64 * NKERNEL]
    L.pgk_get_clock.argtypes = [vp, ctypes.POINTER(Clock)]
    L.pgk_set_clock.argtypes = [vp, ctypes.POINTER(Clock)]
    L.pgk_steps_done.argtypes = [vp]
    L.pgk_steps_done.restype = i64
    L.pgk_last_error.argtypes = [vp]
    L.pgk_last_error.restype = ctypes.c_char_p
    L.pgk_destroy.argtypes = [vp]
    L.pgk_destroy.restype = None
    cp = ctypes.POINTER(Case)
    L.pgk_batch_bytes.argtypes = [cp, ctypes.c_int, ctypes.POINTER(sz)]
    L.pgk_batch_create.argtypes = [cp, ctypes.c_int, vp, vp, sz, ctypes.POINTER(vp)]
    L.pgk_batch_offsets.argtypes = [vp, ctypes.POINTER(i64)]
    L.pgk_batch_init.argtypes = [vp, vp, vp, vp, vp]
    L.pgk_batch_config.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.pgk_batch_run.argtypes = [vp, i64, ctypes.c_double, ctypes.POINTER(i64), dp, ctypes.POINTER(ctypes.c_int)]
    L.pgk_batch_tuned.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), dp]
    L.pgk_batch_read_moments.argtypes = [vp, vp, vp, vp, vp]
    L.pgk_batch_last_error.argtypes = [vp]
    L.pgk_batch_last_error.restype = ctypes.c_char_p
    L.pgk_batch_destroy.argtypes = [vp]
    L.pgk_batch_destroy.restype = None
    fp = ctypes.POINTER(ctypes.c_float)
    L.pgk_mlp_bytes.argtypes = [ctypes.c_int, ctypes.POINTER(sz)]
    L.pgk_mlp_create.argtypes = [vp, vp, sz, ctypes.c_int, ctypes.POINTER(vp)]
    L.pgk_mlp_set_params.argtypes = [vp, vp]
    L.pgk_mlp_get_params.argtypes = [vp, vp]
    L.pgk_mlp_forward.argtypes = [vp, vp, vp, ctypes.c_int]
    L.pgk_mlp_loss_grad.argtypes = [vp, vp, vp, ctypes.c_int, vp, fp]
    L.pgk_mlp_adam_step.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]
    L.pgk_mlp_train.argtypes = [vp, vp, vp, i64, ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_uint64, fp]
    L.pgk_mlp_get_state.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(i64)]
    L.pgk_mlp_set_state.argtypes = [vp, vp, vp, vp, i64]
    L.pgk_mlp_save.argtypes = [vp, ctypes.c_char_p]
    L.pgk_mlp_load.argtypes = [vp, ctypes.c_char_p]
    L.pgk_mlp_forward_static.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    L.pgk_mlp_last_error.argtypes = [vp]
    L.pgk_mlp_last_error.restype = ctypes.c_char_p
    L.pgk_mlp_destroy.argtypes = [vp]
    L.pgk_mlp_destroy.restype = None
    for name in EXPORTS:
        if name not in ("pgk_steps_done", "pgk_last_error", "pgk_destroy", "pgk_batch_last_error",
                        "pgk_batch_destroy", "pgk_mlp_last_error", "pgk_mlp_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def lattice(theta0=0.0):
    """(c[41][3], w[41]) of the library's velocity order (host only)."""
    import numpy as np
    L = load()
    c = np.zeros((41, 3))
    w = np.zeros(41)
    P = ctypes.POINTER(ctypes.c_double)
    L.pgk_lattice(ctypes.c_double(theta0), c.ctypes.data_as(P), w.ctypes.data_as(P))
    return c, w


def equilibrium(kind, rho, u, lam6, theta0=0.0):
    """Populations F[41] (library order) of the F3, E2 or F4 equilibrium (host
    only); raises ValueError when E2 has no solution."""
    import numpy as np
    L = load()
    P = ctypes.POINTER(ctypes.c_double)
    u = np.ascontiguousarray(u, dtype=np.float64)
    lam = np.ascontiguousarray(lam6, dtype=np.float64)
    F = np.zeros(41)
    rc = L.pgk_equilibrium(int(kind), ctypes.c_double(theta0), ctypes.c_double(rho), u.ctypes.data_as(P),
                           lam.ctypes.data_as(P), F.ctypes.data_as(P))
    if rc != PGK_OK:
        raise ValueError("no %s equilibrium for rho=%g u=%s lam=%s (%s)"
                         % ({E2: "E2", F4: "F4"}.get(kind, "F3"), rho, list(u), list(lam), ERRORS.get(rc, rc)))
    return F


def resolve(nu, Pr, mub_over_mu, delta, b=float("nan"), kr=float("nan"), theta0=0.0):
    """Parameter map of the library (host only): targets -> resolved constants."""
    L = load()
    t = Targets(nu, Pr, mub_over_mu, delta, b, kr, theta0)
    r = Resolved()
    rc = L.pgk_resolve(ctypes.byref(t), ctypes.byref(r))
    if rc != PGK_OK:
        raise ValueError("pgk_resolve failed: %s" % ERRORS.get(rc, rc))
    return r.as_dict()


def buffer_sizes(nx, ny, nz, precision=FP64, variant=CN, bc_x=(PERIODIC, PERIODIC), bc_y=(PERIODIC, PERIODIC)):
    L = load()
    g = Grid(nx, ny, nz, precision, variant, F3, (ctypes.c_int * 2)(*bc_x), (ctypes.c_int * 2)(*bc_y))
    out = (ctypes.c_size_t * NBUF)()
    rc = L.pgk_buffer_sizes(ctypes.byref(g), out)
    if rc != PGK_OK:
        raise ValueError("bad grid: %s" % ERRORS.get(rc, rc))
    return list(out)
