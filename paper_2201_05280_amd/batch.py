"""Batched sweep of independent 1D cases (front end of the pgk_batch_* ABI).

Device memory comes from torch; every step runs in the library's persistent
HIP kernel.  A case is a dict:
  L         cells along x
  bc        WALL (Couette between diffuse walls) or DIRICHLET (shock faces)
  vel_axis  velocity component for the residual (Couette: 1, shock: 0)
  variant   CN or LIT
  params    (tau, tau1, b, kr, delta[, theta0])
  rho, u, theta   face data: pairs for the low and high x faces
  equilibrium     F3 or E2
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import CN


def make_case(L, bc, params, rho=(1.0, 1.0), u=((0, 0, 0), (0, 0, 0)), theta=(0.2948964908710633,) * 2,
              vel_axis=1, variant=CN, equilibrium=_lib.F3):
    c = _lib.Case()
    c.L, c.bc, c.vel_axis, c.variant = int(L), int(bc), int(vel_axis), int(variant)
    c.equilibrium = int(equilibrium)
    p = list(params) + [0.0] * (6 - len(params))
    c.p = _lib.Params(*p)
    for s in range(2):
        c.rho[s] = rho[s]
        c.theta[s] = theta[s]
        for a in range(3):
            c.u[s][a] = u[s][a]
    return c


class Batch:
    def __init__(self, cases, device=0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the batched sweep runs only on the GPU")
        self.torch = torch
        self.L = _lib.load()
        self.n = len(cases)
        self.arr = (_lib.Case * self.n)(*cases)
        nb = ctypes.c_size_t()
        rc = self.L.pgk_batch_bytes(self.arr, self.n, ctypes.byref(nb))
        if rc:
            raise ValueError("invalid case table (%s)" % _lib.ERRORS.get(rc, rc))
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.buf = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        rc = self.L.pgk_batch_create(self.arr, self.n, ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.c_void_p(self.buf.data_ptr()), nb.value, ctypes.byref(h))
        if rc:
            raise RuntimeError("pgk_batch_create failed (%s)" % _lib.ERRORS.get(rc, rc))
        self.h = h
        off = (ctypes.c_int64 * (self.n + 1))()
        self.L.pgk_batch_offsets(self.h, off)
        self.off = np.array(list(off), dtype=np.int64)
        self.ns = int(self.off[-1])

    def _check(self, rc):
        if rc:
            raise RuntimeError("pgk batch error %s: %s" % (_lib.ERRORS.get(rc, rc),
                                                           self.L.pgk_batch_last_error(self.h).decode()))

    def close(self):
        if getattr(self, "h", None):
            self.torch.cuda.synchronize(self.device)
            self.L.pgk_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, rho, u, thT, thR):
        t = self.torch
        f = [t.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(sh), device=self.device)
             for a, sh in ((rho, (self.ns,)), (u, (3, self.ns)), (thT, (self.ns,)), (thR, (self.ns,)))]
        self.torch.cuda.current_stream(self.device).synchronize()
        self._check(self.L.pgk_batch_init(self.h, *[x.data_ptr() for x in f]))

    def config(self, wg=0, K=0):
        self._check(self.L.pgk_batch_config(self.h, wg, K))

    def stall(self, window):
        """Stop a case as STALLED after `window` steps without halving its best residual (0: off)."""
        self._check(self.L.pgk_batch_stall(self.h, ctypes.c_int64(int(window))))

    def run(self, max_steps, tol):
        steps = (ctypes.c_int64 * self.n)()
        resid = (ctypes.c_double * self.n)()
        status = (ctypes.c_int * self.n)()
        self._check(self.L.pgk_batch_run(self.h, int(max_steps), float(tol), steps, resid, status))
        return np.array(list(steps)), np.array(list(resid)), np.array(list(status))

    def tuned(self):
        wg, K, ns = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self._check(self.L.pgk_batch_tuned(self.h, ctypes.byref(wg), ctypes.byref(K), ctypes.byref(ns)))
        return wg.value, K.value, ns.value

    def moments(self):
        t, ns = self.torch, self.ns
        out = dict(rho=t.empty(ns, dtype=t.float64, device=self.device),
                   u=t.empty(3, ns, dtype=t.float64, device=self.device),
                   thT=t.empty(ns, dtype=t.float64, device=self.device),
                   thR=t.empty(ns, dtype=t.float64, device=self.device))
        self._check(self.L.pgk_batch_read_moments(self.h, out["rho"].data_ptr(), out["u"].data_ptr(),
                                                  out["thT"].data_ptr(), out["thR"].data_ptr()))
        self.stream.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}

    def checkpoint(self):
        """A copy of the batch buffer: every case's populations, theta_R, step
        count, residual and status live there, so restore() of it continues
        bit for bit under a fixed config (an autotuned run may choose other
        chunk lengths after a resume; stall windows restart)."""
        self.stream.synchronize()
        b = self.buf.clone()
        self.torch.cuda.current_stream(self.device).synchronize()
        return b

    def restore(self, ckpt):
        if ckpt.numel() != self.buf.numel():
            raise ValueError("checkpoint of a different batch")
        self.stream.synchronize()
        self.buf.copy_(ckpt)
        self.torch.cuda.current_stream(self.device).synchronize()

    def case_slice(self, c):
        return slice(int(self.off[c]), int(self.off[c + 1]))
