"""Python front end of the HIP library: device buffers and streams from torch.

Every numerical step runs inside libpgk.so; this class only allocates the
device buffers the library asks for (as torch tensors), passes pointers, and
moves numpy fields to and from the device.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import CN, F3, FP64, PERIODIC


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: the reduced ES-BGK solver runs only on the GPU")
    return torch


class Solver:
    """One grid of nx*ny*nz bcc cells (2 sites per cell) on one GPU.

    precision: _lib.FP64 or _lib.FP32DEV; variant: _lib.CN or _lib.LIT;
    equilibrium: _lib.F3, _lib.E2 or _lib.F4; bc_x, bc_y: kinds of the low and
    high x and y faces (z is periodic).
    """

    def __init__(self, nx, ny, nz, precision=FP64, variant=CN, bc_x=(PERIODIC, PERIODIC),
                 device=0, stream=None, equilibrium=F3, bc_y=(PERIODIC, PERIODIC)):
        torch = _torch()
        self.torch = torch
        self.L = _lib.load()
        self.nx, self.ny, self.nz = nx, ny, nz
        self.ns = 2 * nx * ny * nz
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        g = _lib.Grid(nx, ny, nz, precision, variant, equilibrium, (ctypes.c_int * 2)(*bc_x),
                      (ctypes.c_int * 2)(*bc_y))
        sizes = (ctypes.c_size_t * _lib.NBUF)()
        self._check(self.L.pgk_buffer_sizes(ctypes.byref(g), sizes), None)
        h = ctypes.c_void_p()
        self._check(self.L.pgk_create(ctypes.byref(g), ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(h)), None)
        self.h = h
        # caller-owned device memory: raw byte tensors
        self.bufs = [torch.empty(int(n), dtype=torch.uint8, device=self.device) for n in sizes]
        ptrs = (ctypes.c_void_p * _lib.NBUF)(*[b.data_ptr() for b in self.bufs])
        self._check(self.L.pgk_bind(self.h, ptrs, sizes))
        self.resolved = None

    def _check(self, rc, h="self"):
        if rc != _lib.PGK_OK:
            msg = ""
            if h is not None and getattr(self, "h", None):
                msg = self.L.pgk_last_error(self.h).decode()
            raise RuntimeError("pgk error %s: %s" % (_lib.ERRORS.get(rc, rc), msg))

    def close(self):
        if getattr(self, "h", None):
            self.torch.cuda.synchronize(self.device)
            self.L.pgk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- setup -----------------------------------------------------------
    def set_params(self, tau, tau1, b, kr, delta, theta0=0.0):
        p = _lib.Params(tau, tau1, b, kr, delta, theta0)
        r = _lib.Resolved()
        self._check(self.L.pgk_set_params(self.h, ctypes.byref(p), ctypes.byref(r)))
        self.resolved = r.as_dict()
        return self.resolved

    def set_bc(self, axis, side, rho=1.0, u=(0.0, 0.0, 0.0), theta=0.2948964908710633):
        """State of face `side` (0 low, 1 high) of axis `axis` (0 x, 1 y)."""
        uu = (ctypes.c_double * 3)(*u)
        self._check(self.L.pgk_set_bc(self.h, int(axis), int(side), float(rho), uu, float(theta)))

    def set_bc_x(self, side, rho=1.0, u=(0.0, 0.0, 0.0), theta=0.2948964908710633):
        self.set_bc(0, side, rho, u, theta)

    def _dev(self, a, shape):
        t = self.torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(shape),
                                 device=self.device)
        return t.contiguous()

    def init(self, rho, u, thT, thR):
        """Initial state from host arrays: rho, theta_T, theta_R of ns sites and
        u of [3][ns], site order [sub][z][y][x]."""
        ns = self.ns
        f = [self._dev(rho, (ns,)), self._dev(u, (3, ns)), self._dev(thT, (ns,)), self._dev(thR, (ns,))]
        # the copies ran on torch's current stream; the library works on self.stream
        self.torch.cuda.current_stream(self.device).synchronize()
        self._check(self.L.pgk_init_fields(self.h, *[t.data_ptr() for t in f]))
        self.stream.synchronize()

    def init_device(self, rho, u, thT, thR):
        """Fields already on the device: contiguous float64 tensors of ns (u: 3 x ns)
        values, ready on this solver's stream; they must live until the call returns."""
        ns = self.ns
        for t, n in ((rho, ns), (u, 3 * ns), (thT, ns), (thR, ns)):
            if (t.dtype != self.torch.float64 or not t.is_contiguous() or t.numel() != n
                    or t.device != self.device):
                raise ValueError("init_device needs contiguous float64 tensors of %d values on %s" % (n, self.device))
        self._check(self.L.pgk_init_fields(self.h, rho.data_ptr(), u.data_ptr(), thT.data_ptr(),
                                           thR.data_ptr()))
        self.stream.synchronize()

    # ---- run -------------------------------------------------------------
    def step(self, n=1):
        self._check(self.L.pgk_step(self.h, int(n)))

    def set_graph_steps(self, k):
        """Replay k-step HIP graphs in step() (k even); 0 launches directly."""
        self._check(self.L.pgk_set_graph_steps(self.h, int(k)))

    def set_transport_reference(self, on=True):
        """theta_R transport by the plain global-memory kernels on every grid
        (same bits as the LDS kernels, slower): a check of the LDS kernels."""
        self._check(self.L.pgk_set_transport_reference(self.h, 1 if on else 0))

    def set_timing(self, enable=True):
        self._check(self.L.pgk_set_timing(self.h, 1 if enable else 0))

    def kernel_times(self):
        """{kernel: (total ms, launches)} since timing was enabled or last read."""
        ms = (ctypes.c_double * _lib.NKERNEL)()
        n = (ctypes.c_int64 * _lib.NKERNEL)()
        self._check(self.L.pgk_kernel_times(self.h, ms, n))
        return {name: (ms[i], int(n[i])) for i, name in enumerate(_lib.KERNEL_NAMES)}

    def steps_done(self):
        return int(self.L.pgk_steps_done(self.h))

    # ---- checkpoints -------------------------------------------------------
    def checkpoint(self):
        """The grid's state between steps: copies of the four bound buffers and
        the step clock (pgk_get_clock).  restore() of it continues bit for bit."""
        c = _lib.Clock()
        self._check(self.L.pgk_get_clock(self.h, ctypes.byref(c)))
        self.stream.synchronize()
        bufs = [b.clone() for b in self.bufs]
        self.torch.cuda.current_stream(self.device).synchronize()
        return {"buffers": bufs, "clock": (int(c.steps), int(c.cur), int(c.ghosts_ok), int(c.face_changed))}

    def restore(self, ckpt):
        """Back to a checkpoint of a grid of the same shape, precision and
        equilibrium (parameters and face states are the caller's to set, as
        they were when the checkpoint was taken)."""
        bufs = [self.torch.as_tensor(b) for b in ckpt["buffers"]]
        if len(bufs) != len(self.bufs) or any(a.numel() != b.numel() for a, b in zip(bufs, self.bufs)):
            raise ValueError("checkpoint of a different grid")
        self.stream.synchronize()
        for dst, src in zip(self.bufs, bufs):
            dst.copy_(src.to(self.device))
        self.torch.cuda.current_stream(self.device).synchronize()
        c = _lib.Clock(*ckpt["clock"])
        self._check(self.L.pgk_set_clock(self.h, ctypes.byref(c)))

    def save(self, path):
        """Write a checkpoint to `path` (numpy .npz, no pickled objects)."""
        ck = self.checkpoint()
        arrays = {"buf%d" % i: b.cpu().numpy() for i, b in enumerate(ck["buffers"])}
        np.savez(path, clock=np.array(ck["clock"], dtype=np.int64), **arrays)

    def load(self, path):
        """Restore a checkpoint written by save()."""
        with np.load(path, allow_pickle=False) as d:
            ck = {"buffers": [d["buf%d" % i] for i in range(len(self.bufs))],
                  "clock": tuple(int(v) for v in d["clock"])}
        self.restore(ck)

    def moments_device(self):
        """f-moments as device tensors, written asynchronously on this solver's
        stream (synchronise it before reading them elsewhere)."""
        torch, ns = self.torch, self.ns
        out = dict(rho=torch.empty(ns, dtype=torch.float64, device=self.device),
                   u=torch.empty(3, ns, dtype=torch.float64, device=self.device),
                   thT=torch.empty(ns, dtype=torch.float64, device=self.device),
                   thR=torch.empty(ns, dtype=torch.float64, device=self.device),
                   P=torch.empty(6, ns, dtype=torch.float64, device=self.device))
        self._check(self.L.pgk_read_moments(self.h, out["rho"].data_ptr(), out["u"].data_ptr(),
                                            out["thT"].data_ptr(), out["thR"].data_ptr(),
                                            out["P"].data_ptr()))
        return out

    def moments(self):
        d = self.moments_device()
        self.stream.synchronize()
        return {k: v.cpu().numpy() for k, v in d.items()}

    def conserved(self):
        out = (ctypes.c_double * 5)()
        self._check(self.L.pgk_conserved(self.h, out))
        return np.array(list(out))
