"""Front end of the coordinate MLP (pgk_mlp_* ABI): device memory from torch,
every forward, backward and Adam step in the library's HIP kernels."""
import ctypes

import numpy as np

from . import _lib

NIN, NOUT, NPARAM = 6, 4, _lib.MLP_NPARAM


class MLP:
    def __init__(self, nmax=8192, device=0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the MLP kernels run only on the GPU")
        self.torch = torch
        self.L = _lib.load()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nb = ctypes.c_size_t()
        self._check(self.L.pgk_mlp_bytes(int(nmax), ctypes.byref(nb)), None)
        self.buf = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        self._check(self.L.pgk_mlp_create(ctypes.c_void_p(self.stream.cuda_stream), self.buf.data_ptr(), nb.value,
                                          int(nmax), ctypes.byref(h)), None)
        self.h = h
        self.nmax = nmax

    def _check(self, rc, h="self"):
        if rc:
            msg = self.L.pgk_mlp_last_error(self.h).decode() if h is not None and getattr(self, "h", None) else ""
            raise RuntimeError("pgk mlp error %s: %s" % (_lib.ERRORS.get(rc, rc), msg))

    def close(self):
        if getattr(self, "h", None):
            self.torch.cuda.synchronize(self.device)
            self.L.pgk_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, shape, dtype=None):
        t = self.torch
        if isinstance(a, t.Tensor):
            x = a.to(device=self.device, dtype=t.float32).contiguous()
        else:
            x = t.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=self.device)
        return x.reshape(shape).contiguous()

    def set_params(self, theta):
        th = self._dev(theta, (NPARAM,))
        self._check(self.L.pgk_mlp_set_params(self.h, th.data_ptr()))
        self.stream.synchronize()

    def params(self):
        out = self.torch.empty(NPARAM, dtype=self.torch.float32, device=self.device)
        self._check(self.L.pgk_mlp_get_params(self.h, out.data_ptr()))
        self.stream.synchronize()
        return out.cpu().numpy()

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam update with the gradient of the last loss_grad."""
        self._check(self.L.pgk_mlp_adam_step(self.h, float(lr), float(beta1), float(beta2), float(eps)))
        self.stream.synchronize()

    def state(self):
        """(master FP32, bf16 copies as uint16, Adam m, Adam v, step count) on the host."""
        t = self.torch
        bufs = [t.empty(NPARAM, dtype=dt, device=self.device) for dt in (t.float32, t.int16, t.float32, t.float32)]
        step = ctypes.c_int64()
        self._check(self.L.pgk_mlp_get_state(self.h, *[b.data_ptr() for b in bufs], ctypes.byref(step)))
        self.stream.synchronize()
        master, wbf, m, v = [b.cpu().numpy() for b in bufs]
        return master, wbf.view(np.uint16), m, v, int(step.value)

    def set_state(self, master, m, v, step):
        th, mm, vv = (self._dev(a, (NPARAM,)) for a in (master, m, v))
        self._check(self.L.pgk_mlp_set_state(self.h, th.data_ptr(), mm.data_ptr(), vv.data_ptr(), int(step)))
        self.stream.synchronize()

    def save(self, path):
        self._check(self.L.pgk_mlp_save(self.h, str(path).encode()))

    def load(self, path):
        self._check(self.L.pgk_mlp_load(self.h, str(path).encode()))

    def forward(self, X):
        x = self._dev(X, (-1, NIN))
        n = x.shape[0]
        y = self.torch.empty(n, NOUT, dtype=self.torch.float32, device=self.device)
        self._check(self.L.pgk_mlp_forward(self.h, x.data_ptr(), y.data_ptr(), n))
        self.stream.synchronize()
        return y

    def loss_grad(self, X, Y):
        x, yy = self._dev(X, (-1, NIN)), self._dev(Y, (-1, NOUT))
        g = self.torch.empty(NPARAM, dtype=self.torch.float32, device=self.device)
        loss = ctypes.c_float()
        self._check(self.L.pgk_mlp_loss_grad(self.h, x.data_ptr(), yy.data_ptr(), x.shape[0], g.data_ptr(),
                                             ctypes.byref(loss)))
        return float(loss.value), g.cpu().numpy()

    def train(self, X, Y, epochs, batch=1024, lr=1e-3, seed=1):
        x, yy = self._dev(X, (-1, NIN)), self._dev(Y, (-1, NOUT))
        losses = (ctypes.c_float * max(epochs, 1))()
        self._check(self.L.pgk_mlp_train(self.h, x.data_ptr(), yy.data_ptr(), x.shape[0], int(batch), int(epochs),
                                         float(lr), int(seed), losses))
        self.stream.synchronize()
        return np.array(list(losses))[:epochs]
