"""The allocation-free inference entry point (pgk_mlp_forward_static, its
bf16 weights and activations in the library's fixed device array) against
pgk_mlp_forward of a pgk_mlp object holding the same parameters: the same
kernels, so the same bits, on two calls in a row, the second smaller."""
import ctypes

import numpy as np
import pytest

from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu


def _data(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, (n, 6)).astype(np.float32)


def test_static_forward_equals_object_forward():
    import torch

    from paper_2201_05280_amd import _lib
    from paper_2201_05280_amd.mlp import MLP
    L = _lib.load()
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    th = M.init(29)
    ref_net = MLP(nmax=4096)
    ref_net.set_params(th)
    theta = torch.as_tensor(th, dtype=torch.float32, device=dev)
    for n, seed in ((4096, 1), (1000, 2), (37, 3)):   # full capacity, then smaller calls
        X = _data(n, seed)
        x = torch.as_tensor(X, device=dev)
        y = torch.full((n, 4), float("nan"), dtype=torch.float32, device=dev)
        print("pgk_mlp_forward_static n=%d" % n, flush=True)
        rc = L.pgk_mlp_forward_static(theta.data_ptr(), x.data_ptr(), y.data_ptr(), n,
                                      ctypes.c_void_p(stream.cuda_stream))
        assert rc == 0, _lib.ERRORS.get(rc, rc)
        stream.synchronize()
        ref = ref_net.forward(X).cpu().numpy()
        got = y.cpu().numpy()
        assert np.isfinite(got).all()
        assert np.array_equal(got, ref), np.abs(got - ref).max()
    ref_net.close()


def test_static_forward_refuses_beyond_capacity():
    import torch

    from paper_2201_05280_amd import _lib
    L = _lib.load()
    dev = torch.device("cuda", 0)
    theta = torch.zeros(_lib.MLP_NPARAM, dtype=torch.float32, device=dev)
    x = torch.zeros((8, 6), dtype=torch.float32, device=dev)
    y = torch.zeros((8, 4), dtype=torch.float32, device=dev)
    s = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    # rejected on the host before any GPU work (the pointers are never read)
    assert L.pgk_mlp_forward_static(theta.data_ptr(), x.data_ptr(), y.data_ptr(), _lib.MLP_STATIC_NMAX + 1, s) == -7
    assert L.pgk_mlp_forward_static(theta.data_ptr(), x.data_ptr(), y.data_ptr(), -1, s) == -1
    assert L.pgk_mlp_forward_static(None, x.data_ptr(), y.data_ptr(), 8, s) == -1
    assert L.pgk_mlp_forward_static(theta.data_ptr(), x.data_ptr(), y.data_ptr(), 0, s) == 0
