"""The MLP kernels (BF16 MFMA products, FP32 accumulation) against the FP64
reference that rounds the same values to bfloat16."""
import numpy as np
import pytest

from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (n, 6)).astype(np.float32)
    Y = np.stack([np.sin(2 * X[:, 0]) * X[:, 1], X[:, 2] ** 2 - 0.3, np.cos(X[:, 3] + X[:, 4]),
                  0.5 * X[:, 5] * X[:, 0]], 1).astype(np.float32)
    return X, Y


@pytest.mark.parametrize("n", [1, 63, 200, 1024])
def test_forward_matches_reference(n):
    from paper_2201_05280_amd.mlp import MLP
    th = M.init(7)
    X, _ = _data(n, 1)
    m = MLP(nmax=512)
    m.set_params(th)
    y = m.forward(X).cpu().numpy()
    ref, _, _ = M.forward(th.astype(np.float64), X.astype(np.float64), bf16=True)
    err = np.abs(y - ref).max() / np.abs(ref).max()
    print("forward rel err", n, err)
    assert err < 2e-3, err
    m.close()


@pytest.mark.parametrize("n", [64, 300])
def test_gradient_matches_reference(n):
    from paper_2201_05280_amd.mlp import MLP
    th = M.init(11)
    X, Y = _data(n, 2)
    m = MLP(nmax=512)
    m.set_params(th)
    loss, g = m.loss_grad(X, Y)
    rl, rg = M.loss_and_grad(th.astype(np.float64), X.astype(np.float64), Y.astype(np.float64), bf16=True)
    print("loss", loss, rl)
    assert abs(loss - rl) <= 2e-3 * rl
    # per parameter block, normwise relative error
    o = 0
    for s in M.SHAPES:
        k = int(np.prod(s))
        err = np.linalg.norm(g[o:o + k] - rg[o:o + k]) / max(np.linalg.norm(rg[o:o + k]), 1e-12)
        print("block", s, "grad rel err", err)
        assert err < 1e-2, (s, err)
        o += k
    m.close()


def test_training_reduces_the_loss():
    from paper_2201_05280_amd.mlp import MLP
    X, Y = _data(8192, 3)
    m = MLP(nmax=1024)
    m.set_params(M.init(5))
    losses = m.train(X, Y, epochs=30, batch=512, lr=2e-3, seed=9)
    print("losses", losses[:3], losses[-3:])
    assert losses[-1] < 0.1 * losses[0]
    # the trained parameters reproduce their loss through the reference
    th = m.params()
    rl, _ = M.loss_and_grad(th.astype(np.float64), X[:512].astype(np.float64), Y[:512].astype(np.float64), bf16=True)
    assert rl < 0.2 * losses[0]
    m.close()
