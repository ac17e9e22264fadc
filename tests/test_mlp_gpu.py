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


def _bf16_bits(a):
    """bfloat16 bit patterns (round to nearest even) of float32 values."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return (((b + 0x7FFF + ((b >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


def test_adam_steps_match_reference():
    """Three Adam updates (k_adam) on three different minibatch gradients
    against the FP64 reference Adam fed the same gradients: FP32 master
    weights and both moments to 1e-6, the bf16 copies bit for bit."""
    from paper_2201_05280_amd.mlp import MLP
    th = M.init(13)
    m = MLP(nmax=512)
    m.set_params(th)
    ref_th, ref_m, ref_v, t = th.astype(np.float64), None, None, 0
    for k, (lr, b1, b2, eps) in enumerate([(1e-3, 0.9, 0.999, 1e-8), (2e-3, 0.9, 0.999, 1e-8),
                                           (5e-4, 0.8, 0.99, 1e-6)]):
        X, Y = _data(300, 20 + k)
        _, g = m.loss_grad(X, Y)
        m.adam_step(lr, b1, b2, eps)
        # the library takes the hyperparameters as float32: the reference uses
        # those values (float32(0.999) differs from 0.999 by 1.3e-5 of 1 - 0.999)
        f32 = [float(np.float32(a)) for a in (lr, b1, b2, eps)]
        ref_th, ref_m, ref_v, t = M.adam(ref_th, [g], *f32, ref_m, ref_v, t)
        master, wbf, am, av, tt = m.state()
        assert tt == t == k + 1
        for name, dev, ref in (("master", master, ref_th), ("m", am, ref_m), ("v", av, ref_v)):
            err = np.abs(dev - ref).max() / np.abs(ref).max()
            print("step", k + 1, name, "max rel err", err)
            assert err < 1e-6, (k, name, err)
        # the bf16 copies are the device master rounded to nearest even, bit
        # for bit; the reference master rounded the same way gives the same
        # bits except where the FP32 difference straddles a bf16 rounding
        # boundary (a few in 10^5; up to two bf16 ulps on weights that are
        # nearly zero, where an FP32 ulp is a larger part of the value)
        assert np.array_equal(wbf, _bf16_bits(master))
        rb = _bf16_bits(ref_th.astype(np.float32))
        diff = wbf != rb
        print("bf16 copies differing from the rounded reference:", int(diff.sum()))
        assert diff.sum() <= 1e-3 * diff.size
        assert (np.abs(wbf[diff].astype(np.int64) - rb[diff].astype(np.int64)) <= 2).all()
    m.close()


def test_first_training_minibatch_matches_reference():
    """pgk_mlp_train over one minibatch for one epoch is one gradient and one
    Adam step (beta 0.9/0.999, eps 1e-8): the result equals the reference Adam
    applied to the gradient of that minibatch, and the epoch loss is the
    minibatch's mean loss."""
    from paper_2201_05280_amd.mlp import MLP
    th = M.init(17)
    X, Y = _data(256, 31)
    m = MLP(nmax=512)
    m.set_params(th)
    loss0, g = m.loss_grad(X, Y)
    m.set_params(th)
    losses = m.train(X, Y, epochs=1, batch=256, lr=1e-3, seed=5)
    master, wbf, am, av, t = m.state()
    f32 = [float(np.float32(a)) for a in (1e-3, 0.9, 0.999, 1e-8)]   # the library's float32 hyperparameters
    ref_th, ref_m, ref_v, rt = M.adam(th.astype(np.float64), [g], *f32)
    assert t == rt == 1
    for name, dev, ref in (("master", master, ref_th), ("m", am, ref_m), ("v", av, ref_v)):
        err = np.abs(dev - ref).max() / np.abs(ref).max()
        print(name, "max rel err", err)
        assert err < 1e-6, (name, err)
    assert abs(losses[0] - loss0) <= 1e-6 * loss0
    m.close()


def test_epoch_loss_counts_every_point_once():
    """A partial last minibatch: the epoch loss is the mean squared error over
    all n points, not the mean of the minibatch means.  With lr = 0 the
    weights do not move, so it equals the loss of the whole set."""
    from paper_2201_05280_amd.mlp import MLP
    X, Y = _data(300, 41)
    m = MLP(nmax=512)
    m.set_params(M.init(3))
    losses = m.train(X, Y, epochs=2, batch=256, lr=0.0, seed=2)   # minibatches of 256 and 44
    full, _ = m.loss_grad(X, Y)
    print("epoch losses", losses, "full", full)
    assert np.allclose(losses, full, rtol=2e-6, atol=0)
    m.close()


def test_state_save_load_resumes_training_bit_for_bit(tmp_path):
    from paper_2201_05280_amd.mlp import MLP
    X, Y = _data(1024, 5)
    a = MLP(nmax=512)
    a.set_params(M.init(21))
    a.train(X, Y, epochs=2, batch=256, lr=1e-3, seed=3)
    path = tmp_path / "mlp.bin"
    a.save(path)
    s0 = a.state()
    b = MLP(nmax=512)
    b.load(path)
    s1 = b.state()
    for x0, x1 in zip(s0[:4], s1[:4]):
        assert np.array_equal(x0, x1)
    assert s0[4] == s1[4] == 8
    # one more minibatch step, and one more trained epoch, from the same state
    # on both give the same bits (the gradient sums run in a fixed order)
    for net in (a, b):
        net.loss_grad(X[:256], Y[:256])
        net.adam_step(1e-3)
    assert np.array_equal(a.state()[0], b.state()[0])
    la = a.train(X, Y, epochs=1, batch=256, lr=1e-3, seed=4)
    lb = b.train(X, Y, epochs=1, batch=256, lr=1e-3, seed=4)
    sa, sb = a.state(), b.state()
    assert np.array_equal(la, lb)
    for x0, x1 in zip(sa[:4], sb[:4]):
        assert np.array_equal(x0, x1)
    assert sa[4] == sb[4] == 13
    with pytest.raises(RuntimeError):
        bad = tmp_path / "bad.bin"
        bad.write_bytes(b"not a network")
        b.load(bad)
    a.close()
    b.close()


def _epoch_orders(nb, epochs, seed):
    """The library's minibatch order: Fisher-Yates with xorshift64* per epoch."""
    s = seed or 0x9E3779B97F4A7C15
    mask = (1 << 64) - 1
    out = []
    for _ in range(epochs):
        o = list(range(nb))
        for i in range(nb - 1, 0, -1):
            s ^= s >> 12
            s ^= (s << 25) & mask
            s ^= s >> 27
            j = ((s * 2685821657736338717) & mask) % (i + 1)
            o[i], o[j] = o[j], o[i]
        out.append(o)
    return out


def test_graph_replayed_epochs_equal_direct_minibatch_steps():
    """pgk_mlp_train replays one recorded epoch (each minibatch node reading the
    record the host wrote for it) with the loss read back between replays; three
    epochs of two minibatches (one partial) equal the same minibatches taken in
    the same order by loss_grad + adam_step: weights, moments and step count,
    and the epoch losses."""
    from paper_2201_05280_amd.mlp import MLP
    th = M.init(23)
    n, batch, epochs, seed = 400, 256, 3, 9
    X, Y = _data(n, 51)
    a = MLP(nmax=512)
    a.set_params(th)
    losses = a.train(X, Y, epochs=epochs, batch=batch, lr=1e-3, seed=seed)
    sa = a.state()
    b = MLP(nmax=512)
    b.set_params(th)
    nb = (n + batch - 1) // batch
    ref_losses = []
    for order in _epoch_orders(nb, epochs, seed):
        el = 0.0
        for idx in order:
            b0 = idx * batch
            c = min(batch, n - b0)
            lb, _ = b.loss_grad(X[b0:b0 + c], Y[b0:b0 + c])
            b.adam_step(1e-3)
            el += lb * c / n
        ref_losses.append(el)
    sb = b.state()
    assert sa[4] == sb[4] == nb * epochs
    for name, x, y in (("master", sa[0], sb[0]), ("m", sa[2], sb[2]), ("v", sa[3], sb[3])):
        err = np.abs(x - y).max() / np.abs(y).max()
        print(name, "max rel diff", err)
        assert err < 1e-6, (name, err)
    print("epoch losses", losses, ref_losses)
    assert np.allclose(losses, ref_losses, rtol=1e-6, atol=0)
    a.close()
    b.close()
