"""Pins of the FP64 MLP reference (CPU): central finite differences of its own
loss, and the bfloat16 rounding rule on values whose rounding is known."""
import numpy as np

from oracle import mlp_ref as M


def test_parameter_count():
    assert M.NPARAM == 50948


def test_bf16_rounding_rule():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1)
    # 1 + 3*2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties go to 1 + 2^-6
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.5, 3.0e-3])
    r = M.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1 + 2 ** -6
    assert r[3] == 1 + 2 ** -7 and r[4] == -2.5
    assert abs(r[5] - 3.0e-3) / 3.0e-3 < 2 ** -8


def test_gradient_matches_finite_differences():
    th = M.init(3).astype(np.float64)
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, (40, 6))
    Y = rng.uniform(-1, 1, (40, 4))
    _, g = M.loss_and_grad(th, X, Y)
    idx = rng.choice(M.NPARAM, 40, replace=False)
    # include every parameter block
    starts = np.cumsum([0] + [int(np.prod(s)) for s in M.SHAPES])[:-1]
    idx = np.concatenate([idx, starts])
    for i in idx:
        e = 1e-6
        tp, tm = th.copy(), th.copy()
        tp[i] += e
        tm[i] -= e
        fd = (M.loss_and_grad(tp, X, Y)[0] - M.loss_and_grad(tm, X, Y)[0]) / (2 * e)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), (i, fd, g[i])
