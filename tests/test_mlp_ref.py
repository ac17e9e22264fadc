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


def test_adam_first_steps_move_by_lr_times_sign():
    # With eps = 0 and a constant gradient g, the bias-corrected moments are
    # exactly g and g^2 at every step t, so each step moves every weight by
    # lr * sign(g).  Without the 1 - beta^t corrections step 1 would move by
    # lr (1 - b1)/sqrt(1 - b2) = 3.16 lr.
    th0 = np.array([1.0, -2.0, 0.5, 0.0])
    g = np.array([0.3, -1e-3, 7.0, -40.0])
    th, m, v, t = th0, None, None, 0
    for k in range(1, 6):
        th, m, v, t = M.adam(th, [g], lr=0.01, eps=0.0, m=m, v=v, t=t)
        assert t == k
        assert np.allclose(th, th0 - k * 0.01 * np.sign(g), rtol=0, atol=1e-15)


def test_adam_is_invariant_to_gradient_scale():
    # eps = 0: scaling every gradient by c > 0 scales m by c and v by c^2
    rng = np.random.default_rng(4)
    grads = [rng.normal(size=6) for _ in range(4)]
    a = M.adam(np.zeros(6), grads, lr=0.1, eps=0.0)[0]
    b = M.adam(np.zeros(6), [37.0 * g for g in grads], lr=0.1, eps=0.0)[0]
    assert np.allclose(a, b, rtol=0, atol=1e-15)


def test_adam_two_steps_worked_by_hand():
    # w0 = 1, g1 = 0.5, g2 = -0.25, lr = 0.1, beta = (0.9, 0.999), eps = 0:
    # step 1: m = 0.05, v = 0.00025, mhat = 0.05/0.1 = 0.5, vhat = 0.00025/0.001
    #         = 0.25, w1 = 1 - 0.1 * 0.5/0.5 = 0.9
    # step 2: m = 0.9*0.05 - 0.1*0.25 = 0.02, v = 0.999*0.00025 + 0.001*0.0625
    #         = 0.00031225, mhat = 0.02/0.19 = 2/19, vhat = 0.00031225/0.001999
    #         = 312.25/1999, w2 = 0.9 - 0.1 (2/19)/sqrt(312.25/1999)
    w1, m1, v1, _ = M.adam([1.0], [[0.5]], lr=0.1, eps=0.0)
    assert abs(w1[0] - 0.9) < 1e-15 and abs(m1[0] - 0.05) < 1e-16 and abs(v1[0] - 0.00025) < 1e-18
    w2, m2, v2, t = M.adam([1.0], [[0.5], [-0.25]], lr=0.1, eps=0.0)
    assert t == 2 and abs(m2[0] - 0.02) < 1e-16 and abs(v2[0] - 0.00031225) < 1e-18
    assert abs(w2[0] - (0.9 - 0.1 * (2 / 19) / np.sqrt(312.25 / 1999))) < 1e-15
    assert abs(w2[0] - 0.873366) < 1e-6
