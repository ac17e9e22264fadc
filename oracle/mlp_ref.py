"""FP64 CPU reference of the coordinate MLP (TEST INFRASTRUCTURE ONLY).

Network: 6 inputs -> 4 hidden layers of 128 with SiLU -> 4 linear outputs.
Flat parameter order: W1[128,6], b1[128], W2[128,128], b2, W3[128,128], b3,
W4[128,128], b4, W5[4,128], b5[4]  (50,948 values).
Loss: mean squared error over points and outputs, L = sum (yhat - y)^2 / (4 N).

`bf16=True` rounds, to bfloat16 (round to nearest even), exactly the values the
device rounds: every weight, the activations entering layers 2-5, and the
back-propagated dL/dz of layers 2-4 where they enter a product with a weight or
an activation.  All arithmetic is then done in double precision, so the
comparison with the GPU isolates its float32 accumulation.
"""
import numpy as np

SHAPES = [(128, 6), (128,), (128, 128), (128,), (128, 128), (128,), (128, 128), (128,), (4, 128), (4,)]
NPARAM = sum(int(np.prod(s)) for s in SHAPES)


def bf16_round(a):
    """float -> nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    b = a32.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(theta[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init(seed):
    """Seeded initial weights: the shared input generator (He uniform, zero biases)."""
    from paper_2201_05280_amd.inputs import mlp_init
    return mlp_init(seed)


def forward(theta, X, bf16=False):
    W = unpack(theta)
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    a = np.asarray(X, dtype=np.float64)
    zs, acts = [], [a]
    for li in range(4):
        Wl, bl = r(W[2 * li]), W[2 * li + 1]
        inp = a if li == 0 else r(a)
        z = inp @ Wl.T + bl
        zs.append(z)
        a = silu(z)
        acts.append(a)
    y = r(a) @ r(W[8]).T + W[9]
    return y, zs, acts


def loss_and_grad(theta, X, Y, bf16=False):
    W = unpack(theta)
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    yhat, zs, acts = forward(theta, X, bf16)
    N = X.shape[0]
    diff = yhat - Y
    loss = float((diff ** 2).sum() / (4 * N))
    g = [None] * 10
    dy = 2.0 * diff / (4 * N)
    g[8] = dy.T @ r(acts[4])
    g[9] = dy.sum(0)
    da = dy @ r(W[8])
    for li in (3, 2, 1, 0):
        dz = da * dsilu(zs[li])
        if li == 0:
            g[0] = dz.T @ acts[0]
        else:
            g[2 * li] = r(dz).T @ r(acts[li])
            da = r(dz) @ r(W[2 * li])
        g[2 * li + 1] = dz.sum(0)
    return loss, pack(g)


def adam(theta, grads, lr, beta1=0.9, beta2=0.999, eps=1e-8, m=None, v=None, t=0):
    """Adam (Kingma & Ba, "Adam: a method for stochastic optimization", ICLR
    2015, Algorithm 1) in double precision, one update per gradient of
    `grads` in order: first and second moment estimates m, v, their bias
    corrections by 1 - beta^t, and the step lr * mhat / (sqrt(vhat) + eps).
    Returns (theta, m, v, t) after the last update."""
    th = np.asarray(theta, dtype=np.float64).copy()
    m = np.zeros_like(th) if m is None else np.asarray(m, dtype=np.float64).copy()
    v = np.zeros_like(th) if v is None else np.asarray(v, dtype=np.float64).copy()
    for g in grads:
        g = np.asarray(g, dtype=np.float64)
        t += 1
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        mhat = m / (1.0 - beta1 ** t)
        vhat = v / (1.0 - beta2 ** t)
        th = th - lr * mhat / (np.sqrt(vhat) + eps)
    return th, m, v, t
