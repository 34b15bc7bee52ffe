"""Reference U-Net for the learned warm start (test infrastructure).

Only the test suite may import this module.  Plain numpy, FP64 accumulation,
written independently of the HIP kernels: convolutions are evaluated by explicit
shifted-slice sums, not by the im2col + GEMM lowering the library uses.

Architecture (the one the library builds): 4 levels with 16/32/64/128 channels,
two 3x3 (padding 1) convolutions + ReLU per level, 2x2 stride-2 convolutions
(+ReLU) down, 2x2 stride-2 transposed convolutions (+ReLU) up, skip concatenation
(up-sampled channels first), a 1x1 output head with 5 channels, MSE loss.

Parameters are one flat vector; per layer W then b with
  3x3 conv: W[(ky*3+kx)*C + c][co]      (C input channels incl. the skip)
  down    : W[(dy*2+dx)*C + c][co]
  up      : W[c][(dy*2+dx)*Co + co]
  head    : W[c][o]
With bf16=True the rounding points of the BF16 path are emulated: the network
input, conv/down weights, every stored activation, the up-sampling product before
its bias, and every per-layer gradient fed to the weight/input products are
rounded to BF16 (round to nearest even); accumulation stays FP64.

The optimiser (adam_step) is plain Adam with the library's constants
(beta 0.9 / 0.999, eps 1e-8), FP64.
"""
from __future__ import annotations

import numpy as np

CH = (16, 32, 64, 128)
CIN, COUT = 8, 5


def to_bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def layers():
    """(kind, cin, cin2, cout, level, input, input2, output) in execution order."""
    L = []
    acts = {"x": (CIN, 0)}

    def add(kind, cin, cin2, cout, lev, i, i2, o):
        L.append((kind, cin, cin2, cout, lev, i, i2, o))

    add("conv", CIN, 0, CH[0], 0, "x", None, "e0a")
    add("conv", CH[0], 0, CH[0], 0, "e0a", None, "e0")
    add("down", CH[0], 0, CH[1], 1, "e0", None, "d0")
    add("conv", CH[1], 0, CH[1], 1, "d0", None, "e1a")
    add("conv", CH[1], 0, CH[1], 1, "e1a", None, "e1")
    add("down", CH[1], 0, CH[2], 2, "e1", None, "d1")
    add("conv", CH[2], 0, CH[2], 2, "d1", None, "e2a")
    add("conv", CH[2], 0, CH[2], 2, "e2a", None, "e2")
    add("down", CH[2], 0, CH[3], 3, "e2", None, "d2")
    add("conv", CH[3], 0, CH[3], 3, "d2", None, "e3a")
    add("conv", CH[3], 0, CH[3], 3, "e3a", None, "e3")
    add("up", CH[3], 0, CH[2], 2, "e3", None, "u2")
    add("conv", CH[2], CH[2], CH[2], 2, "u2", "e2", "c2a")
    add("conv", CH[2], 0, CH[2], 2, "c2a", None, "c2")
    add("up", CH[2], 0, CH[1], 1, "c2", None, "u1")
    add("conv", CH[1], CH[1], CH[1], 1, "u1", "e1", "c1a")
    add("conv", CH[1], 0, CH[1], 1, "c1a", None, "c1")
    add("up", CH[1], 0, CH[0], 0, "c1", None, "u0")
    add("conv", CH[0], CH[0], CH[0], 0, "u0", "e0", "c0a")
    add("conv", CH[0], 0, CH[0], 0, "c0a", None, "c0")
    add("head", CH[0], 0, COUT, 0, "c0", None, "out")
    return L


def param_shapes():
    out = []
    for kind, cin, cin2, cout, *_ in layers():
        if kind == "conv":
            out.append(((9 * (cin + cin2), cout), (cout,)))
        elif kind == "down":
            out.append(((4 * cin, cout), (cout,)))
        elif kind == "up":
            out.append(((cin, 4 * cout), (cout,)))
        else:
            out.append(((cin, cout), (cout,)))
    return out


def param_count():
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in param_shapes())


def unpack(theta):
    res, off = [], 0
    for ws, bs in param_shapes():
        nw = int(np.prod(ws))
        W = theta[off:off + nw].reshape(ws)
        off += nw
        b = theta[off:off + bs[0]]
        off += bs[0]
        res.append((W, b))
    return res


def init_params(seed=0):
    """He-normal weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    parts = []
    for (ws, bs), (kind, *_rest) in zip(param_shapes(), layers()):
        fan_in = ws[0] if kind != "up" else ws[0]
        parts.append(rng.standard_normal(int(np.prod(ws))) * np.sqrt(2.0 / fan_in))
        parts.append(np.zeros(bs))
    return np.concatenate(parts)


# --- convolution primitives by shifted slices (NHWC) ---------------------------------
def conv3(X, W, b):
    """3x3 convolution with zero padding 1: out[p] = sum_{ky,kx} X[p + (ky-1,kx-1)] W_k + b."""
    B, H, Wd, C = X.shape
    Wk = W.reshape(3, 3, C, -1)
    Xp = np.zeros((B, H + 2, Wd + 2, C))
    Xp[:, 1:-1, 1:-1] = X
    out = np.zeros((B, H, Wd, Wk.shape[-1]))
    for ky in range(3):
        for kx in range(3):
            out += Xp[:, ky:ky + H, kx:kx + Wd] @ Wk[ky, kx]
    return out + b


def conv3_back(X, W, g):
    """Gradients of conv3 w.r.t. X and W for output gradient g."""
    B, H, Wd, C = X.shape
    Wk = W.reshape(3, 3, C, -1)
    Xp = np.zeros((B, H + 2, Wd + 2, C))
    Xp[:, 1:-1, 1:-1] = X
    dW = np.zeros_like(Wk)
    dXp = np.zeros_like(Xp)
    for ky in range(3):
        for kx in range(3):
            dW[ky, kx] = np.einsum("bhwc,bhwo->co", Xp[:, ky:ky + H, kx:kx + Wd], g)
            dXp[:, ky:ky + H, kx:kx + Wd] += g @ Wk[ky, kx].T
    return dXp[:, 1:-1, 1:-1], dW.reshape(W.shape)


def down(X, W, b):
    """2x2 stride-2 convolution: out[y,x] = sum_{dy,dx} X[2y+dy, 2x+dx] W_k + b."""
    C = X.shape[-1]
    Wk = W.reshape(2, 2, C, -1)
    out = 0.0
    for dy in range(2):
        for dx in range(2):
            out = out + X[:, dy::2, dx::2] @ Wk[dy, dx]
    return out + b


def down_back(X, W, g):
    C = X.shape[-1]
    Wk = W.reshape(2, 2, C, -1)
    dX = np.zeros_like(X)
    dW = np.zeros_like(Wk)
    for dy in range(2):
        for dx in range(2):
            dW[dy, dx] = np.einsum("bhwc,bhwo->co", X[:, dy::2, dx::2], g)
            dX[:, dy::2, dx::2] = g @ Wk[dy, dx].T
    return dX, dW.reshape(W.shape)


def up_prod(X, W, cout):
    """The four per-position products of the transposed convolution: [B,h,w,2,2,cout]."""
    B, h, w, C = X.shape
    return (X @ W).reshape(B, h, w, 2, 2, cout)


def up_place(Y4, b):
    B, h, w, _, _, co = Y4.shape
    out = np.zeros((B, 2 * h, 2 * w, co))
    for dy in range(2):
        for dx in range(2):
            out[:, dy::2, dx::2] = Y4[:, :, :, dy, dx]
    return out + b


def up_back(X, W, g, cout):
    B, h, w, C = X.shape
    g4 = np.zeros((B, h, w, 2, 2, cout))
    for dy in range(2):
        for dx in range(2):
            g4[:, :, :, dy, dx] = g[:, dy::2, dx::2]
    g4 = g4.reshape(B, h, w, 4 * cout)
    dW = np.einsum("bhwc,bhwk->ck", X, g4)
    dX = g4 @ W.T
    return dX, dW


def forward(theta, x, bf16=False):
    """Returns (out, cache)."""
    rnd = to_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    P = unpack(theta)
    acts = {"x": rnd(x)}
    cache = []
    for (kind, cin, cin2, cout, lev, i, i2, o), (W, b) in zip(layers(), P):
        X = acts[i] if i2 is None else np.concatenate([acts[i], acts[i2]], axis=-1)
        if kind == "head":
            out = X @ W + b
            cache.append((X, None))
            return out, (acts, cache)
        Wr = rnd(W)
        if kind == "conv":
            y = conv3(X, Wr, b)
        elif kind == "down":
            y = down(X, Wr, b)
        else:
            y = up_place(rnd(up_prod(X, Wr, cout)), b)
        y = rnd(np.maximum(y, 0.0))
        acts[o] = y
        cache.append((X, y))
    raise AssertionError("no head")


def loss_and_grad(theta, x, t, bf16=False):
    out, (acts, cache) = forward(theta, x, bf16)
    rnd = to_bf16 if bf16 else (lambda a: a)
    n = out.size
    loss = float(np.mean((out - t) ** 2))
    gout = 2.0 * (out - t) / n
    P = unpack(theta)
    grads = [None] * len(P)
    agrad = {k: np.zeros_like(v) for k, v in acts.items()}
    L = layers()
    for li in range(len(L) - 1, -1, -1):
        kind, cin, cin2, cout, lev, i, i2, o = L[li]
        W, b = P[li]
        X, y = cache[li]
        if kind == "head":
            dW = X.reshape(-1, cin).T @ gout.reshape(-1, cout)
            db = gout.reshape(-1, cout).sum(0)
            dX = gout @ W.T
        else:
            g = rnd(agrad[o] * (y > 0))
            db = g.reshape(-1, cout).sum(0)
            Wr = to_bf16(W) if bf16 else W
            if kind == "conv":
                dX, dW = conv3_back(X, Wr, g)
            elif kind == "down":
                dX, dW = down_back(X, Wr, g)
            else:
                dX, dW = up_back(X, Wr, g, cout)
        grads[li] = (dW, db)
        if i2 is None:
            if i != "x":
                agrad[i] += dX
        else:
            agrad[i] += dX[..., :cin]
            agrad[i2] += dX[..., cin:]
    flat = np.concatenate([np.concatenate([dW.ravel(), db.ravel()]) for dW, db in grads])
    return loss, flat, out


# --- optimiser ------------------------------------------------------------------------
def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, Algorithm 1) in FP64: first and second moment
    running averages, their bias corrections by 1 - beta^step (step counts from 1),
    and the update lr * m_hat / (sqrt(v_hat) + eps).  Returns (theta, m, v)."""
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return np.asarray(theta, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
