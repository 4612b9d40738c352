"""CPU oracle of the learned refinement network (test infrastructure).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this module.  It shares no code with the HIP library.

The network proposes the split / no-split decision of a quadtree box from
samples of the source on the box (the refinement of section 3.1, whose plain
criterion still checks every leaf).  Everything here is written out in
FP64 from the definitions:

* features x[288] of a box from its samples s on a 16 x 16 grid of
  first-kind Chebyshev points and its level l:
  A = max |s|, x[k] = s_k / A (k < 256; 0 when A = 0), x[256] = l / 16,
  x[257] = clip((log10 A + 10) / 10, -1, 2) (-1 when A = 0),
  x[258] = max(log10 A, -320) / 320 (-1 when A = 0), x[259:] = 0;
  every feature rounded to BF16 (round to nearest, ties to even);
* the network 288 -> 128 -> 128 -> 1: z1 = x W1^T + b1, h1 = relu(z1),
  z2 = h1 W2^T + b2, h2 = relu(z2), logit = h2 . w3 + b3; the split is
  proposed when logit > 0;
* the loss: mean binary cross-entropy of sigmoid(logit) against the labels,
  and its gradient by the chain rule;
* Adam (Kingma and Ba, 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
  w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

With emulate=True the forward and backward passes round to BF16 exactly
where the GPU kernels store BF16 (the weights W1 and W2, h1, dL/dz2 and
dL/dz1 as matrix operands); sums stay FP64 here (FP32 on the GPU).  With
emulate=False nothing is rounded (the plain FP64 network).

Parameter vector layout (flat, in this order): W1[128][288], b1[128],
W2[128][128], b2[128], w3[128], b3[1].
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID = 288, 128
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("w3", (N_HID,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + k], np.float64).reshape(shp)
        o += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in SHAPES])


def bf16(a) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64.

    BF16 keeps the sign, the 8 exponent bits and the top 7 mantissa bits of an
    IEEE single; the value is first rounded to single (its own round to
    nearest), then the low 16 bits are rounded away."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    return (u.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def features(samples: np.ndarray, level: np.ndarray) -> np.ndarray:
    """x[B][288] (BF16 values as float64) from samples[B][16][16] and level[B]."""
    s = np.asarray(samples, np.float64).reshape(len(samples), 256)
    lv = np.asarray(level, np.float64)
    A = np.abs(s).max(axis=1)
    x = np.zeros((len(s), N_IN))
    nz = A > 0
    x[nz, :256] = s[nz] / A[nz, None]
    x[:, 256] = lv / 16.0
    with np.errstate(divide="ignore"):
        lg = np.log10(np.where(nz, A, 1.0))
        x[:, 257] = np.where(nz, np.clip((lg + 10.0) / 10.0, -1.0, 2.0), -1.0)
        x[:, 258] = np.where(nz, np.maximum(lg, -320.0) / 320.0, -1.0)
    return bf16(x)


def forward(theta: np.ndarray, x: np.ndarray, emulate: bool = True, keep: bool = False):
    """Logits of the boxes x[B][288]; with keep=True also the activations."""
    p = unpack(theta)
    W1 = bf16(p["W1"]) if emulate else p["W1"]
    W2 = bf16(p["W2"]) if emulate else p["W2"]
    z1 = x @ W1.T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    if emulate:
        h1 = bf16(h1)
    z2 = h1 @ W2.T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    logit = h2 @ p["w3"] + p["b3"][0]
    if keep:
        return logit, dict(W1=W1, W2=W2, h1=h1, z2=z2, h2=h2)
    return logit


def bce(logit: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Per-box binary cross-entropy of sigmoid(logit) against y, in a form
    that does not overflow: max(z, 0) - z y + log(1 + exp(-|z|))."""
    z = np.asarray(logit, np.float64)
    return np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))


def loss_and_grad(theta: np.ndarray, x: np.ndarray, y: np.ndarray, emulate: bool = True):
    """Mean BCE over the boxes and its gradient with respect to theta."""
    p = unpack(theta)
    y = np.asarray(y, np.float64)
    N = len(y)
    logit, a = forward(theta, x, emulate, keep=True)
    loss = bce(logit, y).mean()
    sig = 1.0 / (1.0 + np.exp(-logit))
    dz3 = (sig - y) / N                              # dL/dlogit
    g = {"b3": np.array([dz3.sum()]), "w3": a["h2"].T @ dz3}
    dz2 = np.outer(dz3, p["w3"]) * (a["z2"] > 0)     # dL/dz2
    g["b2"] = dz2.sum(axis=0)
    dz2m = bf16(dz2) if emulate else dz2
    g["W2"] = dz2m.T @ a["h1"]
    dz1 = (dz2m @ a["W2"]) * (a["h1"] > 0)           # dL/dz1 (h1 > 0 exactly where z1 > 0)
    g["b1"] = dz1.sum(axis=0)
    dz1m = bf16(dz1) if emulate else dz1
    g["W1"] = dz1m.T @ x
    return loss, pack(g)


def adam_step(theta, grad, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step number t >= 1); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v

