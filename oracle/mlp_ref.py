"""FP64 reference of the warm-start network -- TEST INFRASTRUCTURE ONLY.

A 16-64-64-16 ReLU multilayer perceptron with mean-squared-error loss,
written from the textbook definition of forward and backward propagation
(chain rule).  Parameters are one flat vector in the order W1[16][64],
b1[64], W2[64][64], b2[64], W3[64][16], b3[16] (row-major [in][out]).

With ``bf16=True`` the reference rounds to bfloat16 (round to nearest even)
at the same points as the GPU kernels: inputs, weights, hidden activations,
and the output/hidden gradients that enter matrix products; sums are FP64.
"""
import numpy as np

SIZES = (16, 64, 64, 16)
OFF = {"W1": 0, "b1": 1024, "W2": 1088, "b2": 5184, "W3": 5248, "b3": 6272}
NPARAM = 6288


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    W1 = p[OFF["W1"]:OFF["b1"]].reshape(16, 64)
    b1 = p[OFF["b1"]:OFF["W2"]]
    W2 = p[OFF["W2"]:OFF["b2"]].reshape(64, 64)
    b2 = p[OFF["b2"]:OFF["W3"]]
    W3 = p[OFF["W3"]:OFF["b3"]].reshape(64, 16)
    b3 = p[OFF["b3"]:NPARAM]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def normalise_inputs(x, norm):
    """(x - mean) * inv_sd with FP32 rounding, as the kernels do before BF16."""
    if norm is None:
        return np.asarray(x, dtype=np.float64)
    n32 = np.asarray(norm, dtype=np.float32)
    return ((np.asarray(x, dtype=np.float32) - n32[:16]) * n32[16:32]).astype(np.float64)


def normalise_targets(t, norm):
    if norm is None:
        return np.asarray(t, dtype=np.float64)
    n32 = np.asarray(norm, dtype=np.float32)
    return ((np.asarray(t, dtype=np.float32) - n32[32:48]) / n32[48:64]).astype(np.float64)


def forward(p, x, bf=False, norm=None):
    """Network output in standardised units (the kernels' y before
    de-standardisation)."""
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(p)
    xb = r(normalise_inputs(x, norm))
    W1, W2, W3 = r(W1), r(W2), r(W3)
    h1 = r(np.maximum(xb @ W1 + b1, 0.0))
    h2 = r(np.maximum(h1 @ W2 + b2, 0.0))
    y = h2 @ W3 + b3
    return y, (xb, h1, h2, W1, W2, W3)


def loss_and_grad(p, x, t, bf=False, norm=None):
    """Mean over samples and outputs of (y - t)^2 (standardised units) and its
    gradient."""
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    y, (xb, h1, h2, W1, W2, W3) = forward(p, x, bf, norm)
    t = normalise_targets(t, norm)
    n = x.shape[0]
    e = y - t
    loss = float((e * e).mean())
    dy = 2.0 * e / (n * 16)
    db3 = dy.sum(0)
    dyb = r(dy)
    dW3 = h2.T @ dyb
    dh2 = (dyb @ W3.T) * (h2 > 0)
    db2 = dh2.sum(0)
    dh2b = r(dh2)
    dW2 = h1.T @ dh2b
    dh1 = (dh2b @ W2.T) * (h1 > 0)
    db1 = dh1.sum(0)
    dh1b = r(dh1)
    dW1 = xb.T @ dh1b
    return loss, pack(dW1, db1, dW2, db2, dW3, db3)
