"""FP64 reference of the per-vertex warm-start MLP (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark use
this module; the HIP library never imports or calls it.

The network maps 16 features of a soft vertex to a 3-vector (the correction of the
explicit-velocity displacement h v^t, in units of s = h * 0.05 m/s):

    h1 = relu(W1 x + b1)    W1: 64 x 16
    h2 = relu(W2 h1 + b2)   W2: 64 x 64
    h3 = relu(W3 h2 + b3)   W3: 64 x 64
    y  = W4 h3 + b4         W4:  3 x 64

9,603 parameters, flattened in the order W1, b1, W2, b2, W3, b3, W4, b4 (each W
row-major, [out][in]).  The weight matrices are used rounded to bfloat16 (round to
nearest, ties to even); biases stay FP32.  This reference takes the bf16-rounded
weights and inputs and computes everything else in FP64.

Loss: mean squared error over all 3 B outputs of a batch of B vertices,
L = (1 / 3B) sum_v |y_v - t_v|^2.  Optimiser: Adam (Kingma and Ba, 2015) with bias
correction, beta1 = 0.9, beta2 = 0.999, eps = 1e-8.
"""
from __future__ import annotations

import numpy as np

SIZES = (16, 64, 64, 64, 3)
SHAPES = [("W1", (64, 16)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 64)), ("b3", (64,)),
          ("W4", (3, 64)), ("b4", (3,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def bf16_round(x):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def unflatten(theta):
    """Split a flat parameter vector into the named tensors (views, FP64)."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def effective(theta32):
    """The parameters as the network uses them: W rounded to bf16, b as FP32."""
    p = unflatten(np.asarray(theta32, dtype=np.float32).astype(np.float64))
    for k in ("W1", "W2", "W3", "W4"):
        p[k] = bf16_round(p[k].astype(np.float32)).astype(np.float64)
    return p


def forward(p, x):
    """x: [B, 16] (already in the precision the caller wants).  Returns the output
    [B, 3] and the cache of pre-activations for the backward pass."""
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ p["W3"].T + p["b3"]
    h3 = np.maximum(z3, 0.0)
    y = h3 @ p["W4"].T + p["b4"]
    return y, (x, z1, h1, z2, h2, z3, h3)


def loss(y, t):
    d = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    return float(np.sum(d * d) / d.size)


def backward(p, cache, y, t):
    """Gradient of the MSE loss with respect to every parameter (chain rule through the
    four affine maps and the three ReLUs; the derivative of relu at 0 is taken as 0)."""
    x, z1, h1, z2, h2, z3, h3 = cache
    B = x.shape[0]
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / (3.0 * B)
    g = {}
    g["W4"] = dy.T @ h3
    g["b4"] = dy.sum(0)
    d3 = (dy @ p["W4"]) * (z3 > 0)
    g["W3"] = d3.T @ h2
    g["b3"] = d3.sum(0)
    d2 = (d3 @ p["W3"]) * (z2 > 0)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * (z1 > 0)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(0)
    return g


def loss_and_grad(theta32, x, t):
    """Loss and flat gradient at the bf16-effective parameters on bf16-rounded inputs."""
    p = effective(theta32)
    xb = bf16_round(np.asarray(x, dtype=np.float32)).astype(np.float64)
    y, cache = forward(p, xb)
    return loss(y, t), flatten(backward(p, cache, y, t))


def predict(theta32, x):
    p = effective(theta32)
    xb = bf16_round(np.asarray(x, dtype=np.float32)).astype(np.float64)
    return forward(p, xb)[0]


def adam_step(theta, m, v, grad, step, lr):
    """One Adam update (step counts from 1).  Returns new (theta, m, v)."""
    m = ADAM_B1 * m + (1.0 - ADAM_B1) * grad
    v = ADAM_B2 * v + (1.0 - ADAM_B2) * grad * grad
    mh = m / (1.0 - ADAM_B1 ** step)
    vh = v / (1.0 - ADAM_B2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v
