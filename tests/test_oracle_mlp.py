"""Pins of the FP64 warm-start network reference.

* bf16 rounding equals torch's float32 -> bfloat16 conversion (round to nearest even),
  ties included;
* the backward pass equals central finite differences of the FP64 loss;
* with every ReLU active the network is the affine map W4 W3 W2 W1 x + c, so its
  output equals that matrix chain (a library product);
* with every first-layer ReLU off the output is independent of the input;
* the loss of a constant unit error is 1 (mean over all 3B outputs);
* Adam under a constant gradient g moves each parameter by -lr g / (|g| + eps) at
  every step (the bias corrections make m-hat = g, v-hat = g^2 exactly).
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import mlp


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-8, 8, size=4000),
                        np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.0 - 2.0 ** -7,
                                  1.0 + 2.0 ** -8 + 2.0 ** -20, 0.0, -0.0])]).astype(np.float32)
    ours = mlp.bf16_round(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours.view(np.uint32), ref.view(np.uint32))
    assert ours[-7 + 1] == 1.0                   # tie 1 + 2^-8 rounds to even (1.0)
    assert ours[-7 + 2] == 1.0 + 2.0 ** -6       # tie 1 + 3 * 2^-8 rounds up to even


def _params(seed):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in mlp.SHAPES:
        p[name] = rng.normal(scale=0.4, size=shape)
    return p


def test_backward_matches_finite_differences():
    p = _params(1)
    rng = np.random.default_rng(2)
    x = rng.normal(size=(7, 16))
    t = rng.normal(size=(7, 3))
    y, cache = mlp.forward(p, x)
    g = mlp.backward(p, cache, y, t)
    h = 1e-6
    for name, shape in mlp.SHAPES:
        idx = [tuple(rng.integers(0, s) for s in shape) for _ in range(6)]
        for ix in idx:
            q = {k: v.copy() for k, v in p.items()}
            q[name][ix] += h
            lp = mlp.loss(mlp.forward(q, x)[0], t)
            q[name][ix] -= 2 * h
            lm = mlp.loss(mlp.forward(q, x)[0], t)
            fd = (lp - lm) / (2 * h)
            assert g[name][ix] == pytest.approx(fd, rel=1e-6, abs=1e-9), f"{name}{ix}"


def test_all_active_is_matrix_chain():
    p = _params(3)
    for k in ("b1", "b2", "b3"):
        p[k] = p[k] * 0 + 1e3                    # every pre-activation positive for |x| <= 1
    p["W2"] = np.abs(p["W2"])
    p["W3"] = np.abs(p["W3"])
    x = np.random.default_rng(4).uniform(-1, 1, size=(5, 16))
    y, cache = mlp.forward(p, x)
    assert all((z > 0).all() for z in (cache[1], cache[3], cache[5]))
    A = np.linalg.multi_dot([p["W4"], p["W3"], p["W2"], p["W1"]])
    c = p["W4"] @ (p["W3"] @ (p["W2"] @ p["b1"] + p["b2"]) + p["b3"]) + p["b4"]
    assert np.allclose(y, x @ A.T + c, rtol=1e-12, atol=1e-9)


def test_dead_first_layer_is_constant():
    p = _params(5)
    p["b1"] = p["b1"] * 0 - 1e3
    x = np.random.default_rng(6).uniform(-1, 1, size=(4, 16))
    y, _ = mlp.forward(p, x)
    assert np.array_equal(y, np.broadcast_to(y[0], y.shape))
    # and the gradient reaching W1 vanishes
    g = mlp.backward(p, mlp.forward(p, x)[1], y, np.zeros((4, 3)))
    assert not g["W1"].any() and not g["b1"].any()


def test_loss_normalisation():
    t = np.random.default_rng(7).normal(size=(9, 3))
    assert mlp.loss(t + 1.0, t) == pytest.approx(1.0, rel=1e-15)


def test_adam_constant_gradient():
    rng = np.random.default_rng(8)
    g = rng.normal(size=50) * 10.0 ** rng.integers(-3, 3, size=50)
    th = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr = 1e-3
    th0 = th.copy()
    for step in range(1, 6):
        th, m, v = mlp.adam_step(th, m, v, g, step, lr)
        expect = th0 - step * lr * g / (np.abs(g) + mlp.ADAM_EPS)
        assert np.allclose(th, expect, rtol=0, atol=1e-14 * step + 1e-12)


def test_effective_rounds_weights_only():
    th = sg.mlp_init(0)
    th[1024:1088] = np.float32(0.1234567)        # b1 kept as FP32
    p = mlp.effective(th)
    assert mlp.N_PARAMS == 9603
    assert np.array_equal(p["W1"], mlp.bf16_round(th[:1024].reshape(64, 16)))
    assert np.array_equal(p["b1"], th[1024:1088].astype(np.float64))
