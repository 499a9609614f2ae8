"""Pins of the FP64 surrogate-network oracle: back-propagation against central
finite differences of the forward pass, closed-form forward values, the
closed-form first Adam step, and the bfloat16 rounding rule."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_2312_14172_amd import workloads as W


def test_parameter_count():
    assert M.NPARAM == W.MLP_NPARAM == 8641


def test_silu_closed_form():
    assert M.silu(np.array([0.0]))[0] == 0.0
    assert abs(M.silu(np.array([1.0]))[0] - 1 / (1 + math.exp(-1))) < 1e-16
    z = np.linspace(-4, 4, 9)
    h = 1e-6
    np.testing.assert_allclose(M.dsilu(z), (M.silu(z + h) - M.silu(z - h)) / (2 * h), rtol=1e-8)


def test_forward_single_path_closed_form():
    """Only one path through the network is nonzero: y = b4 + w4 s(w3 s(w2 s(w1 x0)))."""
    th = np.zeros(M.NPARAM)
    p = M.unpack(th)
    p["W1"][5, 0] = 0.7
    p["W2"][9, 5] = -1.3
    p["W3"][2, 9] = 0.4
    p["W4"][2] = 2.5
    p["b4"][0] = 0.125
    th = M.pack(p)
    x = np.array([[0.9, -0.3, 0.2]])
    s = lambda z: z / (1 + math.exp(-z))
    ref = 0.125 + 2.5 * s(0.4 * s(-1.3 * s(0.7 * 0.9)))
    assert abs(M.forward(th, x)[0][0] - ref) < 1e-15
    # all weights zero: the output is the last bias
    z = np.zeros(M.NPARAM)
    z[-1] = -0.3
    np.testing.assert_array_equal(M.forward(z, np.ones((4, 3)))[0], -0.3)


@pytest.mark.parametrize("seed", [0, 1])
def test_backprop_matches_central_differences(seed):
    theta = W.mlp_init_params(seed).astype(np.float64)
    X = W.mlp_points(seed + 10, 24)
    t = np.random.default_rng(seed).normal(size=24) * 0.3
    g, L = M.gradient(theta, X, t)
    assert abs(L - M.loss(theta, X, t)) < 1e-15
    rng = np.random.default_rng(seed + 5)
    idx = np.concatenate([rng.choice(M.NPARAM, 60, replace=False), [M.NPARAM - 1, 0, 192, 8576]])
    h = 1e-6
    for i in idx:
        e = np.zeros(M.NPARAM)
        e[i] = h
        fd = (M.loss(theta + e, X, t) - M.loss(theta - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(abs(g[i]), 1e-3), (i, fd, g[i])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = M.adam_step(th, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    # bias-corrected first moments equal g and g^2
    np.testing.assert_allclose(new, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_bf16_rounding_rule():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 1e-3, 3.0e38])
    r = M.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # halfway between 1 and 1 + 2^-7: ties to even
    assert r[2] == 1.0 + 2 ** -7             # above halfway: rounds up
    assert r[3] == -2.5
    assert abs(r[4] - 1e-3) <= 1e-3 * 2 ** -8
    # bfloat16 keeps 8 significant bits: the error is at most half an ulp,
    # 2^(e - 8) for |v| in [2^e, 2^(e+1)), and the result has 7 fraction bits
    for v in np.random.default_rng(0).normal(size=200):
        rv = M.bf16_round(np.array([v]))[0]
        e = math.floor(math.log2(abs(v)))
        assert abs(rv - v) <= 2.0 ** (e - 8)
        assert (rv / 2.0 ** (e - 7)) == round(rv / 2.0 ** (e - 7)) or abs(rv) == 2.0 ** (e + 1)
