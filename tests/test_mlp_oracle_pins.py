"""Pins of the FP64 surrogate-network reference (oracle/mlp_ref.py) against
facts that do not come from the reference itself: library routines, closed
forms of Adam, finite differences and symmetries of the network."""
import math

import numpy as np
import pytest
import torch
from scipy.stats import norm

from oracle import mlp_ref as M


def test_bf16_rounding_matches_library_round_to_nearest_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-8, 8, 4000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0, -0.0, 65504.0]])
    lib = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x), lib)
    # ties go to the even mantissa
    assert M.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert M.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_gelu_against_normal_cdf_and_symmetry():
    z = np.linspace(-8, 8, 1601)
    assert np.allclose(M.gelu(z), z * norm.cdf(z), rtol=0, atol=1e-14)
    assert np.allclose(M.gelu(z) - M.gelu(-z), z, rtol=0, atol=1e-14)   # erf is odd
    assert M.gelu(np.array([0.0]))[0] == 0.0


def test_gelu_grad_against_finite_differences():
    z = np.linspace(-6, 6, 241)
    h = 1e-5
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - M.gelu_grad(z))) < 1e-9


def test_parameter_count_and_flat_roundtrip():
    widths = [5, 512, 512, 512, 512, 256]
    ps = M.init_params(widths, 1)
    v = M.flat(ps)
    assert v.size == 922368
    back = M.unflat(v, widths)
    for (W, b), (W2, b2) in zip(ps, back):
        assert np.array_equal(W, W2) and np.array_equal(b, b2)
    for (W, b), k in zip(ps, widths[:-1]):   # uniform(-1/sqrt(k), 1/sqrt(k))
        assert np.abs(W).max() <= 1 / math.sqrt(k) and np.abs(W).max() > 0.9 / math.sqrt(k)


def test_single_layer_is_the_affine_map_recovered_by_least_squares():
    rng = np.random.default_rng(1)
    ps = M.init_params([6, 4], 2)
    X = rng.standard_normal((40, 6))
    Y, _ = M.forward(ps, X)
    A = np.hstack([X, np.ones((40, 1))])
    coef, *_ = np.linalg.lstsq(A, Y, rcond=None)
    assert np.allclose(coef[:6].T, ps[0][0], atol=1e-12)
    assert np.allclose(coef[6], ps[0][1], atol=1e-12)


def test_hidden_unit_permutation_leaves_output_unchanged():
    rng = np.random.default_rng(2)
    widths = [5, 8, 8, 3]
    ps = M.init_params(widths, 3)
    X = rng.standard_normal((7, 5))
    y0, _ = M.forward(ps, X)
    p1 = rng.permutation(8)
    p2 = rng.permutation(8)
    (W0, b0), (W1, b1), (W2, b2) = ps
    q = [(W0[p1], b0[p1]), (W1[p2][:, p1], b1[p2]), (W2[:, p2], b2)]
    y1, _ = M.forward(q, X)
    assert np.allclose(y0, y1, rtol=0, atol=1e-14)
    # a transposed operand would not survive the same test
    bad = [(W0[p1], b0[p1]), (W1[p2][:, p1].T, b1[p2]), (W2[:, p2], b2)]
    assert not np.allclose(M.forward(bad, X)[0], y0, atol=1e-3)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(4)
    widths = [3, 8, 6, 4]
    ps = M.init_params(widths, 5)
    X = rng.standard_normal((5, 3))
    T = rng.standard_normal((5, 4))

    def loss(vec):
        return M.mse(M.forward(M.unflat(vec, widths), X)[0], T)[0]

    y, cache = M.forward(ps, X)
    _, dY = M.mse(y, T)
    g = M.flat(M.backward(ps, cache, dY))
    v = M.flat(ps)
    h = 1e-6
    for i in range(v.size):
        e = np.zeros_like(v)
        e[i] = h
        fd = (loss(v + e) - loss(v - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), i


def test_bfloat16_emulated_gradient_stays_close_to_the_exact_one():
    rng = np.random.default_rng(6)
    widths = [5, 64, 64, 32]
    ps = M.init_params(widths, 7)
    X = rng.uniform(-1, 1, (64, 5))
    T = rng.standard_normal((64, 32))
    y, c = M.forward(ps, X)
    ex = M.flat(M.backward(ps, c, M.mse(y, T)[1]))
    yb, cb = M.forward(ps, X, bf=True)
    bf = M.flat(M.backward(ps, cb, M.mse(yb, T)[1], bf=True))
    assert np.linalg.norm(yb - y) / np.linalg.norm(y) < 1e-2
    assert np.linalg.norm(bf - ex) / np.linalg.norm(ex) < 2e-2


def test_adam_first_step_and_constant_gradient_closed_forms():
    rng = np.random.default_rng(8)
    ps = [(rng.standard_normal((3, 2)), rng.standard_normal(3))]
    g = [(rng.standard_normal((3, 2)), rng.standard_normal(3))]
    opt = M.Adam(ps, lr=1e-3)
    cur = ps
    for t in range(1, 6):
        new = opt.step(cur, g)
        for (P0, b0), (P1, b1), (G, gb) in zip(cur, new, g):
            # bias-corrected moments of a constant gradient are g and g^2
            assert np.allclose(P0 - P1, 1e-3 * G / (np.abs(G) + 1e-8), rtol=1e-12, atol=1e-18)
            assert np.allclose(b0 - b1, 1e-3 * gb / (np.abs(gb) + 1e-8), rtol=1e-12, atol=1e-18)
        cur = new


def test_adam_minimises_a_quadratic():
    c = np.array([[0.3, -1.2], [2.0, 0.5]])
    ps = [(np.zeros((2, 2)), np.zeros(2))]
    opt = M.Adam(ps, lr=0.05)
    for _ in range(2000):
        W, b = ps[0]
        ps = opt.step(ps, [(W - c, b - 1.0)])
    assert np.allclose(ps[0][0], c, atol=1e-3) and np.allclose(ps[0][1], 1.0, atol=1e-3)
