"""Pins of the learned-warm-start oracle: central differences of the loss
gradient, one Adam step written out by hand, and the feature histogram
against brute force and its invariants."""
import math

import numpy as np
import pytest

import cases
from oracle import mlp_oracle as M

SIZES = [6, 5, 4, 3]


def test_gradient_central_differences():
    rng = np.random.default_rng(0)
    p = cases.mlp_init(SIZES, seed=1) + 0.05 * rng.normal(size=sum(o * i + o for o, i in M.layer_shapes(SIZES)))
    X = rng.normal(size=(7, SIZES[0]))
    Y = rng.normal(size=(7, SIZES[-1]))
    L, g = M.loss_and_grad(p, SIZES, X, Y)
    for k in range(p.size):
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (M.loss_and_grad(pp, SIZES, X, Y)[0] - M.loss_and_grad(pm, SIZES, X, Y)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_forward_closed_form_two_layers():
    # one hidden unit: y = w2 * relu(w1 x + b1) + b2
    sizes = [1, 1, 1]
    p = np.array([2.0, -1.0, 3.0, 0.5])     # W1, b1, W2, b2
    y, _ = M.forward(p, sizes, np.array([[1.5], [0.2]]))
    np.testing.assert_allclose(y[:, 0], [3.0 * max(2 * 1.5 - 1, 0) + 0.5, 3.0 * max(0.4 - 1, 0) + 0.5])


def test_adam_one_step_by_hand():
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -4.0])
    m = np.zeros(2)
    v = np.zeros(2)
    new, m1, v1 = M.adam_step(p, g, m, v, 1, lr=0.1)
    # first step: m_hat = g, v_hat = g^2, update = lr * g / (|g| + eps) = lr * sign(g)
    np.testing.assert_allclose(new, p - 0.1 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g)
    np.testing.assert_allclose(v1, 0.001 * g * g)


def test_adam_constant_gradient_closed_form():
    # With a constant gradient g the bias-corrected moments are exactly g and
    # g^2 at every step (m_n = (1 - b1^n) g, v_n = (1 - b2^n) g^2), so each of
    # n steps moves the parameter by lr g / (|g| + eps): a pin of both bias
    # corrections at every step count, not only the first.
    g = np.array([0.5, -4.0, 1e-3, 7.0])
    p0 = np.array([1.0, -2.0, 0.3, 0.0])
    lr = 0.01
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    for n in range(1, 41):
        p, m, v = M.adam_step(p, g, m, v, n, lr=lr)
        np.testing.assert_allclose(m, (1 - 0.9 ** n) * g, rtol=1e-12)
        np.testing.assert_allclose(v, (1 - 0.999 ** n) * g * g, rtol=1e-12)
        np.testing.assert_allclose(p, p0 - n * lr * g / (np.abs(g) + 1e-8), rtol=1e-10, atol=1e-14)


def test_adam_two_gradients_by_hand():
    # step 1 with g1, step 2 with g2, written out from the definitions:
    # m2 = b1 (1 - b1) g1 + (1 - b1) g2, v2 = b2 (1 - b2) g1^2 + (1 - b2) g2^2,
    # update = lr (m2 / (1 - b1^2)) / (sqrt(v2 / (1 - b2^2)) + eps)
    g1, g2 = np.array([2.0, -1.0]), np.array([-1.0, 3.0])
    p = np.array([0.0, 0.0])
    p1, m, v = M.adam_step(p, g1, np.zeros(2), np.zeros(2), 1, lr=0.1)
    p2, m, v = M.adam_step(p1, g2, m, v, 2, lr=0.1)
    m2 = 0.9 * 0.1 * g1 + 0.1 * g2
    v2 = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    u1 = 0.1 * np.sign(g1) * np.abs(g1) / (np.abs(g1) + 1e-8)
    u2 = 0.1 * (m2 / (1 - 0.81)) / (np.sqrt(v2 / (1 - 0.999 ** 2)) + 1e-8)
    np.testing.assert_allclose(p2, -u1 - u2, rtol=1e-12)


def test_features_brute_force_and_invariants():
    c = cases.small_case()
    f = M.case_features(c.dwell_xyz, c.pt_xyz, c.group)
    assert f.shape == (64,)
    np.testing.assert_allclose(f.reshape(4, 16).sum(axis=1), 1.0, rtol=1e-14)
    # brute force for one structure
    j = 2
    pts = c.pt_xyz[c.group == j]
    hist = np.zeros(16)
    for q in c.dwell_xyz:
        r = min(math.dist(q, p) for p in pts)
        hist[min(int(r // 0.25), 15)] += 1
    np.testing.assert_allclose(f.reshape(4, 16)[j], hist / c.K, rtol=0, atol=1e-15)
    # translating the whole case leaves the features unchanged (distances
    # change only by rounding, far from the 0.25 cm bin edges)
    shift = np.array([0.37, -1.25, 2.5])
    np.testing.assert_array_equal(M.case_features(c.dwell_xyz + shift, c.pt_xyz + shift, c.group), f)
    # so does a quarter turn about z, (x, y) -> (-y, x): it only swaps the
    # two squared terms of each distance, which FP64 addition commutes exactly
    rot = lambda a: np.stack([-a[:, 1], a[:, 0], a[:, 2]], axis=1)
    np.testing.assert_array_equal(M.case_features(rot(c.dwell_xyz), rot(c.pt_xyz), c.group), f)
    # while moving one structure away from the dwells changes its histogram
    moved = c.pt_xyz.copy()
    moved[c.group == j] += np.array([0.0, 0.0, 10.0])
    g = M.case_features(c.dwell_xyz, moved, c.group).reshape(4, 16)
    assert g[j, 15] == 1.0 and not np.array_equal(g[j], f.reshape(4, 16)[j])


def test_init_layout():
    p = cases.mlp_init([68, 256, 256, 256, 360], seed=3)
    n = 68 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 360 + 360
    assert p.size == n
    layers = M.unpack(p, [68, 256, 256, 256, 360])
    assert layers[0][0].shape == (256, 68) and np.all(layers[-1][1] == 0.0)
    assert np.abs(layers[0][0]).max() <= math.sqrt(6.0 / 68)
