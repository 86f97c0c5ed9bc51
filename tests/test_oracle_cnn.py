"""Pins for oracle.cnn (the proposal network's forward and backward pass in
FP64): the layers against library routines and closed forms, and the whole
gradient against central finite differences on a tiny instance."""

import numpy as np
import pytest
from scipy.signal import correlate2d

from fixtures import random_quats
from oracle import cnn
from oracle import rotations as rot


def test_conv3x3_is_zero_padded_cross_correlation():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 7, 9))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    out = cnn.conv3x3(x, w, b)
    for i in range(2):
        for o in range(4):
            ref = sum(correlate2d(x[i, c], w[o, c], mode="same", boundary="fill") for c in range(3)) + b[o]
            assert np.allclose(out[i, o], ref, atol=1e-12)


def test_maxpool_values_and_first_index_ties():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 3, 6, 4))
    p, idx = cnn.maxpool2(x)
    assert np.allclose(p, x.reshape(2, 3, 3, 2, 2, 2).max(axis=(3, 5)))
    t = np.array([[[[1.0, 3.0], [3.0, 2.0]]]])          # tie between (0, 1) and (1, 0)
    _, it = cnn.maxpool2(t)
    assert it[0, 0, 0, 0] == 1
    z = np.zeros((1, 1, 2, 2))
    _, iz = cnn.maxpool2(z)
    assert iz[0, 0, 0, 0] == 0
    g = cnn.maxpool2_backward(it, np.array([[[[5.0]]]]), t.shape)
    assert np.array_equal(g, np.array([[[[0.0, 5.0], [0.0, 0.0]]]]))


def test_softmax_xent_closed_forms():
    l = 7
    loss, d = cnn.softmax_xent(np.zeros((3, l)), np.array([0, 3, 6]))
    assert abs(loss - np.log(l)) < 1e-15
    assert np.allclose(d.sum(axis=1), 0.0, atol=1e-16)
    assert np.allclose(d[0], (np.full(l, 1.0 / l) - np.eye(l)[0]) / 3)
    # a dominant correct logit drives the loss to zero
    z = np.zeros((1, l))
    z[0, 2] = 50.0
    assert cnn.softmax_xent(z, np.array([2]))[0] < 1e-20


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    ch, size, l, bsz = (2, 3, 3, 4), 16, 5, 2
    shapes = cnn.param_shapes(l, size, ch)
    n = cnn.param_count(l, size, ch)
    params = rng.normal(scale=0.5, size=n)
    x = rng.normal(size=(bsz, size, size))
    y = np.array([1, 4])
    _, g = cnn.loss_and_grad(params, x, y, l, ch)
    h = 1e-6
    fd = np.zeros(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        lp = cnn.softmax_xent(cnn.forward(params + e, x, l, ch)[0], y)[0]
        lm = cnn.softmax_xent(cnn.forward(params - e, x, l, ch)[0], y)[0]
        fd[i] = (lp - lm) / (2 * h)
    k = 0
    for name, s in shapes:
        m = int(np.prod(s))
        a, b = g[k:k + m], fd[k:k + m]
        assert np.linalg.norm(a - b) <= 1e-6 * max(np.linalg.norm(b), 1e-12), name
        assert np.linalg.norm(b) > 0, name
        k += m


def test_full_architecture_shapes():
    assert cnn.param_count(8000) == 240256 + 8000 * 2048 + 8000
    x = np.random.default_rng(3).normal(size=(1, 64, 64))
    logits, _ = cnn.forward(np.zeros(cnn.param_count(10)), x, 10)
    assert logits.shape == (1, 10) and np.all(logits == 0)


def test_nearest_library_is_the_smallest_disorientation():
    rng = np.random.default_rng(4)
    lib = random_quats(rng, 40)
    ops = rot.cubic_operators()
    for t in range(5):
        q = random_quats(rng, 1)[0]
        want = int(np.argmin([rot.disorientation(rot.quat_to_matrix(q), rot.quat_to_matrix(p)) for p in lib]))
        assert cnn.nearest_library(q, lib) == want
        # a symmetry-equivalent copy of entry j is nearest to j
        j = int(rng.integers(40))
        qe = rot.matrix_to_quat(ops[t + 3] @ rot.quat_to_matrix(lib[j]))
        assert cnn.nearest_library(qe, lib) == j


def test_network_input_bins_and_normalises():
    rng = np.random.default_rng(5)
    blocks = rng.normal(size=(64, 64))
    img = np.kron(blocks, np.ones((2, 2)))
    x = cnn.network_input(img)
    assert np.allclose(x, (blocks - blocks.mean()) / blocks.std())
    assert abs(x.mean()) < 1e-12 and abs(x.std() - 1) < 1e-12
    with pytest.raises(ValueError):
        cnn.network_input(np.zeros((96, 96)))


def test_adam_constant_gradient_moves_by_lr():
    # For a constant gradient the bias corrections are exact: m_hat = g and
    # v_hat = g^2 at every step, so each step moves every parameter by
    # lr g / (|g| + eps) (a step without the bias correction moves the first
    # step by lr (1 - b1) / sqrt(1 - b2) = 3.16 lr instead)
    rng = np.random.default_rng(10)
    w0 = rng.normal(size=50)
    g = rng.normal(size=50) * np.logspace(-6, 2, 50)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    lr = 1e-3
    for t in range(1, 6):
        w, m, v = cnn.adam_step(w, g, m, v, t, lr)
        assert np.allclose(w, w0 - t * lr * g / (np.abs(g) + 1e-8), atol=1e-15, rtol=1e-12)
    # zero gradient: nothing moves
    w2, _, _ = cnn.adam_step(w0, np.zeros(50), np.zeros(50), np.zeros(50), 1, lr)
    assert np.array_equal(w2, w0)


def test_adam_alternating_gradient_geometric_series():
    # g_k = (-1)^(k+1): v_hat = 1 exactly, and m_t = (1 - b1) sum_k b1^(t-k) g_k
    # is a geometric series, m_t = (1 - b1) (-1)^(t+1) (1 - (-b1)^t) / (1 + b1),
    # so the step is lr m_t / ((1 - b1^t)(1 + eps)).  Swapped betas or a
    # moment update with the weights exchanged fail this.
    b1 = 0.9
    lr = 0.01
    w, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    for t in range(1, 9):
        g = np.array([(-1.0) ** (t + 1)])
        w_new, m, v = cnn.adam_step(w, g, m, v, t, lr)
        m_t = (1 - b1) * (-1.0) ** (t + 1) * (1 - (-b1) ** t) / (1 + b1)
        assert abs(m[0] - m_t) < 1e-15
        assert abs((w - w_new)[0] - lr * m_t / ((1 - b1 ** t) * (1 + 1e-8))) < 1e-15
        w = w_new
