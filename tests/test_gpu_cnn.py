"""The proposal network's kernels against the FP64 oracle (oracle.cnn).

Forward scores: relative error 1e-4 of the largest |score|.  Gradient of
the mean cross-entropy: every parameter tensor within 1e-3 relative (norm of
the difference over the norm of the oracle's), the loss within 1e-5
relative.  Network inputs (binning and normalisation): 1e-5 absolute.
Labels of the training-data generator: the oracle's nearest library
orientation, exactly.  Top-k: the k largest scores, ties to the smaller
index, exactly.
"""

import numpy as np
import pytest
import torch

from fixtures import band_master, random_fz_quats, random_quats, simulate_patterns
from oracle import cnn as ocnn

from .gpu_util import banner, dev, host, tm

pytestmark = pytest.mark.gpu


def _batch(t, net_l, bsz, seed, n=128):
    lib = random_fz_quats(np.random.default_rng(seed), net_l)
    x = torch.empty((bsz, 64, 64), dtype=torch.float32, device="cuda:0")
    y = torch.empty(bsz, dtype=torch.int32, device="cuda:0")
    q = torch.empty((bsz, 4), dtype=torch.float64, device="cuda:0")
    t.cnn_make_batch(dev(band_master()), (0.5, 0.5, 0.6), dev(lib), n, bsz, 1000, seed, x=x, labels=y, q_true=q)
    return lib, x, y, q


def test_network_input_matches_oracle():
    t = tm()
    rng = np.random.default_rng(0)
    q = random_quats(rng, 3)
    pcs = np.tile([0.5, 0.5, 0.6], (3, 1))
    pats = simulate_patterns(q, 128, pcs, ("poisson", 300.0), seed=1).numpy()
    x = host(t.Cnn.input(dev(pats)))
    for k in range(3):
        assert np.max(np.abs(x[k] - ocnn.network_input(pats[k]))) < 1e-5


def test_batch_generator_labels_and_inputs():
    banner("cnn batch generator")
    t = tm()
    lib, x, y, q = _batch(t, 120, 16, seed=3)
    x, y, q = host(x), host(y), host(q)
    assert np.all(np.isfinite(x))
    assert np.allclose(x.mean(axis=(1, 2)), 0.0, atol=1e-4) and np.allclose(x.std(axis=(1, 2)), 1.0, atol=1e-3)
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-12) and np.all(q[:, 0] >= 0)
    for j in range(16):
        assert y[j] == ocnn.nearest_library(q[j], lib)
    # the same counters give the same samples
    _, x2, y2, q2 = _batch(t, 120, 16, seed=3)
    assert np.array_equal(host(x2), x) and np.array_equal(host(q2), q)


def test_forward_and_gradients_match_oracle():
    banner("cnn forward / backward vs oracle")
    t = tm()
    n_cls, bsz = 50, 4
    net = t.Cnn(n_cls, seed=7)
    _, x, y, _ = _batch(t, n_cls, bsz, seed=5)
    params = host(net.get_params()).astype(np.float64)
    xs, ys = host(x).astype(np.float64), host(y)
    logits = host(net.forward(x))
    ref, _ = ocnn.forward(params, xs, n_cls)
    assert np.max(np.abs(logits - ref)) <= 1e-4 * np.max(np.abs(ref))
    g, loss = net.gradients(x, y)
    g, loss = host(g).astype(np.float64), float(host(loss)[0])
    lref, gref = ocnn.loss_and_grad(params, xs, ys, n_cls)
    assert abs(loss - lref) <= 1e-5 * abs(lref)
    k = 0
    for name, s in ocnn.param_shapes(n_cls):
        m = int(np.prod(s))
        a, b = g[k:k + m], gref[k:k + m]
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        print("[gpu]   %s relative error %.2e" % (name, err), flush=True)
        assert err < 1e-3, name
        k += m
    net.close()


def test_set_params_round_trip_and_train_step_lowers_loss():
    t = tm()
    n_cls = 30
    net = t.Cnn(n_cls, seed=11)
    p0 = net.get_params()
    net.set_params(p0 * 0.5)
    assert torch.equal(net.get_params(), p0 * 0.5)
    net.set_params(p0)
    _, x, y, _ = _batch(t, n_cls, 32, seed=9)
    l0 = float(host(net.gradients(x, y)[1])[0])
    for _ in range(20):
        net.train_step(x, y, 1e-3)
    l1 = float(host(net.gradients(x, y)[1])[0])
    assert l1 < 0.5 * l0
    net.close()


def test_topk_order_and_ties():
    t = tm()
    rng = np.random.default_rng(2)
    z = np.round(rng.normal(size=(5, 300)), 1).astype(np.float32)   # many ties
    z[1, :] = 0.0
    z[2, 7] = np.nan
    idx = host(t.cnn_topk(dev(z), 32))
    for r in range(5):
        v = np.where(np.isnan(z[r]), -np.inf, z[r])
        want = sorted(range(300), key=lambda i: (-v[i], i))[:32]
        assert list(idx[r]) == want
