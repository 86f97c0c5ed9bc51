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
from oracle import generator as ogen

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


def test_batch_generator_matches_oracle():
    # The on-device training-data generator against the oracle's, which draws
    # the same Philox4x32-10 numbers from its own implementation: the
    # orientations to 1e-12, the labels exactly, the noisy binned inputs to
    # 1e-3 (unit variance; the FP32 projection differs from the FP64 one by
    # ~2e-5 of the master's range before the scaling to counts)
    banner("cnn batch generator vs oracle")
    t = tm()
    master = band_master()
    lib, x, y, q = _batch(t, 120, 16, seed=3)
    x, y, q = host(x), host(y), host(q)
    xr, yr, qr = ogen.make_batch(master, (0.5, 0.5, 0.6), lib, 128, 16, 1000, 3)
    assert np.max(np.abs(q - qr)) < 1e-12
    assert np.array_equal(y, yr)
    err = np.max(np.abs(x - xr))
    print("[gpu]   generator inputs max abs error %.2e" % err, flush=True)
    assert err < 1e-3
    # the same counters give the same samples
    _, x2, y2, q2 = _batch(t, 120, 16, seed=3)
    assert np.array_equal(host(x2), x) and np.array_equal(host(q2), q)


def _seeded_params(rng, n_cls):
    """He-normal weights and small biases drawn on the host (seeded), so that
    no oracle input comes from the device."""
    parts = []
    for name, s in ocnn.param_shapes(n_cls):
        fan_in = int(np.prod(s[1:])) if len(s) > 1 else 1
        scale = np.sqrt(2.0 / fan_in) if name.endswith(".w") else 0.05
        parts.append(rng.normal(size=int(np.prod(s))) * scale)
    return np.concatenate(parts).astype(np.float32)


@pytest.mark.parametrize("prec", ["bf16x2", "fp32"])
def test_forward_and_gradients_match_oracle(prec):
    # both precisions of the products (the default splits the inference, the
    # training fc and the backward products into BF16 halves)
    banner("cnn forward / backward vs oracle, %s products" % prec)
    t = tm()
    n_cls, bsz = 50, 4
    rng = np.random.default_rng(5)
    net = t.Cnn(n_cls, seed=7)
    net.set_precision(t.PREC_FP32 if prec == "fp32" else t.PREC_BF16X2)
    params = _seeded_params(rng, n_cls)
    net.set_params(dev(params))
    xs = rng.normal(size=(bsz, 64, 64)).astype(np.float32)
    ys = rng.integers(0, n_cls, size=bsz).astype(np.int32)
    x, y = dev(xs), dev(ys)
    logits = host(net.forward(x))
    ref, _ = ocnn.forward(params.astype(np.float64), xs.astype(np.float64), n_cls)
    assert np.max(np.abs(logits - ref)) <= 1e-4 * np.max(np.abs(ref))
    g, loss = net.gradients(x, y)
    g, loss = host(g).astype(np.float64), float(host(loss)[0])
    lref, gref = ocnn.loss_and_grad(params.astype(np.float64), xs.astype(np.float64), ys, n_cls)
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


def test_forward_at_full_width_matches_oracle_on_sampled_patterns():
    # 2,896 patterns (a pass of 2,048 and one of 848) and 8,000 classes: the
    # convolutions and the fc run on 128-row tiles with whole-step fetches,
    # the last fc row block on the bounds-tested path (the small case above
    # takes the 64 x 64 tiles).  A pattern's scores depend on that pattern
    # alone, so sampled rows are compared with the oracle's forward of them.
    banner("cnn forward at 2896 x 8000 vs oracle on sampled patterns")
    t = tm()
    n_cls, bsz = 8000, 2048 + 848
    rng = np.random.default_rng(11)
    net = t.Cnn(n_cls, seed=7)
    params = _seeded_params(rng, n_cls)
    net.set_params(dev(params))
    xs = rng.normal(size=(bsz, 64, 64)).astype(np.float32)
    logits = host(net.forward(dev(xs)))
    rows = [0, 1, 127, 128, 1023, 2047, 2048, 2815, 2816, bsz - 1]
    ref, _ = ocnn.forward(params.astype(np.float64), xs[rows].astype(np.float64), n_cls)
    err = np.max(np.abs(logits[rows] - ref)) / np.max(np.abs(ref))
    print("[gpu]   sampled logits relative error %.2e" % err, flush=True)
    assert err <= 1e-4
    net.close()


def test_inference_precisions_match_oracle():
    # FP32 inference products within 1e-5 of the largest score, the default
    # BF16 split (hi + lo halves, three products) within 1e-4; at 2,048
    # patterns every layer takes its 128-row tiles
    banner("cnn inference precisions vs oracle")
    t = tm()
    n_cls, bsz = 8000, 2048
    rng = np.random.default_rng(17)
    net = t.Cnn(n_cls, seed=7)
    params = _seeded_params(rng, n_cls)
    net.set_params(dev(params))
    xs = rng.normal(size=(bsz, 64, 64)).astype(np.float32)
    x = dev(xs)
    rows = [0, 5, 1000, 2047]
    ref, _ = ocnn.forward(params.astype(np.float64), xs[rows].astype(np.float64), n_cls)
    scale = np.max(np.abs(ref))
    split = host(net.forward(x))
    net.set_precision(t.PREC_FP32)
    fp32 = host(net.forward(x))
    net.set_precision(t.PREC_BF16X2)
    again = host(net.forward(x))
    e32 = np.max(np.abs(fp32[rows] - ref)) / scale
    esp = np.max(np.abs(split[rows] - ref)) / scale
    print("[gpu]   fp32 %.2e, bf16 split %.2e (relative to the largest score)" % (e32, esp), flush=True)
    assert e32 <= 1e-5
    assert esp <= 1e-4
    assert np.array_equal(split, again)
    with pytest.raises(t.EbsdError):
        net.set_precision(t.PREC_FP16X2)
    with pytest.raises(t.EbsdError):
        net.set_precision(7)
    net.close()


@pytest.mark.parametrize("prec", ["bf16x2", "fp32"])
def test_gradients_of_a_batch_are_the_mean_over_its_slices(prec):
    # A batch of 256 at 8,000 classes takes the 128-row and wide tiles, K
    # split over many slices and the whole-step fetches; the gradient of its
    # mean loss is the mean of the gradients over its 64 slices of 4, which
    # take the paths the oracle test above checks.  Sums in another order:
    # 1e-5 relative per parameter tensor, the loss 1e-6.
    banner("cnn gradients: batch of 256 vs the mean over slices of 4, %s products" % prec)
    t = tm()
    n_cls, bsz, sl = 8000, 256, 4
    rng = np.random.default_rng(13)
    net = t.Cnn(n_cls, seed=7)
    net.set_precision(t.PREC_FP32 if prec == "fp32" else t.PREC_BF16X2)
    params = _seeded_params(rng, n_cls)
    net.set_params(dev(params))
    x = dev(rng.normal(size=(bsz, 64, 64)).astype(np.float32))
    y = dev(rng.integers(0, n_cls, size=bsz).astype(np.int32))
    g, loss = net.gradients(x, y)
    g_big, loss_big = host(g).astype(np.float64), float(host(loss)[0])
    acc, lacc = np.zeros_like(g_big), 0.0
    for i in range(0, bsz, sl):
        g, loss = net.gradients(x[i:i + sl], y[i:i + sl])
        acc += host(g)
        lacc += float(host(loss)[0])
    acc /= bsz // sl
    lacc /= bsz // sl
    assert abs(loss_big - lacc) <= 1e-6 * abs(lacc)
    k = 0
    for name, s in ocnn.param_shapes(n_cls):
        m = int(np.prod(s))
        a, b = g_big[k:k + m], acc[k:k + m]
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        print("[gpu]   %s relative difference %.2e" % (name, err), flush=True)
        assert err < 1e-5, name
        k += m
    net.close()


def test_adam_steps_match_oracle():
    # three Adam steps from seeded gradients spanning eight decades (and a few
    # exact zeros) against the FP64 oracle: 1e-6 relative to max(|w|, lr)
    banner("cnn adam vs oracle")
    t = tm()
    n_cls = 20
    rng = np.random.default_rng(12)
    net = t.Cnn(n_cls, seed=3)
    w = _seeded_params(rng, n_cls)
    net.set_params(dev(w))
    cnt = w.size
    wr, m, v = w.astype(np.float64), np.zeros(cnt), np.zeros(cnt)
    lr = 1e-3
    for step in range(1, 4):
        g = (rng.normal(size=cnt) * 10.0 ** rng.uniform(-7, 1, size=cnt)).astype(np.float32)
        g[rng.integers(0, cnt, size=20)] = 0.0
        net.apply_gradient(dev(g), lr)
        wr, m, v = ocnn.adam_step(wr, g.astype(np.float64), m, v, step, lr)
        got = host(net.get_params()).astype(np.float64)
        err = np.max(np.abs(got - wr) / np.maximum(np.abs(wr), lr))
        print("[gpu]   adam step %d: max relative error %.2e" % (step, err), flush=True)
        assert err < 1e-6
    net.close()


def test_train_step_is_gradients_then_adam():
    # train_step = gradients + one Adam step, bit for bit (same kernels)
    t = tm()
    n_cls = 30
    rng = np.random.default_rng(13)
    w = dev(_seeded_params(rng, n_cls))
    a, b = t.Cnn(n_cls, seed=1), t.Cnn(n_cls, seed=2)
    a.set_params(w)
    b.set_params(w)
    x = dev(rng.normal(size=(16, 64, 64)).astype(np.float32))
    y = dev(rng.integers(0, n_cls, size=16).astype(np.int32))
    for _ in range(2):
        a.train_step(x, y, 1e-3)
        g, _ = b.gradients(x, y)
        b.apply_gradient(g, 1e-3)
    assert torch.equal(a.get_params(), b.get_params())
    a.close()
    b.close()


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


@pytest.mark.parametrize("l,k", [(300, 32), (300, 1), (300, 64), (300, 65), (50, 32), (40, 40), (8000, 32),
                                 (3000, 32)])
def test_topk_order_and_ties(l, k):
    # k <= 64 takes the threshold kernel: few entries at or above the
    # threshold (random rows), up to 1,024 (the coarse row 0: ties), more
    # (the constant rows 1 and 5: its block-argmax fallback); k = 65 the
    # block-argmax kernel; l = 50 and l = k leave threads without entries
    t = tm()
    rng = np.random.default_rng(2 + l + k)
    z = np.round(rng.normal(size=(7, l)), 1).astype(np.float32)   # many ties
    z[0, :] = np.round(rng.normal(size=l), 0)
    z[1, :] = 0.0
    z[2, 7] = np.nan
    z[3, ::3] = -0.0                                             # ties with +0.0 by value
    z[4, ::5] = -np.inf
    z[5, :] = -np.inf
    idx = host(t.cnn_topk(dev(z), k))
    for r in range(z.shape[0]):
        v = np.where(np.isnan(z[r]), -np.inf, z[r])
        want = sorted(range(l), key=lambda i: (-v[i], i))[:k]
        assert list(idx[r]) == want, r
