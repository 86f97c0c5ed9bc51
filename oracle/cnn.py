"""Proposal network in FP64 (oracle; test only).

The method ranks every library template by correlation; the learned
proposal replaces that exhaustive ranking by a small convolutional network
that maps a pattern to scores over the library orientations, so that the
correlation runs only on the best k.  The network (the paper names no
network; this is the reading built here):

    input   the pattern binned by block means to 64 x 64, then (x - mean) / std
    conv i  3 x 3, zero padding 1, stride 1, bias, ReLU, then 2 x 2 max pool,
            for i = 1..4 with 1 -> 32 -> 64 -> 128 -> 128 channels
            (64 -> 32 -> 16 -> 8 -> 4 pixels per side)
    fc      the 128 x 4 x 4 features (channel-major) -> L scores, bias
    loss    softmax cross-entropy against the nearest library orientation
            (cubic disorientation), mean over the batch

Conventions fixed here: ReLU'(0) = 0; a 2 x 2 max pool passes its gradient to
the first maximal input in the order (0, 0), (0, 1), (1, 0), (1, 1).
Parameters are one flat vector, in the order conv1.w, conv1.b, ..., conv4.w,
conv4.b, fc.w, fc.b, each row-major (conv weights [out][in][3][3], fc
weights [L][features]).
"""

import numpy as np

from . import rotations

CHANNELS = (32, 64, 128, 128)
IN_SIZE = 64


def param_shapes(n_classes, in_size=IN_SIZE, channels=CHANNELS):
    shapes = []
    ci = 1
    for i, co in enumerate(channels):
        shapes.append(("conv%d.w" % (i + 1), (co, ci, 3, 3)))
        shapes.append(("conv%d.b" % (i + 1), (co,)))
        ci = co
    side = in_size // 2 ** len(channels)
    shapes.append(("fc.w", (n_classes, ci * side * side)))
    shapes.append(("fc.b", (n_classes,)))
    return shapes


def param_count(n_classes, in_size=IN_SIZE, channels=CHANNELS):
    return int(sum(np.prod(s) for _, s in param_shapes(n_classes, in_size, channels)))


def unpack(flat, shapes):
    out, k = {}, 0
    for name, s in shapes:
        m = int(np.prod(s))
        out[name] = np.asarray(flat[k:k + m], dtype=np.float64).reshape(s)
        k += m
    return out


def pack(tensors, shapes):
    return np.concatenate([np.asarray(tensors[name], dtype=np.float64).reshape(-1) for name, _ in shapes])


def conv3x3(x, w, b):
    """x [B][Ci][H][W], w [Co][Ci][3][3]: out[b, o, y, x] = b[o] +
    sum_{c, dy, dx} x[b, c, y + dy - 1, x + dx - 1] w[o, c, dy, dx] (zeros outside)."""
    bsz, _, h, wd = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.zeros((bsz, w.shape[0], h, wd))
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("bchw,oc->bohw", xp[:, :, dy:dy + h, dx:dx + wd], w[:, :, dy, dx])
    return out + b[None, :, None, None]


def conv3x3_backward(x, w, g):
    """Gradients of sum(g * conv3x3(x, w, b)) with respect to x, w and b."""
    bsz, _, h, wd = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for dy in range(3):
        for dx in range(3):
            dw[:, :, dy, dx] = np.einsum("bohw,bchw->oc", g, xp[:, :, dy:dy + h, dx:dx + wd])
            dxp[:, :, dy:dy + h, dx:dx + wd] += np.einsum("bohw,oc->bchw", g, w[:, :, dy, dx])
    return dxp[:, :, 1:-1, 1:-1], dw, g.sum(axis=(0, 2, 3))


def maxpool2(x):
    """2 x 2 max pool; also the index (0..3) of the first maximal input."""
    bsz, c, h, wd = x.shape
    v = x.reshape(bsz, c, h // 2, 2, wd // 2, 2).transpose(0, 1, 2, 4, 3, 5).reshape(bsz, c, h // 2, wd // 2, 4)
    return v.max(axis=-1), v.argmax(axis=-1)


def maxpool2_backward(idx, g, shape):
    bsz, c, h, wd = shape
    onehot = np.zeros(idx.shape + (4,))
    np.put_along_axis(onehot, idx[..., None], 1.0, axis=-1)
    d = onehot * g[..., None]
    return d.reshape(bsz, c, h // 2, wd // 2, 2, 2).transpose(0, 1, 2, 4, 3, 5).reshape(shape)


def forward(params, x, n_classes, channels=CHANNELS):
    """x [B][H][W] network inputs.  Returns (logits [B][L], cache)."""
    shapes = param_shapes(n_classes, x.shape[-1], channels)
    p = unpack(params, shapes)
    a = np.asarray(x, dtype=np.float64)[:, None]
    cache = []
    for i in range(len(channels)):
        z = conv3x3(a, p["conv%d.w" % (i + 1)], p["conv%d.b" % (i + 1)])
        r = np.maximum(z, 0.0)
        pooled, idx = maxpool2(r)
        cache.append((a, z, idx, r.shape))
        a = pooled
    f = a.reshape(a.shape[0], -1)
    logits = f @ p["fc.w"].T + p["fc.b"]
    return logits, (p, shapes, cache, f)


def softmax_xent(logits, labels):
    """Mean cross-entropy and its gradient with respect to the logits."""
    z = logits - logits.max(axis=1, keepdims=True)
    e = np.exp(z)
    s = e.sum(axis=1, keepdims=True)
    bsz = logits.shape[0]
    loss = float(np.mean(np.log(s[:, 0]) - z[np.arange(bsz), labels]))
    d = e / s
    d[np.arange(bsz), labels] -= 1.0
    return loss, d / bsz


def loss_and_grad(params, x, labels, n_classes, channels=CHANNELS):
    """Mean softmax cross-entropy and the gradient (flat, parameter order)."""
    logits, (p, shapes, cache, f) = forward(params, x, n_classes, channels)
    loss, dz = softmax_xent(logits, np.asarray(labels))
    grads = {"fc.w": dz.T @ f, "fc.b": dz.sum(axis=0)}
    da = (dz @ p["fc.w"]).reshape((f.shape[0],) + cache[-1][3][1:2] + (cache[-1][3][2] // 2, cache[-1][3][3] // 2))
    for i in reversed(range(len(channels))):
        a_in, z, idx, rshape = cache[i]
        dr = maxpool2_backward(idx, da, rshape)
        dzc = dr * (z > 0.0)
        dx, dw, db = conv3x3_backward(a_in, p["conv%d.w" % (i + 1)], dzc)
        grads["conv%d.w" % (i + 1)] = dw
        grads["conv%d.b" % (i + 1)] = db
        da = dx
    return loss, pack(grads, shapes)


def network_input(img, size=IN_SIZE):
    """Block-mean binning of a square pattern to size x size, then (x - mean) / std."""
    img = np.asarray(img, dtype=np.float64)
    f = img.shape[0] // size
    if f * size != img.shape[0]:
        raise ValueError("pattern side must be a multiple of %d" % size)
    b = img.reshape(size, f, size, f).mean(axis=(1, 3))
    sd = b.std()
    return (b - b.mean()) / sd if sd > 0 else b - b.mean()


def nearest_library(q, lib_q):
    """Index of the library orientation with the smallest cubic disorientation
    from q (ties: smallest index): the largest trace of R_q^T S R_l over the
    24 proper operators S (trace = 1 + 2 cos(angle))."""
    ops = rotations.cubic_operators()
    rq = rotations.quat_to_matrix(np.asarray(q, dtype=np.float64))
    rl = rotations.quat_to_matrix(np.asarray(lib_q, dtype=np.float64).reshape(-1, 4))
    srl = np.einsum("sij,ljk->slik", ops, rl)
    tr = np.einsum("ij,slij->sl", rq, srl).max(axis=0)
    return int(np.argmax(tr))


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, ICLR 2015, Algorithm 1) on parameters w
    with gradient g at step t = 1, 2, ...: biased moment estimates m and v,
    their bias-corrected forms m / (1 - beta1^t) and v / (1 - beta2^t), and
    w - lr m_hat / (sqrt(v_hat) + eps).  Returns (w, m, v)."""
    w, g, m, v = (np.asarray(a, dtype=np.float64) for a in (w, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return w - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
