"""FP64 CPU oracle of the learned warm start (a project extension, not in the
paper): case features, a fully connected ReLU network, its mean-squared-error
gradient and the Adam update.

TEST INFRASTRUCTURE ONLY: the product path never imports this module.

Parameter layout (shared convention with the library, written separately):
for each layer k = 0..L-1, W_k (n_out x n_in, row-major) followed by b_k
(n_out); hidden layers use ReLU, the output layer is linear.
"""
from __future__ import annotations

import numpy as np

FEATURE_BINS = 16
FEATURE_BIN_CM = 0.25


def case_features(dwell_xyz, pt_xyz, group, n_groups=4):
    """(n_groups * 16,) histogram features of one case: for every dwell l and
    structure j the distance r_lj from the dwell to the nearest point of j;
    the dwells' r_lj fall into 16 bins of 0.25 cm (the last bin also takes
    everything beyond 4 cm); each histogram is divided by the dwell count.
    Distances are (dx^2 + dy^2) + dz^2 under the square root, no fused ops."""
    K = dwell_xyz.shape[0]
    out = np.zeros((n_groups, FEATURE_BINS))
    for j in range(n_groups):
        pts = pt_xyz[group == j]
        if pts.shape[0] == 0:
            continue
        for l in range(K):
            dx = pts[:, 0] - dwell_xyz[l, 0]
            dy = pts[:, 1] - dwell_xyz[l, 1]
            dz = pts[:, 2] - dwell_xyz[l, 2]
            r = np.sqrt((dx * dx + dy * dy) + dz * dz).min()
            b = min(int(np.floor(r / FEATURE_BIN_CM)), FEATURE_BINS - 1)
            out[j, b] += 1.0
    return (out / K).reshape(-1)


def layer_shapes(sizes):
    return [(sizes[k + 1], sizes[k]) for k in range(len(sizes) - 1)]


def unpack(params, sizes):
    """Flat parameter vector -> list of (W, b)."""
    out, off = [], 0
    for (o, i) in layer_shapes(sizes):
        W = params[off:off + o * i].reshape(o, i)
        off += o * i
        b = params[off:off + o]
        off += o
        out.append((W, b))
    assert off == params.size
    return out


def forward(params, sizes, X):
    """Network output and the per-layer activations (inputs of each layer)."""
    acts = [np.asarray(X, dtype=np.float64)]
    layers = unpack(np.asarray(params, dtype=np.float64), sizes)
    h = acts[0]
    for k, (W, b) in enumerate(layers):
        z = h @ W.T + b
        h = np.maximum(z, 0.0) if k < len(layers) - 1 else z
        acts.append(h)
    return h, acts


def loss_and_grad(params, sizes, X, Y):
    """L = mean over all B x n_out entries of (f(X) - Y)^2, and dL/dparams."""
    out, acts = forward(params, sizes, X)
    layers = unpack(np.asarray(params, dtype=np.float64), sizes)
    diff = out - Y
    L = float(np.mean(diff * diff))
    g = 2.0 * diff / diff.size           # dL/d(output)
    grads = []
    for k in range(len(layers) - 1, -1, -1):
        W, _ = layers[k]
        if k < len(layers) - 1:
            g = g * (acts[k + 1] > 0.0)   # through the ReLU of layer k
        grads.append((g.T @ acts[k], g.sum(axis=0)))
        g = g @ W
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in grads])
    return L, flat


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
