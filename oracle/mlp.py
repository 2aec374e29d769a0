"""Surrogate network of the learned form (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper computes I(w_in, w) with the solver only; the learned form places a
small regression network beside it that maps the model and grid parameters
(U, t', U_c, Gamma, w_in, w) to I and falls back to the solver where an
ensemble of such networks disagrees.  Nothing here comes from the paper: the
pieces are textbook definitions, written out plainly in float64:

* multilayer perceptron 6 -> 512 -> 512 -> 512 -> 1, affine layers
  z = h W + b with W stored [in][out], GELU between them and a linear output;
* GELU(x) = x Phi(x) with the exact normal CDF Phi(x) = (1 + erf(x / sqrt 2)) / 2
  (Hendrycks and Gimpel), derivative Phi(x) + x phi(x);
* loss = mean over the batch of (y - t)^2;
* gradients by the chain rule, layer by layer (reverse mode);
* Adam (Kingma and Ba) with bias correction:
  m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
  p <- p - lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps).

Mixed precision.  The GPU kernels multiply bfloat16 operands with float32
accumulation: weights are rounded to bfloat16 before every product and the
activations that feed a product are stored in bfloat16 (the first layer's
inputs and the last layer's weights excepted: they are kept in float32).
``forward``/``backward`` take ``bf16_ops=True`` to apply exactly these roundings
(round to nearest even of the float32 value) so that the kernels can be
compared element by element; all other arithmetic stays float64.

Parameters are one flat float vector per network in the order
W1[6][512], b1[512], W2[512][512], b2[512], W3[512][512], b3[512], W4[512], b4[1]
(``layout``); widths are arguments so that the pins can use small networks.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

WIDTHS = (6, 512, 512, 512, 1)


def layout(widths=WIDTHS):
    """[(name, shape)] of the flat parameter vector."""
    out = []
    for i in range(len(widths) - 1):
        out.append((f"W{i + 1}", (widths[i], widths[i + 1])))
        out.append((f"b{i + 1}", (widths[i + 1],)))
    return out


def num_params(widths=WIDTHS) -> int:
    return sum(int(np.prod(s)) for _, s in layout(widths))


def unflatten(p, widths=WIDTHS):
    """Views of the flat vector as {name: array}."""
    out, o = {}, 0
    for name, shape in layout(widths):
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def flatten(d, widths=WIDTHS):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in layout(widths)])


def bf16(x):
    """Round to bfloat16 (nearest even) through float32, returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def normalize(X, shift, scale):
    """Network inputs (x - shift) * scale, feature by feature."""
    return (np.asarray(X, dtype=np.float64) - np.asarray(shift)) * np.asarray(scale)


def _operand_weight(W, i, L, bf16_ops):
    """Weight as the layer-i product sees it: bfloat16 for the inner
    (matrix-core) layers, float32 for the first and the last layer."""
    if not bf16_ops:
        return W
    if i == 1 or i == L:
        return W.astype(np.float32).astype(np.float64)
    return bf16(W)


def forward(p, Xn, widths=WIDTHS, bf16_ops=False):
    """Outputs y [n] and the cache for ``backward``.  Xn: normalized inputs [n][6]."""
    P = unflatten(np.asarray(p, dtype=np.float64), widths)
    L = len(widths) - 1
    h = np.asarray(Xn, dtype=np.float64)
    if bf16_ops:
        h = h.astype(np.float32).astype(np.float64)
    cache = {"h0": h}
    for i in range(1, L + 1):
        z = h @ _operand_weight(P[f"W{i}"], i, L, bf16_ops) + P[f"b{i}"]
        cache[f"z{i}"] = z
        if i < L:
            h = gelu(z)
            if bf16_ops:
                h = bf16(h)                  # stored activations feed the next product
            cache[f"h{i}"] = h
    return z[:, 0], cache


def loss(y, t):
    return float(np.mean((np.asarray(y) - np.asarray(t)) ** 2))


def backward(p, cache, y, t, widths=WIDTHS, bf16_ops=False):
    """Gradient of ``loss`` with respect to the flat parameters.

    With ``bf16_ops`` the back-propagated dz of every hidden layer is stored in
    bfloat16 (it is the operand of the weight-gradient and of the next
    product), as on the GPU; the output-layer dz stays float32."""
    P = unflatten(np.asarray(p, dtype=np.float64), widths)
    L = len(widths) - 1
    n = len(y)
    g = {}
    dz = (2.0 / n) * (np.asarray(y) - np.asarray(t))[:, None]      # d loss / d z_L
    for i in range(L, 0, -1):
        g[f"W{i}"] = cache[f"h{i - 1}"].T @ dz
        g[f"b{i}"] = dz.sum(axis=0)
        if i > 1:
            dh = dz @ _operand_weight(P[f"W{i}"], i, L, bf16_ops).T
            dz = dh * gelu_grad(cache[f"z{i - 1}"])
            if bf16_ops:
                dz = bf16(dz)
    return flatten(g, widths)


def adam_step(p, grad, m, v, k, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number k >= 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** k)
    vh = v / (1.0 - b2 ** k)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def fallback_rows(mean, std, frac):
    """Rows of a [n_win][n_w] prediction grid whose ensemble spread exceeds
    frac times the peak of the mean prediction anywhere in the row."""
    peak = float(np.max(mean))
    return np.any(std > frac * peak, axis=1)
