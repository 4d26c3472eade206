"""FP64 reference of the surrogate network (test infrastructure only, see
``oracle/__init__.py``): forward, mean-squared-error backward and AdamW,
written from the definitions.

Network: a_0 = x; z_l = a_{l-1} W_l^T + b_l; a_l = GELU(z_l) for hidden
layers, y = z_L for the last.  GELU(z) = z Phi(z) with the exact normal CDF
Phi(z) = (1 + erf(z / sqrt 2)) / 2.  Loss = mean over batch and outputs of
(y - t)^2.  AdamW: moments m, v with bias correction; the weight decay acts
on the weights directly (decoupled), not on the biases.
Parameters travel as one flat vector [W_1 (out x in), b_1, W_2, b_2, ...].
"""
import numpy as np
from scipy.special import erf

SQRT2 = np.sqrt(2.0)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def unflatten(flat, dims):
    flat = np.asarray(flat, dtype=np.float64)
    out, off = [], 0
    for l in range(len(dims) - 1):
        n_in, n_out = dims[l], dims[l + 1]
        w = flat[off:off + n_in * n_out].reshape(n_out, n_in)
        off += n_in * n_out
        b = flat[off:off + n_out]
        off += n_out
        out.append((w, b))
    assert off == flat.size
    return out


def flatten(layers):
    return np.concatenate([np.concatenate([w.ravel(), b]) for w, b in layers])


def forward(flat, dims, x):
    layers = unflatten(flat, dims)
    a = np.asarray(x, dtype=np.float64)
    cache = [(a, None)]
    for l, (w, b) in enumerate(layers):
        z = a @ w.T + b
        a = gelu(z) if l + 1 < len(layers) else z
        cache.append((a, z))
    return a, cache


def loss_and_grads(flat, dims, x, t):
    layers = unflatten(flat, dims)
    y, cache = forward(flat, dims, x)
    t = np.asarray(t, dtype=np.float64)
    r = y - t
    loss = np.mean(r * r)
    dz = 2.0 * r / r.size
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        a_prev = cache[l][0]
        grads[l] = (dz.T @ a_prev, dz.sum(axis=0))
        if l > 0:
            dz = (dz @ layers[l][0]) * gelu_grad(cache[l][1])
    return loss, flatten(grads)


def init_params(dims, seed):
    """He-style normal weights scaled by 1/sqrt(fan_in), zero biases."""
    rng = np.random.default_rng(seed)
    layers = []
    for l in range(len(dims) - 1):
        w = rng.standard_normal((dims[l + 1], dims[l])) / np.sqrt(dims[l])
        layers.append((w, np.zeros(dims[l + 1])))
    return flatten(layers)


def adamw(flat, grad, m, v, step, dims, lr, b1, b2, eps, wd):
    """One AdamW step; returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    decay = np.concatenate([np.concatenate([np.full(dims[l] * dims[l + 1], wd), np.zeros(dims[l + 1])])
                            for l in range(len(dims) - 1)])
    new = flat - lr * (mh / (np.sqrt(vh) + eps) + decay * flat)
    return new, m, v
