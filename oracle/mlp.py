"""FP64 NumPy reference of the surrogate MLP.  TEST INFRASTRUCTURE ONLY.

Network (a reading; the paper motivates a fast substitute for repeated FTLM runs
over field directions by its powder averages, Sec. 3.3): a multilayer perceptron
7 -> 256 -> 256 -> 256 -> 3 with SiLU activations, silu(z) = z / (1 + exp(-z)).

Layer k computes z_k = a_{k-1} W_k + b_k with W_k stored [fan_in, fan_out] and
a_k = silu(z_k) for the hidden layers; the output layer is linear.

Loss: mean squared error over the batch and the three outputs,
L = 1/(B*3) sum (y - t)^2.  Optimiser: Adam (Kingma & Ba, ICLR 2015) with bias
correction.

Parity status: gradients pinned to central finite differences; the first Adam
step pinned to its closed form.
"""
from __future__ import annotations

import numpy as np

LAYERS = (7, 256, 256, 256, 3)


def init_params(rng, layers=LAYERS):
    params = []
    for fi, fo in zip(layers[:-1], layers[1:]):
        W = rng.standard_normal((fi, fo)) * np.sqrt(2.0 / fi)
        b = np.zeros(fo)
        params += [W, b]
    return params


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x):
    a = np.asarray(x, np.float64)
    n = len(params) // 2
    cache = []
    for k in range(n):
        W, b = params[2 * k], params[2 * k + 1]
        z = a @ W + b
        cache.append((a, z))
        a = silu(z) if k < n - 1 else z
    return a, cache


def loss_and_grad(params, x, t):
    y, cache = forward(params, x)
    B = y.shape[0]
    diff = y - t
    loss = float(np.sum(diff ** 2) / (B * y.shape[1]))
    g = 2.0 * diff / (B * y.shape[1])
    n = len(params) // 2
    grads = [None] * len(params)
    for k in reversed(range(n)):
        a_in, z = cache[k]
        if k < n - 1:
            g = g * dsilu(z)
        grads[2 * k] = a_in.T @ g
        grads[2 * k + 1] = g.sum(0)
        g = g @ params[2 * k].T
    return loss, grads


def adam_step(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for p, g, mk, vk in zip(params, grads, m, v):
        mk = b1 * mk + (1 - b1) * g
        vk = b2 * vk + (1 - b2) * g * g
        mh = mk / (1 - b1 ** step)
        vh = vk / (1 - b2 ** step)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mk)
        out_v.append(vk)
    return out_p, out_m, out_v
