"""FP64 reference of the surrogate network -- TEST INFRASTRUCTURE ONLY.

The surrogate stands in for the ionic one-step map (V, g) -> (V + dt(-I_ion), g+)
of the explicit scheme (eq (Euler) and eqs (RL), (RLcoeff)).  It is a plain
multilayer perceptron nin -> H -> H -> nout with SiLU activations, on normalised
inputs x = (s - mu_in) / sigma_in, predicting normalised increments
d = ((s+ - s) - mu_out) / sigma_out.  Training minimises the mean squared error
over the batch and the nout outputs with Adam.

Everything here is written from those definitions in float64 with numpy (a
matmul is the only library primitive).  Parameters use the canonical flat
layout shared with the GPU library's parameter import/export:
    W1 [H][nin], b1 [H], W2 [H][H], b2 [H], W3 [nout][H], b3 [nout].
Pinned by the CPU tests: gradients against central finite differences, SiLU
derivative against its closed form, Adam against its closed form on a known
gradient sequence.
"""
from __future__ import annotations

import numpy as np


def sizes(nin: int, hid: int, nout: int):
    return [("W1", (hid, nin)), ("b1", (hid,)), ("W2", (hid, hid)), ("b2", (hid,)),
            ("W3", (nout, hid)), ("b3", (nout,))]


def nparams(nin: int, hid: int, nout: int) -> int:
    return sum(int(np.prod(s)) for _, s in sizes(nin, hid, nout))


def unpack(theta, nin, hid, nout):
    out, o = {}, 0
    for name, s in sizes(nin, hid, nout):
        n = int(np.prod(s))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(s)
        o += n
    return out


def pack(p, nin, hid, nout):
    return np.concatenate([np.asarray(p[name], np.float64).ravel()
                           for name, _ in sizes(nin, hid, nout)])


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X, nin, hid, nout):
    """X: (N, nin) normalised inputs -> (N, nout) outputs, plus the intermediates."""
    p = unpack(theta, nin, hid, nout)
    Z1 = X @ p["W1"].T + p["b1"]
    H1 = silu(Z1)
    Z2 = H1 @ p["W2"].T + p["b2"]
    H2 = silu(Z2)
    O = H2 @ p["W3"].T + p["b3"]
    return O, (X, Z1, H1, Z2, H2)


def loss_and_grad(theta, X, T, nin, hid, nout):
    """Mean squared error over N samples and nout outputs, and its gradient."""
    O, (X, Z1, H1, Z2, H2) = forward(theta, X, nin, hid, nout)
    p = unpack(theta, nin, hid, nout)
    N = X.shape[0]
    R = O - T
    L = float((R * R).sum() / (N * nout))
    dO = 2.0 * R / (N * nout)
    g = {"W3": dO.T @ H2, "b3": dO.sum(0)}
    dZ2 = (dO @ p["W3"]) * silu_grad(Z2)
    g["W2"], g["b2"] = dZ2.T @ H1, dZ2.sum(0)
    dZ1 = (dZ2 @ p["W2"]) * silu_grad(Z1)
    g["W1"], g["b1"] = dZ1.T @ X, dZ1.sum(0)
    return L, pack(g, nin, hid, nout)


def adam_step(theta, m, v, grad, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step index t >= 1) with bias-corrected moments."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def normalise_in(S, mean, scale):
    """x = (s - mean) * scale, scale = 1/sigma."""
    return (np.asarray(S, np.float64) - mean) * scale


def denormalise_out(D, mean, sigma):
    """Increment from a normalised prediction: sigma * d + mean."""
    return np.asarray(D, np.float64) * sigma + mean
