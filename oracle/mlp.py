"""Density and color MLPs, FP64 -- Sec. 5/6: a 1-hidden-layer density MLP and
a 2-hidden-layer color MLP, both 64 wide (iNGP-style); the color head ends
in a sigmoid so colors are PQ values in (0, 1) (Sec. 4.1, Sec. 6.1).

Readings: density = exp(o_0) (the workloads' activation); the color MLP
input is [o_1..o_15, SH(d)]; biases are part of the format (zero allowed).
Weights are row-major [in][out].
"""
import numpy as np


def _w(m, k):
    """Weight or bias array of the MLP dict as FP64 (Sec. 6)."""
    return np.asarray(m[k], np.float64)


def relu(z):
    """Hidden-layer activation (Sec. 6)."""
    return np.maximum(z, 0.0)


def sigmoid(z):
    """Color output activation, in PQ units (Sec. 4.1)."""
    return 1.0 / (1.0 + np.exp(-z))


def density_mlp(feats, mlp):
    """sigma = exp(o_0), geo = o_1..o_15 for encoded features [n, 2L].
    Sec. 6 (one hidden layer of 64); readings R16, R17, R19."""
    h = relu(np.asarray(feats, np.float64) @ _w(mlp, "W1") + _w(mlp, "b1"))
    o = h @ _w(mlp, "W2") + _w(mlp, "b2")
    with np.errstate(over="ignore"):
        sigma = np.exp(o[:, 0])
    return sigma, o[:, 1:]


def color_mlp(geo, sh, mlp):
    """PQ RGB = sigmoid(W5 relu(W4 relu(W3 [geo, sh] + b3) + b4) + b5).
    Sec. 6 (two hidden layers of 64), Sec. 4.1 (sigmoid in PQ units); readings R17, R19."""
    z = np.concatenate([np.asarray(geo, np.float64), np.asarray(sh, np.float64)], axis=1)
    h1 = relu(z @ _w(mlp, "W3") + _w(mlp, "b3"))
    h2 = relu(h1 @ _w(mlp, "W4") + _w(mlp, "b4"))
    return sigmoid(h2 @ _w(mlp, "W5") + _w(mlp, "b5"))
