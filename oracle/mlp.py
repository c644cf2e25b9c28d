"""O5: the learned initial-guess network, in float64 (test infrastructure).

A three-layer perceptron (two tanh hidden layers of width h, linear output)
maps the features of a shifted system to the reduced coordinates of its
solution; it is trained by least squares.  This module is the definition the
GPU training kernels are checked against:

  z1 = X W1^T + b1,  a1 = tanh(z1)
  z2 = a1 W2^T + b2, a2 = tanh(z2)
  Y  = a2 W3^T + b3
  L  = 1/(2N) sum_n sum_k (Y[n,k] - T[n,k])^2

and its gradients by the chain rule (d tanh(z)/dz = 1 - tanh(z)^2).  The Adam
step follows Kingma and Ba (2015), Algorithm 1, with bias correction.

Parameters travel as one flat vector in the order W1, b1, W2, b2, W3, b3, each
weight row-major [out][in].

Pins (tests/test_oracle_mlp.py): central finite differences of L; a network
whose hidden layers are bypassed (h used only through W3 = 0) reduces to the
closed-form gradient of a linear least-squares loss; the Adam step of the first
iteration moves each parameter by lr * sign(grad) up to eps.
"""
from __future__ import annotations

import numpy as np


def shapes(din: int, h: int, dout: int):
    return [(h, din), (h,), (h, h), (h,), (dout, h), (dout,)]


def n_params(din: int, h: int, dout: int) -> int:
    return sum(int(np.prod(s)) for s in shapes(din, h, dout))


def unpack(theta, din, h, dout):
    out, o = [], 0
    for s in shapes(din, h, dout):
        k = int(np.prod(s))
        out.append(np.asarray(theta[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def forward(theta, X, din, h, dout):
    W1, b1, W2, b2, W3, b3 = unpack(theta, din, h, dout)
    a1 = np.tanh(X @ W1.T + b1)
    a2 = np.tanh(a1 @ W2.T + b2)
    return a2 @ W3.T + b3, (a1, a2)


def loss(theta, X, T, din, h, dout):
    Y, _ = forward(theta, X, din, h, dout)
    return 0.5 * np.sum((Y - T) ** 2) / X.shape[0]


def grad(theta, X, T, din, h, dout):
    """(L, dL/dtheta) by back-propagation."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, din, h, dout)
    N = X.shape[0]
    Y, (a1, a2) = forward(theta, X, din, h, dout)
    dY = (Y - T) / N
    gW3 = dY.T @ a2
    gb3 = dY.sum(axis=0)
    dz2 = (dY @ W3) * (1.0 - a2 ** 2)
    gW2 = dz2.T @ a1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - a1 ** 2)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    L = 0.5 * np.sum((Y - T) ** 2) / N
    return L, np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init(din, h, dout, rng):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    parts = []
    for s in shapes(din, h, dout):
        if len(s) == 2:
            lim = 1.0 / np.sqrt(s[1])
            parts.append(rng.uniform(-lim, lim, size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)
