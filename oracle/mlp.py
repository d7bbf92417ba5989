"""FP64 oracle of the correction network of the learned preconditioner.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy: a 3-layer perceptron
in -> hidden -> hidden -> out with ReLU, the loss of the rank-8 block correction and the
gradients written out by the chain rule, and one Adam step.  Parameter layout: one flat
vector, W1 [in][hid], b1, W2 [hid][hid], b2, W3 [hid][out], b3 (row-major).

The loss of one sample: U, V (64 x 8, complex when the PDE is Helmholtz) are the network
output ([U | V] real, [Re U | Im U | Re V | Im V] complex); E = T - U V^T with the target
T = (X_b - D_b^{-1}) / s_b; L_b = ||E||_F^2 / ||T||_F^2; the batch loss is the mean.  By the
Eckart-Young theorem the minimiser over rank-8 U V^T is the rank-8 truncated SVD of T,
so fitting T itself is the same as fitting that truncation.
"""
from __future__ import annotations

import numpy as np

SLOTS, RANK = 64, 8


def split(p, n_in, hid, out):
    o = 0
    parts = []
    for shape in ((n_in, hid), (hid,), (hid, hid), (hid,), (hid, out), (out,)):
        n = int(np.prod(shape))
        parts.append(p[o:o + n].reshape(shape))
        o += n
    return parts


def nparams(n_in, hid, out):
    return n_in * hid + hid + hid * hid + hid + hid * out + out


def forward(p, X, n_in, hid, out):
    W1, b1, W2, b2, W3, b3 = split(p, n_in, hid, out)
    Z1 = X @ W1 + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2 + b2
    H2 = np.maximum(Z2, 0.0)
    O = H2 @ W3 + b3
    return O, (H1, H2)


def unpack(o, cplx):
    n = SLOTS * RANK
    if cplx:
        U = (o[:n] + 1j * o[n:2 * n]).reshape(SLOTS, RANK)
        V = (o[2 * n:3 * n] + 1j * o[3 * n:]).reshape(SLOTS, RANK)
    else:
        U = o[:n].reshape(SLOTS, RANK)
        V = o[n:].reshape(SLOTS, RANK)
    return U, V


def loss_and_grad(p, X, T, n_in, hid, out, cplx):
    """T: (batch, 64, 64) real or complex.  Returns (loss, grad) in FP64."""
    B = X.shape[0]
    O, (H1, H2) = forward(p, X, n_in, hid, out)
    W1, b1, W2, b2, W3, b3 = split(p, n_in, hid, out)
    dO = np.zeros_like(O)
    loss = 0.0
    n = SLOTS * RANK
    for b in range(B):
        U, V = unpack(O[b], cplx)
        E = T[b] - U @ V.T
        den = float(np.sum(np.abs(T[b]) ** 2)) or 1.0
        loss += float(np.sum(np.abs(E) ** 2)) / den / B
        # L = sum |E|^2: dL/dRe U = -2 Re(conj(E) V), dL/dIm U = 2 Im(conj(E) V),
        # dL/dRe V = -2 Re(conj(E)^T U), dL/dIm V = 2 Im(conj(E)^T U)
        GU = np.conj(E) @ V
        GV = np.conj(E).T @ U
        sc = 2.0 / den / B
        if cplx:
            dO[b] = np.concatenate([(-sc * GU.real).ravel(), (sc * GU.imag).ravel(),
                                    (-sc * GV.real).ravel(), (sc * GV.imag).ravel()])
        else:
            dO[b] = np.concatenate([(-sc * GU).ravel(), (-sc * GV).ravel()])
    gW3 = H2.T @ dO
    gb3 = dO.sum(axis=0)
    dH2 = (dO @ W3.T) * (H2 > 0)
    gW2 = H1.T @ dH2
    gb2 = dH2.sum(axis=0)
    dH1 = (dH2 @ W2.T) * (H1 > 0)
    gW1 = X.T @ dH1
    gb1 = dH1.sum(axis=0)
    g = np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return loss, g


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
