"""Learned right preconditioner for the Krylov solve: a small convolutional
network, its exact gradient and one Adam step, in FP64.

ORACLE - test infrastructure only.  Plain numpy loops over the 3 x 3 (2D) or
3 x 3 x 3 (3D) taps.

The paper's preconditioning discussion (section 2.5.2) motivates approximating
J^{-1} cheaply; the network form follows the design of this project:

    z = (dt/2) r + s N(r / s),       s = RMS of r over all fields and points
                                      (s = 1 for r = 0)
    N = conv(n_f -> 16) - GELU - conv(16 -> 16) - GELU - conv(16 -> 16) - GELU
        - conv(16 -> n_f),   3 x 3 kernels in 2D, 3 x 3 x 3 in 3D, with
        dilation d_l (taps at offsets d_l * (-1, 0, 1) along each axis), zero
        padding ("same"), with bias,
    GELU(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2.

Loss of a pair (r, du), averaged over a batch, in one of two norms:
  solution space   ||z(r) - du||^2 / ||du||^2
  weighted by A    ||A (z(r) - du)||^2 / ||A du||^2, A a fixed linear operator
                   (the Jacobian at rest, so that the loss measures the residual
                   J z - r that right-preconditioned GMRES sees).
Adam (Kingma and Ba 2015): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
w <- w - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Parameters are one flat vector: for each layer l, W_l[co][ci][kz][kx] in 2D,
W_l[co][ci][kz][ky][kx] in 3D (offsets dz = kz - 1, ...), then b_l[co].
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.special import erf

HIDDEN = 16
NLAYER = 4


def channels(nf):
    return [nf, HIDDEN, HIDDEN, HIDDEN, nf]


def param_shapes(nf, dim=2):
    ch = channels(nf)
    k = (3,) * dim
    out = []
    for l in range(NLAYER):
        out.append(((ch[l + 1], ch[l]) + k, (ch[l + 1],)))
    return out


def param_count(nf, dim=2):
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in param_shapes(nf, dim))


def unpack(theta, nf, dim=2):
    layers = []
    o = 0
    for ws, bs in param_shapes(nf, dim):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        layers.append((theta[o:o + nw].reshape(ws), theta[o + nw:o + nw + nb]))
        o += nw + nb
    return layers


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def _pad(x, d):
    return np.pad(x, [(0, 0)] + [(d, d)] * (x.ndim - 1))


def _taps(nsp):
    return list(itertools.product(range(3), repeat=nsp))


def _window(k, d, shape):
    """Slices of the padded array seen by tap k (one index per spatial axis)."""
    return (slice(None),) + tuple(slice(kk * d, kk * d + S) for kk, S in zip(k, shape))


def conv(x, W, b, d=1):
    """out[co, p] = b[co] + sum_ci sum_taps W[co, ci, k] x[ci, p + d(k - 1)],
    zero outside the grid.  x: (C_in, Z, X) or (C_in, Z, Y, X)."""
    S = x.shape[1:]
    xp = _pad(x, d)
    out = np.zeros((W.shape[0],) + S) + b.reshape((-1,) + (1,) * len(S))
    for k in _taps(len(S)):
        out += np.einsum("oc,c...->o...", W[(slice(None), slice(None)) + k], xp[_window(k, d, S)])
    return out


def conv_grad_input(g, W, shape_in, d=1):
    """d/dx of sum(g * conv(x)) for zero padding (the transposed convolution)."""
    S = tuple(shape_in[1:])
    gx = np.zeros((shape_in[0],) + tuple(n + 2 * d for n in S))
    for k in _taps(len(S)):
        gx[_window(k, d, S)] += np.einsum("oc,o...->c...", W[(slice(None), slice(None)) + k], g)
    return gx[(slice(None),) + tuple(slice(d, d + n) for n in S)]


def conv_grad_weight(g, x, d=1):
    S = x.shape[1:]
    xp = _pad(x, d)
    gW = np.zeros((g.shape[0], x.shape[0]) + (3,) * len(S))
    axes = "".join("zyx"[-len(S):])
    for k in _taps(len(S)):
        gW[(slice(None), slice(None)) + k] = np.einsum(f"o{axes},c{axes}->oc", g, xp[_window(k, d, S)])
    return gW, g.sum(axis=tuple(range(1, 1 + len(S))))


def field_scale(r):
    """One scale for every field: the RMS of r over all fields and points (1 when
    r = 0).  A single scale keeps the cross-field part of the inverse
    representable: a residual in one field needs a correction in the others."""
    s = float(np.sqrt(np.mean(r ** 2)))
    return np.full(r.shape[0], s if s > 0 else 1.0)


def _grid(r):
    """(n_f, nz, 1, nx) state -> (n_f, nz, nx) image; a 3D state (n_f, nz, ny,
    nx) is its own volume."""
    if r.ndim == 4 and r.shape[2] == 1:
        return r[:, :, 0, :]
    return r


def _bcast(s, nsp):
    return s.reshape((-1,) + (1,) * nsp)


def forward(theta, r, dt, keep=False, dils=(1, 1, 1, 1)):
    """z = (dt/2) r + s * N(r/s) for one 2D state-shaped r."""
    img = _grid(r)
    nf, nsp = img.shape[0], img.ndim - 1
    layers = unpack(theta, nf, nsp)
    s = field_scale(img)
    a = img / _bcast(s, nsp)
    acts, pres = [a], []
    for l, (W, b) in enumerate(layers):
        h = conv(a, W, b, dils[l])
        pres.append(h)
        a = gelu(h) if l < NLAYER - 1 else h
        acts.append(a)
    z = 0.5 * dt * img + _bcast(s, nsp) * a
    z = z.reshape(r.shape)
    if keep:
        return z, (s, acts, pres)
    return z


def loss_and_grad(theta, R, DU, dt, dils=(1, 1, 1, 1), op=None):
    """Mean over the batch of the pair loss and its gradient.  op = None: the
    solution-space loss; op = (A, AT): the loss weighted by A, with AT its
    transpose (both map state-shaped arrays)."""
    img0 = _grid(R[0])
    nf, nsp = img0.shape[0], img0.ndim - 1
    layers = unpack(theta, nf, nsp)
    total = 0.0
    grads = [(np.zeros_like(W), np.zeros_like(b)) for W, b in layers]
    B = len(R)
    for r, du in zip(R, DU):
        z, (s, acts, pres) = forward(theta, r, dt, keep=True, dils=dils)
        if op is None:
            d = _grid(z) - _grid(du)
            nd = float(np.sum(_grid(du) ** 2))
            total += float(np.sum(d * d)) / nd / B
            gz = d
        else:
            A, AT = op
            t = A(z - du)
            nd = float(np.sum(A(du) ** 2))
            total += float(np.sum(t * t)) / nd / B
            gz = _grid(AT(t))
        g = (2.0 / nd / B) * gz * _bcast(s, nsp)           # dL / d(network output)
        for l in range(NLAYER - 1, -1, -1):
            if l < NLAYER - 1:
                g = g * gelu_grad(pres[l])
            W, _ = layers[l]
            gW, gb = conv_grad_weight(g, acts[l], dils[l])
            grads[l] = (grads[l][0] + gW, grads[l][1] + gb)
            if l > 0:
                g = conv_grad_input(g, W, acts[l].shape, dils[l])
    return total, pack(grads)


def adam_step(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
