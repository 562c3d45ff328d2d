"""FP64 CPU oracle of the learned subspace initialisation (test infrastructure only).

A small 4D convolutional network maps per-site inputs (the gauge field and
noise) to Ns start fields for the subspace generation of section 5.3; it is
trained to make the block-projected span of its outputs contain low modes
produced by the inverse iteration of eq. (5.1). The paper has no network; this
module fixes the definitions the HIP kernels are checked against:

* inputs: 96 reals per site, 72 from the links (``link_features``) and 24 from
  a seeded Gaussian noise field;
* ``conv4d``: out[x, co] = b[co] + sum_{o in {-1,0,1}^4} sum_ci W[o+1, ci, co] in[x+o, ci]
  with periodic boundaries, followed by SiLU z*sigmoid(z) on all but the last
  layer;
* ``outputs_to_fields``: output channel (l*12 + c)*2 + r is the real (r = 0)
  or imaginary (r = 1) part of component c of start field l;
* ``deficit_loss``: the mean over target fields t_k of the deficit of
  eq. (3.15), ||(1 - P) t_k||^2 / ||t_k||^2, where P projects block by block
  onto the span of the network's fields (the subspace that the block
  Gram-Schmidt of eq. (4.2) turns into a basis); its gradient with respect to
  conj(Psi) on block Lambda is -sum_k (t_k - Psi y_k) y_k^+ / (K ||t_k||^2),
  y_k = G^-1 Psi^+ t_k, G = Psi^+ Psi;
* ``adam``: the Adam update (Kingma and Ba) with bias correction.

Arrays are canonical-order numpy arrays: activations (V, C) with the site
index of ``latgen`` (x0 slowest); fields (n, V, 12) complex.
"""
from __future__ import annotations

import itertools

import numpy as np

from .dfl import to_blocks

OFFSETS = list(itertools.product((-1, 0, 1), repeat=4))  # tap t <-> offsets o, t = sum (o_mu+1) 3^(3-mu)
N_LINK_FEATURES = 72
N_NOISE = 24


def link_features(U) -> np.ndarray:
    """(V, 72): Re and Im of U_mu(x)[a, b], channel ((mu*3 + a)*3 + b)*2 + r."""
    U = np.asarray(U, dtype=np.complex128)
    V = U.shape[0]
    return np.stack([U.real, U.imag], axis=-1).reshape(V, N_LINK_FEATURES)


def net_inputs(U, noise) -> np.ndarray:
    """(V, 96): link features followed by the 24 noise channels."""
    return np.concatenate([link_features(U), np.asarray(noise, dtype=np.float64).reshape(-1, N_NOISE)], axis=1)


def _lat(a, dims):
    return np.asarray(a, dtype=np.float64).reshape(tuple(dims) + (-1,))


def shifted(a4, o):
    """b[x] = a[x + o] on the periodic lattice (a4: (L0, L1, L2, L3, C))."""
    return np.roll(a4, shift=tuple(-int(v) for v in o), axis=(0, 1, 2, 3))


def conv4d(x, W, b, dims) -> np.ndarray:
    """Periodic 3^4 convolution: (V, Cin) -> (V, Cout); W (3,3,3,3,Cin,Cout), b (Cout,)."""
    x4 = _lat(x, dims)
    out = np.zeros(tuple(dims) + (W.shape[-1],))
    for o in OFFSETS:
        out += shifted(x4, o) @ W[tuple(v + 1 for v in o)]
    out += b
    return out.reshape(-1, W.shape[-1])


def conv4d_backward(x, W, dout, dims):
    """Gradients of sum(dout * conv4d(x, W, b)): returns (dx, dW, db)."""
    x4 = _lat(x, dims)
    g4 = _lat(dout, dims)
    dW = np.zeros_like(W, dtype=np.float64)
    dx = np.zeros_like(x4)
    for o in OFFSETS:
        t = tuple(v + 1 for v in o)
        xs = shifted(x4, o)                                   # x[y + o]
        dW[t] = xs.reshape(-1, x4.shape[-1]).T @ g4.reshape(-1, g4.shape[-1])
        dx += shifted(g4, tuple(-v for v in o)) @ W[t].T      # dout[y - o] W^T
    db = g4.reshape(-1, g4.shape[-1]).sum(axis=0)
    return dx.reshape(-1, x4.shape[-1]), dW, db


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, dims):
    """Layers (W_i, b_i); returns the output and the per-layer (input, pre-activation) cache."""
    cache = []
    a = np.asarray(x, dtype=np.float64)
    for i, (W, b) in enumerate(params):
        z = conv4d(a, W, b, dims)
        cache.append((a, z))
        a = silu(z) if i < len(params) - 1 else z
    return a, cache


def backward(params, cache, dout, dims):
    """Gradients [(dW_i, db_i)] of sum(dout * forward(...)) by the chain rule."""
    grads = [None] * len(params)
    g = np.asarray(dout, dtype=np.float64)
    for i in range(len(params) - 1, -1, -1):
        a, z = cache[i]
        if i < len(params) - 1:
            g = g * silu_grad(z)
        dx, dW, db = conv4d_backward(a, params[i][0], g, dims)
        grads[i] = (dW, db)
        g = dx
    return grads


def outputs_to_fields(out, Ns: int) -> np.ndarray:
    """(V, 24*Ns) real -> (Ns, V, 12) complex."""
    o = np.asarray(out, dtype=np.float64).reshape(out.shape[0], Ns, 12, 2)
    return (o[..., 0] + 1j * o[..., 1]).transpose(1, 0, 2)


def fields_grad_to_outputs(g) -> np.ndarray:
    """dL/dconj(Psi) (Ns, V, 12) -> dL/d(output channels) (V, 24*Ns): 2 Re, 2 Im."""
    g = np.asarray(g)
    Ns, V = g.shape[:2]
    r = np.stack([2.0 * g.real, 2.0 * g.imag], axis=-1)      # (Ns, V, 12, 2)
    return r.transpose(1, 0, 2, 3).reshape(V, Ns * 24)


def deficit_loss(Psi, targets, dims, b):
    """Mean deficit of the targets w.r.t. the block span of Psi, and dL/dconj(Psi).

    Per block: G = Psi^+ Psi, c_k = Psi^+ t_k, y_k = G^-1 c_k,
    ||(1 - P) t_k||^2 = ||t_k||^2 - c_k^+ y_k summed over the blocks.
    """
    P = to_blocks(np.asarray(Psi, dtype=np.complex128), dims, b)        # (Ns, Nb, n)
    T = to_blocks(np.asarray(targets, dtype=np.complex128), dims, b)    # (K, Nb, n)
    K = T.shape[0]
    tn2 = np.einsum("knj,knj->k", T.conj(), T).real                     # ||t_k||^2
    loss = 0.0
    grad = np.zeros_like(P)
    for blk in range(P.shape[1]):
        Pb = P[:, blk, :].T                                              # (n, Ns)
        Tb = T[:, blk, :].T                                              # (n, K)
        G = Pb.conj().T @ Pb
        C = Pb.conj().T @ Tb                                             # (Ns, K)
        Y = np.linalg.solve(G, C)
        proj = np.einsum("lk,lk->k", C.conj(), Y).real                  # ||P t_k||^2 on this block
        loss += np.sum((np.einsum("jk,jk->k", Tb.conj(), Tb).real - proj) / tn2)
        R = (Tb - Pb @ Y) / tn2                                          # (n, K)
        grad[:, blk, :] = (-(R @ Y.conj().T) / K).T
    from .dfl import from_blocks
    return loss / K, from_blocks(grad, dims, b)


def adam(theta, g, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t >= 1): returns the new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
