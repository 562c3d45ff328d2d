"""Learned start fields for the deflation subspace.

A 4-layer 4D convolutional network (3^4 kernels, periodic boundaries, SiLU
between layers; channels 96 -> 32 -> 32 -> 32 -> 24 Ns) maps the gauge field
and a noise field to Ns start fields for the subspace generation of
section 5.3. It is trained with Adam to minimise the block deficit
(eq. (3.15)) of low modes produced by the library's own inverse iteration
(eq. (5.1)); at setup time its fields replace the random start fields, and the
usual inverse-iteration steps, block Gram-Schmidt (eq. (4.2)) and
little-operator assembly (eq. (A.1)) follow.

This module only sequences C-ABI calls (include/dfl_net.h) and holds the
parameters in torch tensors: the features, every convolution forward and
backward, the loss and its gradient, and the Adam update run in the HIP
library.
"""
from __future__ import annotations

import numpy as np

from . import F64, binding

CHANNELS = (96, 32, 32, 32, 576)


class StartFieldNet:
    """Network parameters and Adam state on the device of ``solver``.

    ``weights``: list of (W (3,3,3,3,Cin,Cout), b (Cout,)) numpy arrays, e.g.
    ``latgen.net_init(CHANNELS, seed)``.
    """

    def __init__(self, solver, weights, channels=CHANNELS):
        self.S = solver
        torch = solver.torch
        self.torch = torch
        self.channels = tuple(int(c) for c in channels)
        if self.channels[0] != 96 or self.channels[-1] % 24:
            raise ValueError("the network reads 96 input channels and writes 24 per start field")
        self.Ns = self.channels[-1] // 24
        self.W, self.b, self.mW, self.vW, self.mb, self.vb = [], [], [], [], [], []
        for (W, b), cin, cout in zip(weights, self.channels[:-1], self.channels[1:]):
            if W.shape != (3, 3, 3, 3, cin, cout) or b.shape != (cout,):
                raise ValueError("weight shapes do not match the channels")
            self.W.append(torch.tensor(W.reshape(81, cin, cout), dtype=torch.float32, device="cuda"))
            self.b.append(torch.tensor(b, dtype=torch.float32, device="cuda"))
        for W, b in zip(self.W, self.b):
            self.mW.append(torch.zeros_like(W))
            self.vW.append(torch.zeros_like(W))
            self.mb.append(torch.zeros_like(b))
            self.vb.append(torch.zeros_like(b))
        self.t = 0
        self._cache = None

    def _planes(self, c):
        return self.torch.empty(c * self.S.V, dtype=self.torch.float32, device="cuda")

    def weights_numpy(self):
        out = []
        for W, b, cin, cout in zip(self.W, self.b, self.channels[:-1], self.channels[1:]):
            out.append((W.cpu().numpy().reshape(3, 3, 3, 3, cin, cout).astype(np.float64),
                        b.cpu().numpy().astype(np.float64)))
        return out

    def forward(self, noise, bf16=False):
        """Start fields (Ns native FP64 fields) for the solver's current gauge field.

        noise: (V, 24) canonical-order array or device tensor. bf16: run the
        convolutions with BF16 operands and FP32 sums (inference only; needs
        L3 % 32 == 0 and L2 % 4 == 0).
        """
        torch = self.torch
        if isinstance(noise, np.ndarray):
            noise = torch.tensor(np.ascontiguousarray(noise, dtype=np.float32), device="cuda")
        ctx = self.S.ctx
        x = self._planes(96)
        binding.net_features(ctx, noise, x)
        acts, zs = [x], []
        n = len(self.W)
        for i in range(n):
            cin, cout = self.channels[i], self.channels[i + 1]
            z = self._planes(cout)
            a = self._planes(cout) if i < n - 1 else None
            conv = binding.conv4d_forward_bf16 if bf16 else binding.conv4d_forward
            conv(ctx, acts[-1], cin, self.W[i], self.b[i], cout, z, a)
            zs.append(z)
            acts.append(a if a is not None else z)
        fields = self.S.field(self.Ns, F64)
        binding.net_outputs_to_fields(ctx, acts[-1], self.Ns, fields)
        self._cache = (acts, zs)
        return fields

    def backward(self, grad_fields):
        """Parameter gradients from dL/dconj(fields) of the last forward()."""
        acts, zs = self._cache
        ctx = self.S.ctx
        n = len(self.W)
        g = self._planes(self.channels[-1])
        binding.net_fields_grad_to_outputs(ctx, grad_fields, self.Ns, g)
        grads = [None] * n
        for i in range(n - 1, -1, -1):
            cin, cout = self.channels[i], self.channels[i + 1]
            dW = self.torch.empty_like(self.W[i])
            db = self.torch.empty_like(self.b[i])
            din = self._planes(cin) if i > 0 else None
            binding.conv4d_backward(ctx, acts[i], cin, self.W[i], cout, g, dW, db, din, zs[i - 1] if i > 0 else None)
            grads[i] = (dW, db)
            g = din
        return grads

    def loss(self, fields, targets, K, want_grad=True):
        grad = self.S.field(self.Ns, F64) if want_grad else None
        val = binding.deficit_loss(self.S.ctx, fields, self.Ns, targets, K, grad)
        return val, grad

    def step(self, grads, lr=1e-3):
        self.t += 1
        for i, (dW, db) in enumerate(grads):
            binding.adam_update(self.S.ctx, self.W[i], dW, self.mW[i], self.vW[i], self.t, lr)
            binding.adam_update(self.S.ctx, self.b[i], db, self.mb[i], self.vb[i], self.t, lr)

    def train_step(self, noise, targets, K, lr=1e-3):
        fields = self.forward(noise)
        val, grad = self.loss(fields, targets, K)
        self.step(self.backward(grad), lr)
        return val


def make_targets(solver, init_fields, steps):
    """Inverse-iteration low modes (eq. (5.1)) of the solver's gauge field from
    the given start fields (native FP64, modified in place and returned)."""
    n = init_fields.numel() // (12 * solver.V)
    binding.dfl_inverse_iteration(solver.ctx, init_fields, n, steps)
    return init_fields
