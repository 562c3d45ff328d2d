"""MI355X (gfx950) deflated, Schwarz-preconditioned GCR solver for the Wilson-Dirac equation.

Implements the solver of M. Luescher, "Local coherence and deflation of the
low quark modes in lattice QCD": flexible GCR (section 6.2) on the deflated,
SAP-preconditioned equation (6.2), with a block-projected subspace (sections
4.1-4.2) from inverse iteration (eq. (5.1)) and the little Dirac operator of
eq. (A.1). All arithmetic runs in the HIP library ``libdfl.so`` (C ABI in
include/dfl.h); ``binding`` marshals arguments to it, and ``Solver`` holds a
context plus torch device tensors (torch provides device memory and streams).
"""
from __future__ import annotations

import numpy as np

from . import binding
from .binding import (F64, F32, BF16, PROJ_PL, PROJ_PR, PROJ_P, PROJ_COARSE, SOLVER_GCR, SOLVER_SAP_GCR,
                      SOLVER_DFL_SAP_GCR, DflError, default_params)

__all__ = ["binding", "Solver", "F64", "F32", "BF16", "PROJ_PL", "PROJ_PR", "PROJ_P", "PROJ_COARSE",
           "SOLVER_GCR", "SOLVER_SAP_GCR", "SOLVER_DFL_SAP_GCR", "DflError", "default_params"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the HIP solver needs a visible GPU (no CPU fallback)")
    return torch


class Solver:
    """A solver context on the current device and torch stream.

    Canonical arrays (numpy or torch) follow latgen's layout: quark fields
    (nrhs, V, 12) complex128, gauge field (V, 4, 3, 3) complex128. Native
    fields are torch tensors of complex128 (F64) or complex64 (F32) holding
    nrhs * 12 * V entries in the library's block-major plane layout.
    """

    def __init__(self, dims, **params):
        torch = _torch()
        self.torch = torch
        self.params = default_params(dims=dims, **params)
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.stream = torch.cuda.current_stream()
        self.ctx = binding.dfl_create(self.params, self.stream.cuda_stream)
        self.Nb = binding.dfl_num_blocks(self.ctx)
        self.Ns = int(self.params.Ns)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            binding.dfl_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- buffers
    def _dev(self, a, dtype):
        t = self.torch
        if isinstance(a, np.ndarray):
            return t.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to("cuda")
        return a.contiguous()

    def field(self, nrhs=1, prec=F64):
        dt = self.torch.complex128 if prec == F64 else self.torch.complex64
        return self.torch.empty(nrhs * 12 * self.V, dtype=dt, device="cuda")

    def little_vector(self, nrhs=1, prec=F64):
        dt = self.torch.complex128 if prec == F64 else self.torch.complex64
        return self.torch.empty(nrhs * self.Nb * self.Ns, dtype=dt, device="cuda")

    # ---------------------------------------------------------------- calls
    def set_gauge(self, U):
        Ud = self._dev(U, np.complex128)
        if Ud.numel() != self.V * 36:
            raise ValueError("gauge field must have V*4*3*3 entries")
        binding.dfl_set_gauge(self.ctx, Ud)
        self.stream.synchronize()

    def set_mass(self, m0):
        binding.dfl_set_mass(self.ctx, m0)

    def pack(self, canon, prec=F64):
        c = self._dev(canon, np.complex128)
        nrhs = c.numel() // (12 * self.V)
        if nrhs * 12 * self.V != c.numel():
            raise ValueError("canonical field size must be a multiple of 12 V")
        out = self.field(nrhs, prec)
        binding.dfl_pack(self.ctx, c, out, nrhs, prec)
        return out

    def unpack(self, native, prec=F64):
        per = 12 * self.V
        nrhs = native.numel() // per
        out = self.torch.empty(nrhs * per, dtype=self.torch.complex128, device="cuda")
        binding.dfl_unpack(self.ctx, native, out, nrhs, prec)
        self.stream.synchronize()
        return out.cpu().numpy().reshape(nrhs, self.V, 12)

    def dirac(self, psi, prec=F64):
        nrhs = psi.numel() // (12 * self.V)
        out = self.field(nrhs, prec)
        binding.dirac_apply(self.ctx, psi, out, nrhs, prec)
        return out

    def sap(self, rho):
        nrhs = rho.numel() // (12 * self.V)
        out = self.field(nrhs, F64)
        binding.sap_precond(self.ctx, rho, out, nrhs)
        return out

    def setup(self, init_native):
        binding.dfl_setup(self.ctx, init_native, self.Ns)

    def basis(self):
        out = self.field(self.Ns, F64)
        binding.dfl_get_basis(self.ctx, out)
        return out

    def little_operator(self):
        A = self.torch.empty(self.Nb * 9 * self.Ns * self.Ns, dtype=self.torch.complex128, device="cuda")
        binding.dfl_get_little(self.ctx, A)
        self.stream.synchronize()
        return A.cpu().numpy().reshape(self.Nb, 9, self.Ns, self.Ns)

    def little_apply(self, v, prec=F64):
        nrhs = v.numel() // (self.Nb * self.Ns)
        w = self.little_vector(nrhs, prec)
        binding.little_dirac_apply(self.ctx, v, w, nrhs, prec)
        return w

    def little_solve(self, w, tol):
        v = self.little_vector(1, F64)
        code, it = binding.little_solve(self.ctx, w, v, tol)
        return v, code, it

    def project(self, which, y):
        nrhs = y.numel() // (12 * self.V)
        out = self.field(nrhs, F64)
        binding.deflate_project(self.ctx, which, y, out, nrhs)
        return out

    def use_graphs(self, on=True):
        binding.dfl_use_graphs(self.ctx, on)

    def solve(self, eta):
        nrhs = eta.numel() // (12 * self.V)
        psi = self.field(nrhs, F64)
        info = binding.solve(self.ctx, eta, psi, nrhs)
        return psi, info
