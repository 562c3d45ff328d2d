"""Seeded synthetic inputs for the Wilson-Dirac solver: gauge links, sources, init fields.

This module produces data only. It holds none of the solver's arithmetic (no Dirac
operator, no projector, no Krylov step) and is the one piece of code that both the
FP64 CPU oracle and the HIP path consume, so that both see identical inputs.

Canonical layout (shared by every consumer):

* lattice dims ``(L0, L1, L2, L3)``, ``x0`` slowest; site index
  ``s = ((x0*L1 + x1)*L2 + x2)*L3 + x3``;
* quark field: complex128 array of shape ``(V, 12)``, component ``3*alpha + a``
  for spin ``alpha`` in 0..3 and colour ``a`` in 0..2 (the paper's quark fields
  carry a Dirac and a colour index, section 4.3);
* gauge field: complex128 array of shape ``(V, 4, 3, 3)``; ``U[s, mu]`` is the
  SU(3) link from ``x`` to ``x + mu_hat`` with ``U[s, mu, a, b]`` row ``a``,
  column ``b``.

The paper measures on two-flavour QCD ensembles (section 2.1) that are not
available; these generators stand in for them with fields of the same shapes:

* links ``U = exp(i*eps*H)``, ``H = sum_a h_a lambda_a / 2`` with ``h_a`` i.i.d.
  standard normal and ``lambda_a`` the Gell-Mann matrices (traceless Hermitian,
  so ``det U = 1``); ``eps`` controls the roughness of the field;
* Gaussian sources with real and imaginary parts i.i.d. N(0, 1);
* point sources ``delta_{x,0} delta_{c,j}``;
* Gaussian random start fields for the inverse-iteration setup (section 5.3);
  the random numbers the method draws are generated here and passed in;
* the noise channels and the initial weights of the start-field network
  (per-site Gaussian noise; weights Gaussian with variance 1/(81 C_in), zero
  biases).

All draws use ``numpy.random.default_rng(seed)`` (PCG64) in the order stated in
each function, so a seed fixes the array bit for bit.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "NET_CHANNELS", "net_noise", "net_init",
    "gell_mann",
    "volume",
    "make_links",
    "make_source",
    "point_sources",
    "make_init_fields",
    "random_gauge_transform",
    "random_field",
]


def volume(dims) -> int:
    d = [int(v) for v in dims]
    if len(d) != 4 or min(d) < 1:
        raise ValueError(f"dims must be four positive ints, got {dims!r}")
    return d[0] * d[1] * d[2] * d[3]


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3) complex128."""
    g = np.zeros((8, 3, 3), dtype=np.complex128)
    g[0][0, 1] = g[0][1, 0] = 1
    g[1][0, 1] = -1j
    g[1][1, 0] = 1j
    g[2][0, 0] = 1
    g[2][1, 1] = -1
    g[3][0, 2] = g[3][2, 0] = 1
    g[4][0, 2] = -1j
    g[4][2, 0] = 1j
    g[5][1, 2] = g[5][2, 1] = 1
    g[6][1, 2] = -1j
    g[6][2, 1] = 1j
    g[7][0, 0] = g[7][1, 1] = 1 / np.sqrt(3)
    g[7][2, 2] = -2 / np.sqrt(3)
    return g


def _expi_hermitian(H: np.ndarray, eps: float, chunk: int = 1 << 20) -> np.ndarray:
    """exp(i*eps*H) for a stack of Hermitian 3x3 matrices, via eigh (chunked)."""
    out = np.empty_like(H)
    flat_in = H.reshape(-1, 3, 3)
    flat_out = out.reshape(-1, 3, 3)
    for s in range(0, flat_in.shape[0], chunk):
        w, v = np.linalg.eigh(flat_in[s:s + chunk])
        ph = np.exp(1j * eps * w)
        flat_out[s:s + chunk] = np.einsum("nij,nj,nkj->nik", v, ph, v.conj())
    return out


def make_links(dims, eps: float, seed: int) -> np.ndarray:
    """Gauge field U_mu(x) = exp(i*eps*H_mu(x)), shape (V, 4, 3, 3) complex128.

    Draw order: ``h = rng.standard_normal((V, 4, 8))`` in canonical site order,
    then direction mu, then Gell-Mann index a.
    """
    V = volume(dims)
    if float(eps) == 0.0:
        # the free field, exactly (exp(0) = 1 without eigh round-off)
        return np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((V, 4, 8))
    H = np.einsum("sma,aij->smij", h, gell_mann() / 2.0)
    return _expi_hermitian(H, float(eps))


def make_source(dims, seed: int) -> np.ndarray:
    """Gaussian quark field, shape (V, 12) complex128; draw ``standard_normal((V, 12, 2))``."""
    V = volume(dims)
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((V, 12, 2))
    return z[..., 0] + 1j * z[..., 1]


def random_field(dims, seed: int, n: int | None = None) -> np.ndarray:
    """One (``n=None``) or ``n`` Gaussian quark fields; same recipe as make_source."""
    V = volume(dims)
    rng = np.random.default_rng(seed)
    if n is None:
        z = rng.standard_normal((V, 12, 2))
    else:
        z = rng.standard_normal((n, V, 12, 2))
    return z[..., 0] + 1j * z[..., 1]


def point_sources(dims, components) -> np.ndarray:
    """Point sources delta_{x,0} delta_{c,j} for each j in ``components``: (n, V, 12)."""
    V = volume(dims)
    comps = list(components)
    out = np.zeros((len(comps), V, 12), dtype=np.complex128)
    for i, j in enumerate(comps):
        if not 0 <= j < 12:
            raise ValueError("spin-colour component must be in 0..11")
        out[i, 0, j] = 1.0
    return out


def make_init_fields(dims, ns: int, seed: int) -> np.ndarray:
    """Random start fields for inverse iteration: (ns, V, 12) complex128.

    Draw ``standard_normal((ns, V, 12, 2))``; the fields are not normalised here
    (normalisation is a step of the method).
    """
    return random_field(dims, seed, n=int(ns))


def random_gauge_transform(dims, seed: int) -> np.ndarray:
    """Random SU(3) matrix per site, shape (V, 3, 3): exp(i*H) with the link recipe (eps=1)."""
    V = volume(dims)
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((V, 8))
    H = np.einsum("sa,aij->sij", h, gell_mann() / 2.0)
    return _expi_hermitian(H, 1.0)


NET_CHANNELS = (96, 32, 32, 32, 576)  # 72 link + 24 noise inputs; Ns = 24 complex-12 outputs


def net_noise(dims, seed: int, n: int = 24) -> np.ndarray:
    """Per-site Gaussian noise channels of the start-field network: (V, n) float64,
    drawn as standard_normal((V, n))."""
    return np.random.default_rng(seed).standard_normal((volume(dims), n))


def net_init(channels, seed: int) -> list:
    """Initial weights of the 3^4 convolutions: [(W (3,3,3,3,Cin,Cout), b (Cout,)), ...].

    W is drawn layer by layer as standard_normal((3,3,3,3,Cin,Cout)) times
    sqrt(1/(81*Cin)); biases are zero.
    """
    rng = np.random.default_rng(seed)
    out = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        W = rng.standard_normal((3, 3, 3, 3, cin, cout)) * np.sqrt(1.0 / (81 * cin))
        out.append((W, np.zeros(cout)))
    return out

