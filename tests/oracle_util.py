"""Small helpers for the oracle pins (dense matrices from matrix-free operators)."""
import numpy as np


def dense_from(apply, V: int) -> np.ndarray:
    """Dense matrix of a linear map on (V, 12) fields, column j = apply(e_j)."""
    n = V * 12
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((V, 12), dtype=np.complex128)
    for j in range(n):
        e.reshape(-1)[j] = 1.0
        M[:, j] = np.asarray(apply(e)).reshape(-1)
        e.reshape(-1)[j] = 0.0
    return M


def gamma5_apply(psi):
    """gamma_5 = diag(1, 1, -1, -1) in spin (the chiral basis) on a (V, 12) field."""
    out = np.array(psi, dtype=np.complex128).reshape(-1, 4, 3)
    out[:, 2:, :] *= -1
    return out.reshape(-1, 12)


def site_coords(dims):
    """Coordinates (V, 4) of every site in canonical order."""
    return np.stack(np.unravel_index(np.arange(int(np.prod(dims))), dims), axis=1)


def gauge_transform(U, Lam, dims):
    """U_mu(x) -> Lam(x) U_mu(x) Lam(x+mu)^dagger."""
    d = list(dims)
    V = int(np.prod(d))
    x = site_coords(d)
    out = np.empty_like(U)
    for mu in range(4):
        y = x.copy()
        y[:, mu] = (y[:, mu] + 1) % d[mu]
        nb = np.ravel_multi_index(tuple(y.T), d)
        out[:, mu] = Lam @ U[:, mu] @ Lam[nb].conj().transpose(0, 2, 1)
    assert out.shape == (V, 4, 3, 3)
    return out


def colour_rotate(Lam, psi):
    """psi(x) -> Lam(x) psi(x) (colour index), (V, 12) field."""
    p = np.asarray(psi).reshape(-1, 4, 3)
    return np.einsum("sab,sjb->sja", Lam, p).reshape(-1, 12)
