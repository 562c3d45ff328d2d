"""FP64 CPU oracle, numpy part (test infrastructure only; see the package docstring).

Fields use the canonical layout of ``latgen``: a quark field is ``(V, 12)``
complex128, the gauge field ``(V, 4, 3, 3)``. Blocks are rectangular, of shape
``b = (b0, b1, b2, b3)``, indexed lexicographically by their block coordinates
``n_mu = x_mu // b_mu`` (``n0`` slowest); sites inside a block are in
lexicographic order of ``x_mu % b_mu``. Little vectors have shape ``(Nb, Ns)``
with entry ``[Lambda, k]`` the coefficient of the basis field
``phi^Lambda_k``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "lib", "num_threads", "gamma", "dirac", "dirac_blockdiag", "hop_cross", "dirac_sites",
    "mr_block", "sap", "block_counts", "to_blocks", "from_blocks", "block_colours",
    "block_neighbour", "clover_site", "block_gram_schmidt", "restrict", "prolong", "proj_P",
    "little_operator", "little_apply", "little_dense", "little_solve", "little_gcr",
    "Deflation", "gcr", "inverse_iteration", "setup", "solve", "deficit", "dot", "norm",
    "LITTLE_DIRS",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_c_int4 = ctypes.c_int * 4


def lib():
    """Load liboracle.so, compiling it first only if it is not there."""
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from .build import build_oracle
            build_oracle()
        L = ctypes.CDLL(path)
        vp = ctypes.c_void_p
        d, i = ctypes.c_double, ctypes.c_int
        L.orc_dirac.argtypes = [vp, d, d, i, vp, vp, vp]
        L.orc_dirac_blockdiag.argtypes = [vp, vp, d, d, i, vp, vp, vp]
        L.orc_hop_cross.argtypes = [vp, vp, i, vp, vp, vp, i, i]
        L.orc_dirac_sites.argtypes = [vp, d, d, i, vp, vp, vp, ctypes.c_long, vp]
        L.orc_mr_block.argtypes = [vp, vp, d, d, i, vp, ctypes.c_long, vp, i, vp]
        L.orc_sap.argtypes = [vp, vp, d, d, i, vp, vp, i, i, vp]
        L.orc_clover_site.argtypes = [vp, vp, d, ctypes.c_long, vp]
        L.orc_gamma.argtypes = [vp]
        L.orc_num_threads.restype = ctypes.c_int
        for f in (L.orc_dirac, L.orc_dirac_blockdiag, L.orc_hop_cross, L.orc_dirac_sites,
                  L.orc_mr_block, L.orc_sap, L.orc_gamma, L.orc_clover_site):
            f.restype = None
        _LIB = L
    return _LIB


def num_threads() -> int:
    """OpenMP threads the C part uses."""
    return int(lib().orc_num_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _cfield(a, V: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.size != V * 12:
        raise ValueError(f"quark field must hold V*12 = {V * 12} entries, got {a.size}")
    return a.reshape(V, 12)


def _cgauge(U, V: int) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.complex128)
    if U.size != V * 36:
        raise ValueError("gauge field must have shape (V, 4, 3, 3)")
    return U.reshape(V, 4, 3, 3)


def _dims(dims):
    d = [int(v) for v in dims]
    return d, d[0] * d[1] * d[2] * d[3]


def dot(u, v) -> complex:
    """(u, v) = sum conj(u) v, the scalar product of section 3.1."""
    return complex(np.vdot(u, v))


def norm(u) -> float:
    return float(np.sqrt(np.vdot(u, u).real))


def gamma() -> np.ndarray:
    """The four Euclidean gamma matrices used by the oracle, shape (4, 4, 4)."""
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    lib().orc_gamma(_ptr(g))
    return g


# --------------------------------------------------------------- operators

def _bc0(antiperiodic: bool) -> int:
    return -1 if antiperiodic else 1


def dirac(U, psi, m0: float, dims, *, csw: float = 0.0, antiperiodic: bool = False) -> np.ndarray:
    """D psi, eq. (3.9)'s operator: Wilson plus the clover term csw (i/4) sigma.F
    (section 2.1's O(a) improvement; csw = 0 is plain Wilson); periodic in
    space, periodic or antiperiodic in time (direction 0)."""
    d, V = _dims(dims)
    U = _cgauge(U, V)
    psi = _cfield(psi, V)
    out = np.empty_like(psi)
    lib().orc_dirac(_ptr(np.array(d, dtype=np.int32)), float(m0), float(csw), _bc0(antiperiodic), _ptr(U),
                    _ptr(psi), _ptr(out))
    return out


def dirac_blockdiag(U, psi, m0: float, dims, b, *, csw: float = 0.0, antiperiodic: bool = False) -> np.ndarray:
    """(direct sum of D_Lambda) psi: D with every hop across a block face dropped."""
    d, V = _dims(dims)
    U = _cgauge(U, V)
    psi = _cfield(psi, V)
    out = np.empty_like(psi)
    lib().orc_dirac_blockdiag(_ptr(np.array(d, dtype=np.int32)), _ptr(np.array(b, dtype=np.int32)),
                              float(m0), float(csw), _bc0(antiperiodic), _ptr(U), _ptr(psi), _ptr(out))
    return out


def hop_cross(U, psi, dims, b, mu: int, direction: int, *, antiperiodic: bool = False) -> np.ndarray:
    """The hop terms of D in direction mu (+1 forward, -1 backward) that cross a block face."""
    d, V = _dims(dims)
    U = _cgauge(U, V)
    psi = _cfield(psi, V)
    out = np.empty_like(psi)
    lib().orc_hop_cross(_ptr(np.array(d, dtype=np.int32)), _ptr(np.array(b, dtype=np.int32)),
                        _bc0(antiperiodic), _ptr(U), _ptr(psi), _ptr(out), int(mu), int(direction))
    return out


def dirac_sites(U, psi, m0: float, dims, sites, *, csw: float = 0.0, antiperiodic: bool = False) -> np.ndarray:
    """(D psi)(x) for the listed sites only, shape (len(sites), 12)."""
    d, V = _dims(dims)
    U = _cgauge(U, V)
    psi = _cfield(psi, V)
    s = np.ascontiguousarray(sites, dtype=np.int64)
    if s.size and (s.min() < 0 or s.max() >= V):
        raise ValueError("site index out of range")
    out = np.empty((s.size, 12), dtype=np.complex128)
    lib().orc_dirac_sites(_ptr(np.array(d, dtype=np.int32)), float(m0), float(csw), _bc0(antiperiodic), _ptr(U),
                          _ptr(psi), _ptr(s), s.size, _ptr(out))
    return out


def clover_site(U, dims, csw: float, site: int) -> np.ndarray:
    """The clover matrix csw (i/4) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x) of one site, (12, 12)
    in the spin-colour index 3 alpha + a."""
    d, V = _dims(dims)
    U = _cgauge(U, V)
    out = np.empty((12, 12), dtype=np.complex128)
    lib().orc_clover_site(_ptr(np.array(d, dtype=np.int32)), _ptr(U), float(csw), int(site), _ptr(out))
    return out


def mr_block(U, rhs, m0: float, dims, b, blk: int, nmr: int, *, csw: float = 0.0,
             antiperiodic: bool = False) -> np.ndarray:
    """nmr minimal-residual steps for D_Lambda x = rhs|_Lambda on block blk.

    Returns a full-size field that holds x on the block and zero elsewhere.
    """
    d, V = _dims(dims)
    U = _cgauge(U, V)
    rhs = _cfield(rhs, V)
    x = np.zeros_like(rhs)
    lib().orc_mr_block(_ptr(np.array(d, dtype=np.int32)), _ptr(np.array(b, dtype=np.int32)),
                       float(m0), float(csw), _bc0(antiperiodic), _ptr(U), int(blk), _ptr(rhs), int(nmr), _ptr(x))
    return x


def sap(U, rho, m0: float, dims, b, ncy: int, nmr: int, *, csw: float = 0.0, antiperiodic: bool = False) -> np.ndarray:
    """psi = M_sap rho: the Schwarz alternating procedure (preconditioner of eq. (6.2)).

    Reading (the paper defers the definition to its ref. on Schwarz
    preconditioning): zero start; ``ncy`` cycles; in each, the blocks of colour
    0 and then colour 1 are updated by ``nmr`` minimal-residual steps on the
    block operator D_Lambda applied to the current residual rho - D psi
    restricted to the block. The map is nonlinear in rho but M(c rho) = c M(rho).
    """
    d, V = _dims(dims)
    _check_blocks(d, b)
    U = _cgauge(U, V)
    rho = _cfield(rho, V)
    psi = np.empty_like(rho)
    lib().orc_sap(_ptr(np.array(d, dtype=np.int32)), _ptr(np.array(b, dtype=np.int32)),
                  float(m0), float(csw), _bc0(antiperiodic), _ptr(U), _ptr(rho), int(ncy), int(nmr), _ptr(psi))
    return psi


# ------------------------------------------------------------------ blocks

def _check_blocks(d, b):
    for mu in range(4):
        if b[mu] < 1 or d[mu] % b[mu]:
            raise ValueError(f"block shape {tuple(b)} does not divide lattice {tuple(d)}")


def block_counts(dims, b):
    """(blocks per direction, number of blocks Nb, sites per block Vb)."""
    d, _ = _dims(dims)
    _check_blocks(d, b)
    nb = [d[mu] // b[mu] for mu in range(4)]
    return nb, nb[0] * nb[1] * nb[2] * nb[3], b[0] * b[1] * b[2] * b[3]


def to_blocks(field, dims, b) -> np.ndarray:
    """Gather a field (..., V, 12) into blocks: (..., Nb, Vb*12) (the psi^Lambda of eq. (4.2))."""
    d, V = _dims(dims)
    nb, Nb, Vb = block_counts(d, b)
    f = np.asarray(field)
    lead = f.shape[:-2]
    f = f.reshape(lead + (nb[0], b[0], nb[1], b[1], nb[2], b[2], nb[3], b[3], 12))
    k = len(lead)
    perm = tuple(range(k)) + tuple(k + i for i in (0, 2, 4, 6, 1, 3, 5, 7, 8))
    return f.transpose(perm).reshape(lead + (Nb, Vb * 12))


def from_blocks(fb, dims, b) -> np.ndarray:
    """Inverse of to_blocks: (..., Nb, Vb*12) -> (..., V, 12)."""
    d, V = _dims(dims)
    nb, Nb, Vb = block_counts(d, b)
    f = np.asarray(fb)
    lead = f.shape[:-2]
    k = len(lead)
    f = f.reshape(lead + (nb[0], nb[1], nb[2], nb[3], b[0], b[1], b[2], b[3], 12))
    perm = tuple(range(k)) + tuple(k + i for i in (0, 4, 1, 5, 2, 6, 3, 7, 8))
    return f.transpose(perm).reshape(lead + (V, 12))


def block_colours(dims, b) -> np.ndarray:
    """Colour (sum of block coordinates mod 2) of every block."""
    nb, Nb, _ = block_counts(dims, b)
    n = np.indices(nb).reshape(4, -1)
    return (n.sum(axis=0) % 2).astype(np.int64)


def block_neighbour(dims, b, mu: int, step: int) -> np.ndarray:
    """Index of block Lambda + step*mu_hat for every block Lambda (periodic)."""
    nb, Nb, _ = block_counts(dims, b)
    n = np.indices(nb).reshape(4, -1)
    n[mu] = (n[mu] + step) % nb[mu]
    return np.ravel_multi_index(tuple(n), nb)


def block_gram_schmidt(fields, dims, b, rank_tol: float = 1e-10) -> np.ndarray:
    """Basis fields phi^Lambda_l from global fields psi_l, eq. (4.2) and section 4.2.

    Each psi_l is restricted to every block; on each block the restricted
    fields are orthonormalised by Gram-Schmidt in the order l = 1..Ns
    (modified form: v_l -= (phi_k, v_l) phi_k for k < l, then phi_l = v_l/||v_l||).
    Returns Ns full-volume fields (Ns, V, 12) whose restriction to block Lambda
    is phi^Lambda_l. Raises ValueError if a block loses rank
    (||v_l|| < rank_tol * ||psi_l^Lambda||).
    """
    f = np.asarray(fields, dtype=np.complex128)
    fb = to_blocks(f, dims, b)          # (Ns, Nb, n)
    Ns = fb.shape[0]
    phi = np.empty_like(fb)
    for l in range(Ns):
        v = fb[l].copy()
        for k in range(l):
            c = np.einsum("bi,bi->b", phi[k].conj(), v)
            v -= c[:, None] * phi[k]
        nv = np.sqrt(np.einsum("bi,bi->b", v.conj(), v).real)
        n0 = np.sqrt(np.einsum("bi,bi->b", fb[l].conj(), fb[l]).real)
        if np.any(nv <= rank_tol * n0) or np.any(n0 == 0):
            raise ValueError("block Gram-Schmidt: the restricted fields are linearly dependent")
        phi[l] = v / nv[:, None]
    return from_blocks(phi, dims, b)


def restrict(Phi, psi, dims, b) -> np.ndarray:
    """Little vector w[Lambda, k] = (phi^Lambda_k, psi), the scalar products of eq. (4.1)."""
    Pb = to_blocks(Phi, dims, b)               # (Ns, Nb, n)
    pb = to_blocks(np.asarray(psi).reshape(-1, 12), dims, b)   # (Nb, n)
    return np.einsum("kbi,bi->bk", Pb.conj(), pb)


def prolong(Phi, v, dims, b) -> np.ndarray:
    """Field sum_{Lambda,k} phi^Lambda_k(x) v[Lambda, k]."""
    Pb = to_blocks(Phi, dims, b)
    out = np.einsum("kbi,bk->bi", Pb, np.asarray(v).reshape(Pb.shape[1], Pb.shape[0]))
    return from_blocks(out, dims, b)


def proj_P(Phi, psi, dims, b) -> np.ndarray:
    """P psi of eq. (4.1)."""
    return prolong(Phi, restrict(Phi, psi, dims, b), dims, b)


def deficit(Phi, psi, dims, b) -> float:
    """epsilon = ||(1 - P) psi||^2 / ||psi||^2, eq. (3.15) for a normalised field."""
    r = np.asarray(psi).reshape(-1, 12) - proj_P(Phi, psi, dims, b)
    return norm(r) ** 2 / norm(psi) ** 2


# little operator: d = 0 self; d = 1 + 2*mu for Lambda+mu; d = 2 + 2*mu for Lambda-mu
LITTLE_DIRS = [(None, 0)] + [(mu, s) for mu in range(4) for s in (+1, -1)]


def little_operator(U, Phi, m0: float, dims, b, *, csw: float = 0.0, antiperiodic: bool = False) -> np.ndarray:
    """Block matrices of the little Dirac operator, eq. (A.1): shape (Nb, 9, Ns, Ns).

    A[Lambda, 0][k, l] = (phi^Lambda_k, D phi^Lambda_l) = (phi^Lambda_k, D_Lambda phi^Lambda_l);
    A[Lambda, 1+2mu][k, l] = (phi^Lambda_k, D phi^{Lambda+mu}_l), which only the
    forward hops across the block's upper mu face reach; A[Lambda, 2+2mu] likewise
    for Lambda - mu. Blocks that are not equal or nearest neighbours do not couple
    (fig. 4). With two blocks along mu, Lambda+mu = Lambda-mu; the two parts are
    kept apart and both act on that one block.
    """
    Phi = np.asarray(Phi, dtype=np.complex128)
    Ns = Phi.shape[0]
    nb, Nb, Vb = block_counts(dims, b)
    Pb = to_blocks(Phi, dims, b)   # (Ns, Nb, n)
    A = np.zeros((Nb, 9, Ns, Ns), dtype=np.complex128)
    for l in range(Ns):
        Fl = Phi[l]
        y = to_blocks(dirac_blockdiag(U, Fl, m0, dims, b, csw=csw, antiperiodic=antiperiodic), dims, b)
        A[:, 0, :, l] = np.einsum("kbi,bi->bk", Pb.conj(), y)
        for d in range(1, 9):
            mu, s = LITTLE_DIRS[d]
            y = to_blocks(hop_cross(U, Fl, dims, b, mu, s, antiperiodic=antiperiodic), dims, b)
            A[:, d, :, l] = np.einsum("kbi,bi->bk", Pb.conj(), y)
    return A


def little_apply(A, v, dims, b) -> np.ndarray:
    """w = A v with the 9-point block stencil: w_L = sum_d A[L, d] v_{L+d}."""
    v = np.asarray(v).reshape(A.shape[0], A.shape[2])
    w = np.einsum("bkl,bl->bk", A[:, 0], v)
    for d in range(1, 9):
        mu, s = LITTLE_DIRS[d]
        w += np.einsum("bkl,bl->bk", A[:, d], v[block_neighbour(dims, b, mu, s)])
    return w


def little_dense(A, dims, b) -> np.ndarray:
    """The little operator as a dense (Nb*Ns) x (Nb*Ns) matrix, index Lambda*Ns + k."""
    Nb, _, Ns, _ = A.shape
    M = np.zeros((Nb * Ns, Nb * Ns), dtype=np.complex128)
    for d in range(9):
        if d == 0:
            nbr = np.arange(Nb)
        else:
            mu, s = LITTLE_DIRS[d]
            nbr = block_neighbour(dims, b, mu, s)
        for L in range(Nb):
            M[L * Ns:(L + 1) * Ns, nbr[L] * Ns:(nbr[L] + 1) * Ns] += A[L, d]
    return M


def little_gcr(A, w, dims, b, tol: float = 1e-13, nkv: int = 32, maxiter: int = 20000):
    """GCR for the little system A v = w (eq. (6.1)), to ||w - A v|| <= tol ||w||.

    Plain restarted GCR (the paper's appendix A.4 uses GCR for this system).
    Returns (v, iterations).
    """
    w = np.asarray(w, dtype=np.complex128).reshape(A.shape[0], A.shape[2])
    app = lambda x: little_apply(A, x, dims, b)
    v, it, _ = gcr(app, w, tol=tol, nkv=nkv, maxiter=maxiter)
    return v, it


def little_solve(A, w, dims, b, tol: float = 1e-13):
    """v = A^{-1} w: dense LU for N <= 6144, else little_gcr to ``tol``."""
    Nb, _, Ns, _ = A.shape
    w = np.asarray(w, dtype=np.complex128).reshape(Nb, Ns)
    if Nb * Ns <= 6144:
        M = little_dense(A, dims, b)
        return np.linalg.solve(M, w.reshape(-1)).reshape(Nb, Ns)
    return little_gcr(A, w, dims, b, tol=tol)[0]


class Deflation:
    """Deflation projectors of section 3.1 for a block subspace (Phi, A).

    coarse(y) = Phi A^{-1} Phi^dagger y; PL(y) = y - D coarse(y) (eq. (3.3));
    PR(y) = y - coarse(D y) (eq. (3.4)). Little solves are exact (dense LU) or
    to ``little_tol``.
    """

    def __init__(self, U, Phi, A, m0, dims, b, little_tol: float = 1e-13, *, csw: float = 0.0,
                 antiperiodic: bool = False):
        self.U, self.Phi, self.A = U, np.asarray(Phi), A
        self.csw, self.antiperiodic = float(csw), bool(antiperiodic)
        self.m0, self.dims, self.b = float(m0), list(dims), list(b)
        self.little_tol = little_tol
        Nb, _, Ns, _ = A.shape
        self._lu = None
        if Nb * Ns <= 6144:
            import scipy.linalg
            self._lu = scipy.linalg.lu_factor(little_dense(A, dims, b))

    def little_inverse(self, w):
        if self._lu is not None:
            import scipy.linalg
            return scipy.linalg.lu_solve(self._lu, np.asarray(w).reshape(-1)).reshape(self.A.shape[0], -1)
        return little_gcr(self.A, w, self.dims, self.b, tol=self.little_tol)[0]

    def D(self, psi):
        return dirac(self.U, psi, self.m0, self.dims, csw=self.csw, antiperiodic=self.antiperiodic)

    def coarse(self, y):
        return prolong(self.Phi, self.little_inverse(restrict(self.Phi, y, self.dims, self.b)),
                       self.dims, self.b)

    def PL(self, y):
        return np.asarray(y).reshape(-1, 12) - self.D(self.coarse(y))

    def PR(self, y):
        return np.asarray(y).reshape(-1, 12) - self.coarse(self.D(y))

    def P(self, y):
        return proj_P(self.Phi, y, self.dims, self.b)


# ------------------------------------------------------------------- solvers

def gcr(apply_op, eta, precond=None, project=None, tol: float = 1e-10, nkv: int = 16,
        maxiter: int = 1000, history=None):
    """Flexible restarted GCR (section 6.2) for op(psi) = eta, optionally deflated.

    With ``project`` = P_L this solves the deflated system P_L D chi = P_L eta of
    eq. (3.11) preconditioned on the right as in eq. (6.2); without it, the plain
    system. Each step extends the Krylov space by xi_k = M rho (M = ``precond``,
    identity if None), computes chi_k = P_L D xi_k, orthogonalises it against the
    earlier chi_j (modified Gram-Schmidt), normalises it and removes its
    component from the residue rho. After nkv steps (or convergence) the
    coefficients alpha solve the triangular system, psi += sum alpha_k xi_k,
    and the residue is recomputed from scratch, rho = P_L (eta - D psi)
    (appendix A.5). Stops when ||rho|| <= tol ||eta||.

    Returns (psi, iterations, converged).
    """
    eta = np.asarray(eta, dtype=np.complex128)
    shape = eta.shape
    M = precond if precond is not None else (lambda r: r.copy())
    Pj = project if project is not None else (lambda r: r)
    eta_norm = norm(eta)
    psi = np.zeros_like(eta)
    if eta_norm == 0.0:
        return psi, 0, True
    rho = Pj(eta).reshape(shape)
    it = 0
    while True:
        rn = norm(rho)
        if history is not None:
            history.append(rn / eta_norm)
        if rn <= tol * eta_norm:
            return psi, it, True
        if it >= maxiter:
            return psi, it, False
        xis, chis = [], []
        a = np.zeros((nkv, nkv), dtype=np.complex128)
        bk = np.zeros(nkv)
        c = np.zeros(nkv, dtype=np.complex128)
        k = 0
        while k < nkv and it < maxiter:
            xi = M(rho).reshape(shape)
            chi = Pj(apply_op(xi)).reshape(shape).copy()
            for j in range(k):
                a[j, k] = dot(chis[j], chi)
                chi -= a[j, k] * chis[j]
            bk[k] = norm(chi)
            chi /= bk[k]
            c[k] = dot(chi, rho)
            rho = rho - c[k] * chi
            xis.append(xi)
            chis.append(chi)
            k += 1
            it += 1
            if history is not None:
                history.append(norm(rho) / eta_norm)
            if norm(rho) <= tol * eta_norm:
                break
        alpha = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            alpha[i] = (c[i] - np.dot(a[i, i + 1:k], alpha[i + 1:k])) / bk[i]
        for i in range(k):
            psi = psi + alpha[i] * xis[i]
        rho = Pj(eta - apply_op(psi)).reshape(shape)


def inverse_iteration(U, init, m0: float, dims, sap_block, ncy: int, nmr: int, n_iter: int, *, csw: float = 0.0,
                      antiperiodic: bool = False, n_boot: int = 0, dfl_block=None):
    """Relaxed inverse iteration of eq. (5.1): psi_l <- "D^-1" psi_l, normalised.

    The start fields are normalised first; each step applies an approximate
    inverse of D to every field and normalises it again. No orthogonalisation
    between fields (the block Gram-Schmidt follows).

    The approximate inverse is one Schwarz procedure M_sap (ncy cycles), as
    section 5.3 proposes. With n_boot > 0 the last n_boot steps are
    bootstrapped (the last paragraph of section 5.3): before such a step the
    current fields span a deflation subspace (eq. (4.2) on blocks dfl_block,
    little operator eq. (A.1) at this mass), and the step solves D chi = psi_l
    with it the way section 6 does, stopped after the preconditioner: the
    deflated equation P_L D chi = P_L psi (eq. (3.11)) is solved approximately
    by chi = M_sap P_L psi, and the solution is completed by eq. (3.10),
    psi <- P_R chi + Phi A^-1 Phi^dagger psi. (With M_sap = D^-1 this is D^-1 psi
    exactly, since P_R D^-1 P_L = D^-1 - Phi A^-1 Phi^dagger.)
    """
    n_iter, n_boot = int(n_iter), int(n_boot)
    if not 0 <= n_boot <= n_iter:
        raise ValueError("n_boot must lie in 0..n_iter")
    if n_boot and dfl_block is None:
        raise ValueError("a bootstrapped step needs the deflation block shape")
    kw = dict(csw=csw, antiperiodic=antiperiodic)
    fields = [np.asarray(f, dtype=np.complex128).reshape(-1, 12) for f in init]
    fields = [f / norm(f) for f in fields]
    for step in range(n_iter):
        if step < n_iter - n_boot:
            fields = [sap(U, f, m0, dims, sap_block, ncy, nmr, **kw) for f in fields]
        else:
            Phi = block_gram_schmidt(np.stack(fields), dims, dfl_block)
            A = little_operator(U, Phi, m0, dims, dfl_block, **kw)
            dfl = Deflation(U, Phi, A, m0, dims, dfl_block, **kw)
            fields = [dfl.PR(sap(U, dfl.PL(f), m0, dims, sap_block, ncy, nmr, **kw)) + dfl.coarse(f)
                      for f in fields]
        fields = [f / norm(f) for f in fields]
    return np.stack(fields)


def setup(U, init, m0: float, dims, sap_block, dfl_block, ncy: int, nmr: int, n_iter: int, *, csw: float = 0.0,
          antiperiodic: bool = False, n_boot: int = 0):
    """Subspace generation (section 5.3) + eq. (4.2) + eq. (A.1): returns (Phi, A)."""
    fields = inverse_iteration(U, init, m0, dims, sap_block, ncy, nmr, n_iter, csw=csw, antiperiodic=antiperiodic,
                               n_boot=n_boot, dfl_block=dfl_block)
    Phi = block_gram_schmidt(fields, dims, dfl_block)
    A = little_operator(U, Phi, m0, dims, dfl_block, csw=csw, antiperiodic=antiperiodic)
    return Phi, A


def solve(U, eta, m0: float, dims, *, sap_block=None, ncy=5, nmr=4, dfl=None,
          tol: float = 1e-10, nkv: int = 16, maxiter: int = 1000, history=None, csw: float = 0.0,
          antiperiodic: bool = False):
    """Solve D psi = eta (eq. (3.9)) to ||eta - D psi|| <= tol ||eta||.

    dfl = Deflation or None; sap_block = SAP block shape or None (no
    preconditioner). With deflation this is DFL+SAP+GCR: GCR on eq. (6.2) and
    the final solution of eq. (3.10), psi = psi_acc + Phi A^{-1} Phi^dagger (eta - D psi_acc),
    i.e. P_R applied to the GCR iterate plus the coarse part.
    Returns (psi, iterations, converged).
    """
    op = lambda x: dirac(U, x, m0, dims, csw=csw, antiperiodic=antiperiodic)
    M = None
    if sap_block is not None:
        M = lambda r: sap(U, r, m0, dims, sap_block, ncy, nmr, csw=csw, antiperiodic=antiperiodic)
    Pj = dfl.PL if dfl is not None else None
    psi, it, ok = gcr(op, eta, precond=M, project=Pj, tol=tol, nkv=nkv, maxiter=maxiter,
                      history=history)
    if dfl is not None:
        eta2 = np.asarray(eta).reshape(-1, 12)
        psi = psi + dfl.coarse(eta2 - op(psi))
    return psi, it, ok
