"""Pins of the oracle's O(a)-improvement term and antiperiodic time (section 2.1).

The paper runs O(a)-improved Wilson quarks (a clover coefficient csw) and does
not print the operator; the oracle takes the standard Sheikholeslami-Wohlert
form csw (i/4) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x), Fhat from the four
plaquette "leaves" around x. What fixes it independently of the oracle:

* an abelian background with constant field strength f in one (mu, nu) plane
  (a U(1) field in the lambda_3 direction, twisted so that every plaquette of
  the periodic lattice carries the phase f): Fhat_{mu nu} = i sin(f)
  diag(1, -1, 0) exactly, all other planes vanish, so the clover matrix is
  -(csw/2) sin(f) sigma_{mu nu} x diag(1, -1, 0) at every site;
* the clover matrix is hermitian, commutes with gamma_5, vanishes on the free
  field and transforms as Lambda(x) C(x) Lambda(x)^dagger under gauge
  transformations;
* the whole operator keeps gamma_5-hermiticity and gauge covariance;
* antiperiodic time: free plane waves with p_0 = 2 pi (n_0 + 1/2) / L_0 are
  eigenvectors with the free-field symbol, and the dense free spectrum is the
  closed form at those momenta;
* D = (direct sum of D_Lambda) + block-crossing hops still holds, and SAP
  with the clover term converges to D^{-1} at heavy mass.
"""
import numpy as np
import pytest

import latgen
import oracle
from oracle_util import dense_from, gamma5_apply, gauge_transform, colour_rotate, site_coords

CSW = 1.90952


def abelian_background(dims, mu, nu, k):
    """U_rho(x) = diag(e^{i t}, e^{-i t}, 1) with t = theta_rho(x): every plaquette
    in the (mu, nu) plane has the phase f = 2 pi k / (L_mu L_nu)."""
    d = np.array(dims)
    x = site_coords(dims)
    f = 2 * np.pi * k / (d[mu] * d[nu])
    theta = np.zeros((len(x), 4))
    theta[:, nu] = f * x[:, mu]
    last = x[:, mu] == d[mu] - 1
    theta[last, mu] = -f * d[mu] * x[last, nu]
    U = np.zeros((len(x), 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = np.exp(1j * theta)
    U[:, :, 1, 1] = np.exp(-1j * theta)
    U[:, :, 2, 2] = 1.0
    return U, f


def sigma(mu, nu):
    g = oracle.gamma()
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])


@pytest.mark.parametrize("mu,nu", [(0, 1), (0, 3), (1, 2), (2, 3), (3, 1)])
def test_constant_abelian_field_closed_form(mu, nu):
    dims = (4, 3, 4, 2)
    U, f = abelian_background(dims, mu, nu, 1)
    # the background is what it claims: plaquette phase f in the (mu, nu) plane
    x = site_coords(dims)
    V = len(x)
    want = -(CSW / 2) * np.sin(f) * np.kron(sigma(mu, nu), np.diag([1.0, -1.0, 0.0]))
    for s in (0, 7, V // 2, V - 1):
        C = oracle.clover_site(U, dims, CSW, s)
        assert np.abs(C - want).max() < 1e-13
    # the operator adds exactly C(x) psi(x) to the Wilson operator
    psi = latgen.make_source(dims, 5)
    d = oracle.dirac(U, psi, -0.1, dims, csw=CSW) - oracle.dirac(U, psi, -0.1, dims)
    assert np.abs(d - psi @ want.T).max() < 1e-13


def test_clover_matrix_properties():
    dims = (4, 4, 2, 4)
    U = latgen.make_links(dims, 0.5, 301)
    g5 = np.kron(np.diag([1.0, 1, -1, -1]), np.eye(3))
    Lam = latgen.random_gauge_transform(dims, 302)
    Ug = gauge_transform(U, Lam, dims)
    free = latgen.make_links(dims, 0.0, 1)
    for s in (0, 13, 77):
        C = oracle.clover_site(U, dims, CSW, s)
        assert np.abs(C - C.conj().T).max() < 1e-14
        assert np.abs(C @ g5 - g5 @ C).max() < 1e-14
        assert np.abs(C).max() > 0.05
        L12 = np.kron(np.eye(4), Lam[s])
        assert np.abs(oracle.clover_site(Ug, dims, CSW, s) - L12 @ C @ L12.conj().T).max() < 1e-13
        assert np.abs(oracle.clover_site(free, dims, CSW, s)).max() == 0
        assert np.abs(oracle.clover_site(U, dims, 2 * CSW, s) - 2 * C).max() < 1e-14


@pytest.mark.parametrize("antiperiodic", [False, True])
def test_gamma5_hermiticity_and_covariance(antiperiodic):
    dims = (4, 4, 2, 2)
    kw = dict(csw=CSW, antiperiodic=antiperiodic)
    U = latgen.make_links(dims, 0.6, 311)
    phi = latgen.make_source(dims, 312)
    psi = latgen.make_source(dims, 313)
    m0 = -0.3
    lhs = np.vdot(phi, gamma5_apply(oracle.dirac(U, gamma5_apply(psi), m0, dims, **kw)))
    rhs = np.vdot(oracle.dirac(U, phi, m0, dims, **kw), psi)
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)
    Lam = latgen.random_gauge_transform(dims, 314)
    Ug = gauge_transform(U, Lam, dims)
    a = oracle.dirac(Ug, colour_rotate(Lam, psi), m0, dims, **kw)
    b = colour_rotate(Lam, oracle.dirac(U, psi, m0, dims, **kw))
    assert np.abs(a - b).max() < 1e-13


def test_antiperiodic_free_plane_waves_and_spectrum():
    dims = (4, 3, 2, 2)
    V = int(np.prod(dims))
    U = latgen.make_links(dims, 0.0, 1)
    g = oracle.gamma()
    x = site_coords(dims)
    m0 = -0.2
    rng = np.random.default_rng(3)
    for trial in range(4):
        n = np.array([rng.integers(0, L) for L in dims], dtype=float)
        n[0] += 0.5
        p = 2 * np.pi * n / np.array(dims)
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * (x @ p))
        psi = (phase[:, None, None] * u[None]).reshape(V, 12)
        Dp = (m0 + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(g[mu] * np.sin(p[mu]) for mu in range(4))
        want = (phase[:, None, None] * (Dp @ u)[None]).reshape(V, 12)
        assert np.abs(oracle.dirac(U, psi, m0, dims, antiperiodic=True) - want).max() < 1e-13
        # the periodic operator does not have this eigenvector
        assert np.abs(oracle.dirac(U, psi, m0, dims) - want).max() > 1e-2
    M = dense_from(lambda f: oracle.dirac(U, f, m0, dims, antiperiodic=True, csw=CSW), V)
    ev = np.linalg.eigvals(M)
    want = []
    for n in np.ndindex(*dims):
        q = np.array(n, dtype=float)
        q[0] += 0.5
        p = 2 * np.pi * q / np.array(dims)
        re = m0 + np.sum(1 - np.cos(p))
        im = np.sqrt(np.sum(np.sin(p) ** 2))
        want += [re + 1j * im] * 6 + [re - 1j * im] * 6
    key = lambda z: (round(z.real, 8), round(z.imag, 8))
    assert np.abs(np.array(sorted(ev, key=key)) - np.array(sorted(want, key=key))).max() < 1e-10


def test_block_decomposition_with_clover_and_antiperiodic_time():
    dims = (4, 4, 4, 8)
    b = (2, 2, 4, 4)
    U = latgen.make_links(dims, 0.4, 321)
    psi = latgen.make_source(dims, 322)
    m0 = -0.2
    kw = dict(csw=CSW, antiperiodic=True)
    full = oracle.dirac(U, psi, m0, dims, **kw)
    parts = oracle.dirac_blockdiag(U, psi, m0, dims, b, **kw)
    for mu in range(4):
        for s in (+1, -1):
            parts = parts + oracle.hop_cross(U, psi, dims, b, mu, s, antiperiodic=True)
    assert np.abs(parts - full).max() < 1e-13
    sites = np.array([0, 5, 77, 300, 511])
    assert np.abs(oracle.dirac_sites(U, psi, m0, dims, sites, **kw) - full[sites]).max() < 1e-14
    # the time-boundary sign sits on the x0 faces only
    d = full - oracle.dirac(U, psi, m0, dims, csw=CSW)
    x0 = site_coords(dims)[:, 0]
    inner = (x0 != 0) & (x0 != dims[0] - 1)
    assert np.abs(d[inner]).max() == 0 and np.abs(d[~inner]).max() > 0.1


def test_sap_with_clover_converges_to_inverse():
    dims = (4, 4, 4, 8)
    b = (2, 2, 2, 4)
    m0 = 0.5
    kw = dict(csw=CSW, antiperiodic=True)
    U = latgen.make_links(dims, 0.4, 331)
    rho = latgen.make_source(dims, 332)
    psi = oracle.sap(U, rho, m0, dims, b, 40, 30, **kw)
    r = rho - oracle.dirac(U, psi, m0, dims, **kw)
    assert np.linalg.norm(r) < 1e-10 * np.linalg.norm(rho)
    # the MR block solver runs on the block operator with the clover term
    blk = 3
    x = oracle.mr_block(U, rho, m0, dims, b, blk, 200, **kw)
    res = rho - oracle.dirac_blockdiag(U, x, m0, dims, b, **kw)
    on = np.any(x != 0, axis=1)
    assert on.sum() == 2 * 2 * 2 * 4 and np.linalg.norm(res[on]) < 1e-11 * np.linalg.norm(rho[on])
