"""Pins of the oracle's Dirac operator against facts that do not come from the oracle.

* Clifford algebra and gamma_5 of the gamma basis;
* free field (U = 1): plane waves u e^{ipx} are mapped to D(p) u e^{ipx} with
  D(p) = m0 + sum_mu (1 - cos p_mu) + i sum_mu gamma_mu sin p_mu, and the dense
  spectrum is m0 + sum (1 - cos p) +- i (sum sin^2 p)^{1/2}, each 6-fold;
* gamma_5-hermiticity gamma_5 D gamma_5 = D^dagger on a random gauge field;
* gauge covariance D[U^Lambda] Lambda psi = Lambda D[U] psi;
* decomposition D = (direct sum of D_Lambda) + (block-crossing hops).
"""
import numpy as np
import pytest

import latgen
import oracle
from oracle_util import dense_from, gamma5_apply, gauge_transform, colour_rotate, site_coords


def test_clifford_algebra():
    g = oracle.gamma()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.abs(ac - 2 * (mu == nu) * np.eye(4)).max() == 0
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    assert np.abs(g5 - np.diag([1, 1, -1, -1])).max() == 0


@pytest.mark.parametrize("dims", [(4, 3, 2, 5), (8, 8, 8, 8)])
def test_free_plane_waves(dims):
    rng = np.random.default_rng(0)
    V = int(np.prod(dims))
    U = latgen.make_links(dims, 0.0, 1)
    g = oracle.gamma()
    x = site_coords(dims)
    m0 = -0.2
    for trial in range(4):
        n = np.array([rng.integers(0, L) for L in dims])
        p = 2 * np.pi * n / np.array(dims)
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * (x @ p))
        psi = (phase[:, None, None] * u[None]).reshape(V, 12)
        Dp = (m0 + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(g[mu] * np.sin(p[mu]) for mu in range(4))
        want = (phase[:, None, None] * (Dp @ u)[None]).reshape(V, 12)
        got = oracle.dirac(U, psi, m0, dims)
        assert np.abs(got - want).max() < 1e-13


def test_free_dense_spectrum():
    dims = (2, 3, 4, 4)
    V = int(np.prod(dims))
    m0 = -0.2
    U = latgen.make_links(dims, 0.0, 1)
    M = dense_from(lambda f: oracle.dirac(U, f, m0, dims), V)
    ev = np.linalg.eigvals(M)
    want = []
    for n in np.ndindex(*dims):
        p = 2 * np.pi * np.array(n) / np.array(dims)
        re = m0 + np.sum(1 - np.cos(p))
        im = np.sqrt(np.sum(np.sin(p) ** 2))
        want += [re + 1j * im] * 6 + [re - 1j * im] * 6
    key = lambda z: (round(z.real, 8), round(z.imag, 8))
    a = sorted(ev, key=key)
    b = sorted(want, key=key)
    assert np.abs(np.array(a) - np.array(b)).max() < 1e-10


def test_gamma5_hermiticity():
    dims = (4, 4, 2, 2)
    U = latgen.make_links(dims, 0.6, 21)
    phi = latgen.make_source(dims, 22)
    psi = latgen.make_source(dims, 23)
    m0 = -0.3
    lhs = np.vdot(phi, gamma5_apply(oracle.dirac(U, gamma5_apply(psi), m0, dims)))
    rhs = np.vdot(oracle.dirac(U, phi, m0, dims), psi)
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)
    # and the operator is not hermitian itself
    assert abs(np.vdot(phi, oracle.dirac(U, psi, m0, dims)) - rhs) > 1e-3


def test_gauge_covariance():
    dims = (4, 2, 4, 2)
    U = latgen.make_links(dims, 0.5, 31)
    psi = latgen.make_source(dims, 32)
    Lam = latgen.random_gauge_transform(dims, 33)
    Ug = gauge_transform(U, Lam, dims)
    m0 = -0.1
    lhs = oracle.dirac(Ug, colour_rotate(Lam, psi), m0, dims)
    rhs = colour_rotate(Lam, oracle.dirac(U, psi, m0, dims))
    assert np.abs(lhs - rhs).max() < 1e-13


def test_mass_is_diagonal():
    dims = (2, 2, 2, 4)
    U = latgen.make_links(dims, 0.4, 41)
    psi = latgen.make_source(dims, 42)
    d = oracle.dirac(U, psi, 0.3, dims) - oracle.dirac(U, psi, -0.2, dims)
    assert np.abs(d - 0.5 * psi).max() < 1e-14


def test_block_decomposition_and_sites():
    dims = (4, 4, 4, 8)
    b = (2, 2, 4, 4)
    U = latgen.make_links(dims, 0.4, 51)
    psi = latgen.make_source(dims, 52)
    m0 = -0.2
    full = oracle.dirac(U, psi, m0, dims)
    parts = oracle.dirac_blockdiag(U, psi, m0, dims, b)
    for mu in range(4):
        for s in (+1, -1):
            parts = parts + oracle.hop_cross(U, psi, dims, b, mu, s)
    assert np.abs(parts - full).max() < 1e-13
    sites = np.array([0, 5, 77, 300, 511])
    assert np.abs(oracle.dirac_sites(U, psi, m0, dims, sites) - full[sites]).max() < 1e-14


def test_blockdiag_does_not_couple_blocks():
    dims = (4, 4, 2, 2)
    b = (2, 2, 2, 2)
    U = latgen.make_links(dims, 0.4, 61)
    V = int(np.prod(dims))
    M = dense_from(lambda f: oracle.dirac_blockdiag(U, f, -0.2, dims, b), V)
    x = site_coords(dims)
    blk = np.ravel_multi_index(tuple((x // np.array(b)).T), [d // bb for d, bb in zip(dims, b)])
    blk12 = np.repeat(blk, 12)
    off = blk12[:, None] != blk12[None, :]
    assert np.abs(M[off]).max() == 0
    assert np.abs(M[~off]).max() > 0.4


def test_spectrum_conjugate_pairs():
    # gamma5-hermiticity makes det(D - z) a real polynomial: eigenvalues in conjugate pairs
    dims = (2, 2, 2, 2)
    U = latgen.make_links(dims, 0.6, 71)
    M = dense_from(lambda f: oracle.dirac(U, f, -0.2, dims), 16)
    ev = np.linalg.eigvals(M)
    for z in ev:
        assert np.min(np.abs(ev - np.conj(z))) < 1e-8
