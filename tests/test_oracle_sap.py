"""Pins of the oracle's block solver (MR) and Schwarz alternating procedure.

The paper defers SAP to its Schwarz-preconditioning reference, so these pins
check what the mathematics fixes for the reading the oracle implements:

* MR on D_Lambda: residual norms never increase; many steps at heavy mass give
  the dense block inverse;
* with exact block solves one SAP cycle is the multiplicative Schwarz map
  psi = K0 rho + K1 (rho - D K0 rho) (colour 0 first), K_c the direct sum of
  the block inverses on colour c (built densely here, not by the oracle);
* many cycles at heavy mass converge to D^{-1} rho;
* M_sap(c rho) = c M_sap(rho) and gauge covariance.
"""
import numpy as np

import latgen
import oracle
from oracle_util import dense_from, gauge_transform, colour_rotate, site_coords


def _block_of_sites(dims, b):
    x = site_coords(dims)
    nb = [d // bb for d, bb in zip(dims, b)]
    return np.ravel_multi_index(tuple((x // np.array(b)).T), nb)


def test_mr_residual_monotone_and_converges():
    dims = (4, 4, 4, 4)
    b = (2, 2, 2, 2)
    U = latgen.make_links(dims, 0.5, 101)
    rhs = latgen.make_source(dims, 102)
    blk = 5
    on = _block_of_sites(dims, b) == blk
    res = []
    for nmr in range(0, 7):
        x = oracle.mr_block(U, rhs, -0.2, dims, b, blk, nmr)
        assert np.all(x[~on] == 0)
        r = rhs - oracle.dirac_blockdiag(U, x, -0.2, dims, b)
        res.append(np.linalg.norm(r[on]))
    assert all(res[i + 1] <= res[i] * (1 + 1e-14) for i in range(len(res) - 1))
    assert res[-1] < res[0]
    # heavy mass, many steps: the dense block inverse
    m0 = 0.5
    V = int(np.prod(dims))
    Mbd = dense_from(lambda f: oracle.dirac_blockdiag(U, f, m0, dims, b), V)
    idx = np.repeat(on, 12)
    sub = Mbd[np.ix_(idx, idx)]
    want = np.linalg.solve(sub, rhs.reshape(-1)[idx])
    x = oracle.mr_block(U, rhs, m0, dims, b, blk, 200)
    assert np.abs(x.reshape(-1)[idx] - want).max() < 1e-12 * np.abs(want).max()


def _dense_colour_inverse(U, m0, dims, b, colour):
    V = int(np.prod(dims))
    Mbd = dense_from(lambda f: oracle.dirac_blockdiag(U, f, m0, dims, b), V)
    col = oracle.block_colours(dims, b)[_block_of_sites(dims, b)]
    K = np.zeros_like(Mbd)
    blks = _block_of_sites(dims, b)
    for k in np.unique(blks):
        on = np.repeat(blks == k, 12)
        if col[blks == k][0] != colour:
            continue
        K[np.ix_(on, on)] = np.linalg.inv(Mbd[np.ix_(on, on)])
    return K


def test_sap_exact_blocks_is_multiplicative_schwarz():
    dims = (4, 4, 4, 4)
    b = (2, 2, 2, 2)
    m0 = 0.6
    V = int(np.prod(dims))
    U = latgen.make_links(dims, 0.4, 111)
    rho = latgen.make_source(dims, 112).reshape(-1)
    D = dense_from(lambda f: oracle.dirac(U, f, m0, dims), V)
    K0 = _dense_colour_inverse(U, m0, dims, b, 0)
    K1 = _dense_colour_inverse(U, m0, dims, b, 1)
    psi = np.zeros_like(rho)
    for ncy in (1, 2):
        psi = psi + K0 @ (rho - D @ psi)
        psi = psi + K1 @ (rho - D @ psi)
        got = oracle.sap(U, rho, m0, dims, b, ncy, 120).reshape(-1)
        assert np.abs(got - psi).max() < 1e-11 * np.abs(psi).max()
    # the order of the colours matters: colour 1 first gives a different map
    other = K1 @ rho
    other = other + K0 @ (rho - D @ other)
    got1 = oracle.sap(U, rho, m0, dims, b, 1, 120).reshape(-1)
    assert np.abs(got1 - other).max() > 1e-3


def test_sap_converges_to_inverse_at_heavy_mass():
    dims = (4, 4, 4, 8)
    b = (2, 2, 2, 4)
    m0 = 0.5
    U = latgen.make_links(dims, 0.4, 121)
    rho = latgen.make_source(dims, 122)
    psi = oracle.sap(U, rho, m0, dims, b, 40, 30)
    r = rho - oracle.dirac(U, psi, m0, dims)
    assert np.linalg.norm(r) < 1e-10 * np.linalg.norm(rho)


def test_sap_scale_and_gauge_covariance():
    dims = (4, 4, 4, 4)
    b = (2, 2, 2, 2)
    m0 = -0.2
    U = latgen.make_links(dims, 0.5, 131)
    rho = latgen.make_source(dims, 132)
    M = oracle.sap(U, rho, m0, dims, b, 3, 4)
    c = 0.7 - 2.1j
    assert np.abs(oracle.sap(U, c * rho, m0, dims, b, 3, 4) - c * M).max() < 1e-12 * np.abs(M).max()
    Lam = latgen.random_gauge_transform(dims, 133)
    Ug = gauge_transform(U, Lam, dims)
    Mg = oracle.sap(Ug, colour_rotate(Lam, rho), m0, dims, b, 3, 4)
    assert np.abs(Mg - colour_rotate(Lam, M)).max() < 1e-12 * np.abs(M).max()
    # the map is not linear (the MR step lengths depend on the residue)
    rho2 = latgen.make_source(dims, 134)
    lin = oracle.sap(U, rho + rho2, m0, dims, b, 3, 4) - M - oracle.sap(U, rho2, m0, dims, b, 3, 4)
    assert np.abs(lin).max() > 1e-6


def test_sap_reduces_residual():
    dims = (8, 8, 8, 8)
    b = (4, 4, 4, 4)
    m0 = -0.2
    U = latgen.make_links(dims, 0.4, 1001)
    rho = latgen.make_source(dims, 1002)
    psi = oracle.sap(U, rho, m0, dims, b, 5, 4)
    r = rho - oracle.dirac(U, psi, m0, dims)
    assert np.linalg.norm(r) < 0.5 * np.linalg.norm(rho)
