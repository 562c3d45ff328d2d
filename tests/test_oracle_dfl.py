"""Pins of the oracle's deflation part (sections 3, 4, 5, 6 and appendix A).

* block Gram-Schmidt (eq. (4.2)) equals the library QR with a positive R
  diagonal, block by block;
* free field with the 12 constant block modes: the deficit of a plane wave has
  the exact closed form 1 - prod_mu [sin(p_mu b_mu/2)/(b_mu sin(p_mu/2))]^2, whose
  small-p limit is eq. (4.4), p^2 (b^2 - a^2)/12 with a = 1;
* the little operator equals Phi^dagger D Phi from the dense D and vanishes
  outside the nearest-neighbour block stencil (eq. (A.1), fig. 4); with a
  complete block basis its spectrum is that of D;
* projector identities (3.5)-(3.8), the solution split (3.10), the Schur
  inverse (3.14) and the determinant factorisation (6.3), with dense matrices;
* GCR solves agree with the dense LU solution; deflated SAP-GCR reaches the
  stopping criterion of section 6.3 with a true residual below it.
"""
import numpy as np
import pytest

import latgen
import oracle
from oracle_util import dense_from, site_coords


def test_block_gs_is_qr():
    dims = (4, 4, 4, 4)
    b = (2, 2, 2, 4)
    f = latgen.make_init_fields(dims, 5, 201)
    Phi = oracle.block_gram_schmidt(f, dims, b)
    Pb = oracle.to_blocks(Phi, dims, b)        # (Ns, Nb, n)
    Fb = oracle.to_blocks(f, dims, b)
    for k in range(Pb.shape[1]):
        Q = Pb[:, k, :].T                       # n x Ns
        assert np.abs(Q.conj().T @ Q - np.eye(5)).max() < 1e-14
        q, r = np.linalg.qr(Fb[:, k, :].T)
        ph = np.diag(r) / np.abs(np.diag(r))
        q = q * ph[None, :]
        assert np.abs(q - Q).max() < 1e-13
    # restriction to a block keeps the span: P psi_l = psi_l
    for l in range(5):
        assert np.abs(oracle.proj_P(Phi, f[l], dims, b) - f[l]).max() < 1e-12


def test_block_gs_rank_loss():
    dims = (2, 2, 2, 4)
    b = (1, 1, 2, 2)
    f = latgen.make_init_fields(dims, 3, 202)
    f[2] = 2.0 * f[0] - 1j * f[1]
    with pytest.raises(ValueError):
        oracle.block_gram_schmidt(f, dims, b)


def test_to_from_blocks_roundtrip():
    dims = (4, 2, 6, 4)
    b = (2, 2, 3, 2)
    f = latgen.make_source(dims, 203)
    fb = oracle.to_blocks(f, dims, b)
    assert fb.shape == (2 * 1 * 2 * 2, 24 * 12)
    assert np.array_equal(oracle.from_blocks(fb, dims, b), f)
    # block 0 holds exactly the sites with x_mu < b_mu
    x = site_coords(dims)
    on = np.all(x < np.array(b), axis=1)
    assert np.array_equal(np.sort(np.abs(fb[0])), np.sort(np.abs(f[on].reshape(-1))))


def _constant_modes(dims):
    V = int(np.prod(dims))
    f = np.zeros((12, V, 12), dtype=np.complex128)
    for j in range(12):
        f[j, :, j] = 1.0
    return f


@pytest.mark.parametrize("dims,b", [((16, 16, 16, 16), (4, 4, 4, 4)), ((8, 12, 8, 4), (4, 3, 2, 2))])
def test_free_field_deficit_closed_form(dims, b):
    Phi = oracle.block_gram_schmidt(_constant_modes(dims), dims, b)
    x = site_coords(dims)
    rng = np.random.default_rng(204)
    for n in [(1, 0, 0, 0), (0, 1, 1, 0), (1, 2, 0, 1), (0, 0, 0, 1)]:
        p = 2 * np.pi * np.array(n) / np.array(dims)
        u = rng.standard_normal(12) + 1j * rng.standard_normal(12)
        psi = np.exp(1j * (x @ p))[:, None] * u[None, :]
        eps = oracle.deficit(Phi, psi, dims, b)
        fac = 1.0
        for mu in range(4):
            if n[mu]:
                fac *= (np.sin(p[mu] * b[mu] / 2) / (b[mu] * np.sin(p[mu] / 2))) ** 2
        assert abs(eps - (1 - fac)) < 1e-12


def test_free_field_deficit_small_p_limit_eq_4_4():
    # eq. (4.4): eps_p = p^2 (b^2 - a^2)/12 + O(p^4 b^4); a = 1, b = 4, p along x0 only
    b = (4, 2, 2, 2)
    ratios = []
    for L in (32, 64, 128):
        dims = (L, 2, 2, 2)
        Phi = oracle.block_gram_schmidt(_constant_modes(dims), dims, b)
        x = site_coords(dims)
        p = 2 * np.pi / L
        psi = np.exp(1j * p * x[:, 0])[:, None] * np.ones(12)[None, :]
        eps = oracle.deficit(Phi, psi, dims, b)
        ratios.append(eps / (p * p * (b[0] ** 2 - 1) / 12))
    dev = [abs(r - 1) for r in ratios]
    assert dev[0] > dev[1] > dev[2] and dev[2] < 5e-3
    # the O(p^4 b^4) correction shrinks like p^2: quartered when p halves
    assert 3.5 < dev[0] / dev[1] < 4.5


def _small_setup(dims, b, Ns, seed, eps=0.5):
    U = latgen.make_links(dims, eps, seed)
    f = latgen.make_init_fields(dims, Ns, seed + 1)
    Phi = oracle.block_gram_schmidt(f, dims, b)
    return U, Phi


def _block_index(dims, b):
    x = site_coords(dims)
    nb = [d // bb for d, bb in zip(dims, b)]
    return np.ravel_multi_index(tuple((x // np.array(b)).T), nb), nb


def test_little_operator_is_projected_D_and_block_sparse():
    dims = (4, 8, 4, 4)
    b = (2, 2, 2, 2)          # 2 x 4 x 2 x 2 blocks: both the 2-block and the 4-block case
    Ns = 3
    m0 = -0.25
    U, Phi = _small_setup(dims, b, Ns, 211)
    V = int(np.prod(dims))
    A = oracle.little_operator(U, Phi, m0, dims, b)
    Ad = oracle.little_dense(A, dims, b)
    # dense Phi^dagger D Phi, column by column, from the plain operator
    Pb = oracle.to_blocks(Phi, dims, b)
    Nb = Pb.shape[1]
    cols = np.empty((Nb * Ns, Nb * Ns), dtype=np.complex128)
    for L in range(Nb):
        for l in range(Ns):
            e = np.zeros((Nb, Ns), dtype=np.complex128)
            e[L, l] = 1
            cols[:, L * Ns + l] = oracle.restrict(Phi, oracle.dirac(U, oracle.prolong(Phi, e, dims, b), m0, dims),
                                                  dims, b).reshape(-1)
    assert np.abs(cols - Ad).max() < 1e-13
    # fig. 4: zero unless the blocks coincide or are nearest neighbours
    nb = [d // bb for d, bb in zip(dims, b)]
    n = np.array(np.unravel_index(np.arange(Nb), nb)).T
    for L in range(Nb):
        for M in range(Nb):
            dist = [min((n[L, mu] - n[M, mu]) % nb[mu], (n[M, mu] - n[L, mu]) % nb[mu]) for mu in range(4)]
            blk = cols[L * Ns:(L + 1) * Ns, M * Ns:(M + 1) * Ns]
            if sum(dist) > 1:
                assert np.abs(blk).max() == 0
            else:
                assert np.abs(blk).max() > 1e-3
    # the matrix-free apply agrees with the dense matrix
    v = np.random.default_rng(5).standard_normal((Nb, Ns)) * (1 + 0.5j)
    assert np.abs(oracle.little_apply(A, v, dims, b).reshape(-1) - Ad @ v.reshape(-1)).max() < 1e-13
    del V


@pytest.mark.parametrize("dims,b", [((2, 2, 2, 2), (1, 1, 1, 1)), ((4, 2, 2, 2), (2, 1, 1, 1))])
def test_complete_basis_spectrum(dims, b):
    V = int(np.prod(dims))
    Vb = int(np.prod(b))
    Ns = 12 * Vb
    m0 = -0.3
    U, Phi = _small_setup(dims, b, Ns, 221)
    A = oracle.little_operator(U, Phi, m0, dims, b)
    ea = np.sort_complex(np.round(np.linalg.eigvals(oracle.little_dense(A, dims, b)), 9))
    ed = np.sort_complex(np.round(np.linalg.eigvals(dense_from(lambda f: oracle.dirac(U, f, m0, dims), V)), 9))
    assert np.abs(ea - ed).max() < 1e-8


@pytest.fixture(scope="module")
def dense_dfl():
    dims = (4, 4, 2, 2)
    b = (2, 2, 1, 1)
    Ns = 6
    m0 = -0.3
    U, Phi = _small_setup(dims, b, Ns, 231)
    A = oracle.little_operator(U, Phi, m0, dims, b)
    dfl = oracle.Deflation(U, Phi, A, m0, dims, b)
    V = int(np.prod(dims))
    mats = {
        "D": dense_from(dfl.D, V),
        "P": dense_from(dfl.P, V),
        "PL": dense_from(dfl.PL, V),
        "PR": dense_from(dfl.PR, V),
        "Q": dense_from(dfl.coarse, V),
    }
    return dfl, mats


def test_projector_identities(dense_dfl):
    _, m = dense_dfl
    D, P, PL, PR = m["D"], m["P"], m["PL"], m["PR"]
    one = np.eye(D.shape[0])
    tol = 1e-11
    assert np.abs(P @ P - P).max() < tol and np.abs(P - P.conj().T).max() < tol
    assert np.abs(PL @ PL - PL).max() < tol                 # (3.5)
    assert np.abs(PR @ PR - PR).max() < tol                 # (3.5)
    assert np.abs(PL @ D - D @ PR).max() < tol              # (3.6)
    assert np.abs(P @ PL).max() < tol                       # (3.7)
    assert np.abs(PR @ P).max() < tol                       # (3.7)
    assert np.abs(PL @ (one - P) - (one - P)).max() < tol   # (3.8)
    assert np.abs((one - P) @ PR - (one - P)).max() < tol   # (3.8)
    # oblique, not orthogonal
    assert np.abs(PL - PL.conj().T).max() > 1e-3


def test_solution_split_and_schur_inverse(dense_dfl):
    dfl, m = dense_dfl
    D, P, PL, PR, Q = m["D"], m["P"], m["PL"], m["PR"], m["Q"]
    one = np.eye(D.shape[0])
    Dinv = np.linalg.inv(D)
    eta = latgen.make_source(dfl.dims, 232).reshape(-1)
    psi = Dinv @ eta
    chi = PR @ psi
    assert np.abs(PL @ D @ chi - PL @ eta).max() < 1e-11    # (3.11)
    assert np.abs(chi + Q @ eta - psi).max() < 1e-11        # (3.10)
    assert np.abs(PL @ D - PL @ D @ (one - P)).max() < 1e-11   # (3.13)
    # (3.14): on the orthogonal complement, (1-P) D^{-1} (1-P) inverts P_L D
    y = (one - P) @ latgen.make_source(dfl.dims, 233).reshape(-1)
    z = (one - P) @ Dinv @ (one - P) @ y
    assert np.abs(PL @ D @ z - y).max() < 1e-11


def test_determinant_factorisation_eq_6_3():
    dims = (2, 2, 2, 2)
    b = (1, 1, 1, 1)
    Ns = 5
    m0 = -0.2
    U, Phi = _small_setup(dims, b, Ns, 241, eps=0.6)
    A = oracle.little_operator(U, Phi, m0, dims, b)
    dfl = oracle.Deflation(U, Phi, A, m0, dims, b)
    V = 16
    D = dense_from(dfl.D, V)
    PL = dense_from(dfl.PL, V)
    P = dense_from(dfl.P, V)
    # orthonormal basis of the complement of the deflation subspace
    w, vecs = np.linalg.eigh(np.eye(V * 12) - P)
    Qp = vecs[:, w > 0.5]
    assert Qp.shape[1] == V * 12 - 16 * Ns
    Dhat = Qp.conj().T @ PL @ D @ Qp
    s1, l1 = np.linalg.slogdet(D)
    s2, l2 = np.linalg.slogdet(oracle.little_dense(A, dims, b))
    s3, l3 = np.linalg.slogdet(Dhat)
    assert abs(l1 - (l2 + l3)) < 1e-9
    assert abs(s1 - s2 * s3) < 1e-9


def test_gcr_matches_dense_solve():
    dims = (4, 4, 4, 4)
    m0 = -0.2
    U = latgen.make_links(dims, 0.4, 251)
    eta = latgen.make_source(dims, 252)
    V = int(np.prod(dims))
    D = dense_from(lambda f: oracle.dirac(U, f, m0, dims), V)
    want = np.linalg.solve(D, eta.reshape(-1))
    hist = []
    psi, it, ok = oracle.solve(U, eta, m0, dims, tol=1e-12, nkv=16, history=hist)
    assert ok
    assert np.linalg.norm(psi.reshape(-1) - want) < 1e-9 * np.linalg.norm(want)
    psi2, it2, ok2 = oracle.solve(U, eta, m0, dims, sap_block=(2, 2, 2, 2), ncy=5, nmr=4, tol=1e-12)
    assert ok2 and it2 < it
    assert np.linalg.norm(psi2.reshape(-1) - want) < 1e-9 * np.linalg.norm(want)


def test_deflated_sap_gcr_small():
    dims = (8, 8, 8, 8)
    b = (4, 4, 4, 4)
    m0 = -0.2
    U = latgen.make_links(dims, 0.4, 1001)
    eta = latgen.make_source(dims, 1002)
    init = latgen.make_init_fields(dims, 8, 1003)
    Phi, A = oracle.setup(U, init, m0, dims, b, b, 5, 4, 3)
    dfl = oracle.Deflation(U, Phi, A, m0, dims, b)
    hist = []
    psi, it, ok = oracle.solve(U, eta, m0, dims, sap_block=b, ncy=5, nmr=4, dfl=dfl, tol=1e-10, history=hist)
    assert ok
    r = eta - oracle.dirac(U, psi, m0, dims)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(eta)
    _, it_sap, ok_sap = oracle.solve(U, eta, m0, dims, sap_block=b, ncy=5, nmr=4, tol=1e-10)
    assert ok_sap and it <= it_sap


def test_inverse_iteration_lowers_rayleigh_bound():
    # bound (5.2): ||D psi_l|| / ||psi_l|| falls as inverse-iteration steps accumulate
    dims = (8, 8, 8, 8)
    b = (4, 4, 4, 4)
    m0 = -0.2
    U = latgen.make_links(dims, 0.4, 1001)
    init = latgen.make_init_fields(dims, 2, 1003)
    ratios = []
    for n in (0, 1, 3):
        f = oracle.inverse_iteration(U, init, m0, dims, b, 5, 4, n)
        ratios.append(max(np.linalg.norm(oracle.dirac(U, g, m0, dims)) / np.linalg.norm(g) for g in f))
    assert ratios[0] > ratios[1] > ratios[2]


def test_inverse_iteration_is_normalised_inverse_power():
    # eq. (5.1) with the Schwarz procedure replaced by its limit: at a heavy
    # setup mass, with many cycles and MR steps, M_sap is D^-1 to rounding, so
    # n steps of the relaxed inverse iteration give D^-n psi_0 / ||D^-n psi_0||
    # (psi_0 normalised first, each step normalised); the dense D comes from
    # the oracle's stencil at the setup mass, not at another mass
    dims, b = (4, 4, 2, 2), (2, 2, 1, 1)
    V = int(np.prod(dims))
    m_setup = 1.0
    U = latgen.make_links(dims, 0.4, 1101)
    init = latgen.make_init_fields(dims, 2, 1102)
    D = dense_from(lambda f: oracle.dirac(U, f, m_setup, dims), V)
    D_other = dense_from(lambda f: oracle.dirac(U, f, 0.3, dims), V)
    for n in (1, 2):
        got = oracle.inverse_iteration(U, 7.0 * init, m_setup, dims, b, 30, 30, n)
        for l in range(2):
            assert abs(np.linalg.norm(got[l]) - 1.0) < 1e-13
            want = init[l].reshape(-1)
            other = want.copy()
            for _ in range(n):
                want = np.linalg.solve(D, want)
                other = np.linalg.solve(D_other, other)
            want /= np.linalg.norm(want)
            other /= np.linalg.norm(other)
            assert np.abs(got[l].reshape(-1) - want).max() < 1e-10
            assert np.abs(got[l].reshape(-1) - other).max() > 1e-3
    # zero steps: the normalised start fields
    got0 = oracle.inverse_iteration(U, 3.0 * init, m_setup, dims, b, 30, 30, 0)
    for l in range(2):
        assert np.abs(got0[l] - init[l] / np.linalg.norm(init[l])).max() < 1e-15


def test_bootstrapped_inverse_iteration_exact_limit():
    # with M_sap -> D^-1 (heavy setup mass, many cycles and MR steps) the
    # bootstrapped step P_R M_sap P_L + Phi A^-1 Phi^dagger is D^-1 itself, so n
    # steps with any number of bootstrapped ones give the normalised D^-n psi_0
    dims, b = (4, 4, 2, 2), (2, 2, 1, 1)
    V = int(np.prod(dims))
    m_setup = 1.0
    U = latgen.make_links(dims, 0.4, 1101)
    init = latgen.make_init_fields(dims, 2, 1102)
    D = dense_from(lambda f: oracle.dirac(U, f, m_setup, dims), V)
    for n, nb in ((1, 1), (2, 1), (2, 2)):
        got = oracle.inverse_iteration(U, 3.0 * init, m_setup, dims, b, 30, 30, n, n_boot=nb, dfl_block=b)
        for l in range(2):
            want = init[l].reshape(-1)
            for _ in range(n):
                want = np.linalg.solve(D, want)
            want /= np.linalg.norm(want)
            assert abs(np.linalg.norm(got[l]) - 1.0) < 1e-13
            assert np.abs(got[l].reshape(-1) - want).max() < 1e-10


def test_bootstrapped_inverse_iteration_lowers_bound_5_2():
    # at a light mass with the standard Schwarz parameters, deflating the last
    # steps with the current fields (section 5.3) gives fields with a smaller
    # bound M of eq. (5.2) than plain inverse iteration with the same steps,
    # and a subspace that is no worse for the lowest modes of D^dagger D
    # (deficits eq. (3.15) of the 8 lowest right singular vectors of the dense D)
    dims, b = (4, 4, 4, 4), (2, 2, 2, 2)
    V = int(np.prod(dims))
    m0 = -0.3
    U = latgen.make_links(dims, 0.4, 1201)
    init = latgen.make_init_fields(dims, 6, 1202)
    D = dense_from(lambda f: oracle.dirac(U, f, m0, dims), V)
    low = np.linalg.svd(D)[2][-8:].conj()

    def stats(n_iter, n_boot):
        f = oracle.inverse_iteration(U, init, m0, dims, b, 5, 4, n_iter, n_boot=n_boot, dfl_block=b)
        Phi = oracle.block_gram_schmidt(f, dims, b)
        dfc = np.mean([oracle.deficit(Phi, low[k].reshape(V, 12), dims, b) for k in range(8)])
        ray = np.mean([np.linalg.norm(oracle.dirac(U, g, m0, dims)) / np.linalg.norm(g) for g in f])
        return ray, dfc

    r_plain, d_plain = stats(3, 0)
    r_boot, d_boot = stats(3, 1)
    assert r_boot < 0.75 * r_plain
    assert d_boot <= d_plain + 1e-3
    r_plain4, d_plain4 = stats(4, 0)
    r_boot4, d_boot4 = stats(4, 2)
    assert r_boot4 < 0.75 * r_plain4 and d_boot4 <= d_plain4 + 1e-3
