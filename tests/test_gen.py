"""Seeded input generator: SU(3) links, reproducibility, recipes."""
import numpy as np

import latgen


def test_gell_mann_algebra():
    g = latgen.gell_mann()
    for a in range(8):
        assert np.allclose(g[a], g[a].conj().T)
        assert abs(np.trace(g[a])) < 1e-15
        for b in range(8):
            # tr(lambda_a lambda_b) = 2 delta_ab
            assert abs(np.trace(g[a] @ g[b]) - 2.0 * (a == b)) < 1e-14


def test_links_are_su3_and_seeded():
    dims = (2, 2, 2, 4)
    U = latgen.make_links(dims, 0.4, seed=11)
    assert U.shape == (32, 4, 3, 3)
    eye = np.eye(3)
    uu = np.einsum("smab,smcb->smac", U, U.conj())
    assert np.abs(uu - eye).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    U2 = latgen.make_links(dims, 0.4, seed=11)
    assert np.array_equal(U, U2)
    assert not np.array_equal(U, latgen.make_links(dims, 0.4, seed=12))


def test_links_eps_zero_is_free_field():
    U = latgen.make_links((2, 2, 2, 2), 0.0, seed=1)
    assert np.abs(U - np.eye(3)).max() == 0


def test_mean_plaquette_like_trace_decreases_with_eps():
    # <Re tr U>/3 falls as eps grows (0.4 -> about 0.9, 0.6 -> about 0.78)
    t = [np.mean(np.trace(latgen.make_links((4, 4, 4, 4), e, 3), axis1=-2, axis2=-1).real) / 3
         for e in (0.4, 0.5, 0.6)]
    assert t[0] > t[1] > t[2]
    assert 0.85 < t[0] < 0.95 and 0.72 < t[2] < 0.83


def test_sources():
    s = latgen.make_source((2, 2, 2, 2), 5)
    assert s.shape == (16, 12) and s.dtype == np.complex128
    assert np.array_equal(s, latgen.make_source((2, 2, 2, 2), 5))
    p = latgen.point_sources((2, 2, 2, 2), range(12))
    assert p.shape == (12, 16, 12)
    assert np.array_equal(p[:, 0, :], np.eye(12))
    assert np.count_nonzero(p) == 12
    f = latgen.make_init_fields((2, 2, 2, 2), 3, 7)
    assert f.shape == (3, 16, 12)
