"""Pins of the network / deficit-loss oracle (oracle.net) against facts fixed
independently of its own formulas: a brute-force convolution with explicit
coordinate arithmetic, translation equivariance, central finite differences of
the forward maps, the deficit through the block Gram-Schmidt projector of
eq. (4.2) (a separate path), its invariances, and Adam's first step in closed
form."""
import itertools

import numpy as np
import pytest

import latgen
import oracle
from oracle import net


def brute_conv(x, W, b, dims):
    V = int(np.prod(dims))
    out = np.zeros((V, W.shape[-1]))
    coords = list(itertools.product(*[range(L) for L in dims]))
    index = {c: i for i, c in enumerate(coords)}
    for i, c in enumerate(coords):
        acc = b.copy()
        for o in itertools.product((-1, 0, 1), repeat=4):
            nb = tuple((c[mu] + o[mu]) % dims[mu] for mu in range(4))
            acc = acc + x[index[nb]] @ W[o[0] + 1, o[1] + 1, o[2] + 1, o[3] + 1]
        out[i] = acc
    return out


DIMS = (3, 2, 4, 2)


def test_conv_matches_brute_force():
    rng = np.random.default_rng(1)
    V = int(np.prod(DIMS))
    x = rng.standard_normal((V, 3))
    W = rng.standard_normal((3, 3, 3, 3, 3, 2))
    b = rng.standard_normal(2)
    assert np.allclose(net.conv4d(x, W, b, DIMS), brute_conv(x, W, b, DIMS), atol=1e-12)


def test_conv_delta_kernel_is_a_shift_and_equivariant():
    rng = np.random.default_rng(2)
    dims = (4, 3, 2, 5)
    V = int(np.prod(dims))
    x = rng.standard_normal((V, 2))
    W = np.zeros((3, 3, 3, 3, 2, 2))
    W[2, 1, 0, 1] = np.eye(2)            # offset (+1, 0, -1, 0)
    out = net.conv4d(x, W, np.zeros(2), dims).reshape(dims + (2,))
    x4 = x.reshape(dims + (2,))
    for c in [(0, 0, 0, 0), (3, 2, 1, 4), (1, 0, 0, 2)]:
        src = ((c[0] + 1) % 4, c[1], (c[2] - 1) % 2, c[3])
        assert np.array_equal(out[c], x4[src])
    Wr = rng.standard_normal((3, 3, 3, 3, 2, 3))
    y = net.conv4d(x, Wr, np.zeros(3), dims).reshape(dims + (3,))
    xs = np.roll(x.reshape(dims + (2,)), shift=(1, -2, 1, 3), axis=(0, 1, 2, 3)).reshape(V, 2)
    ys = net.conv4d(xs, Wr, np.zeros(3), dims).reshape(dims + (3,))
    assert np.allclose(ys, np.roll(y, shift=(1, -2, 1, 3), axis=(0, 1, 2, 3)), atol=1e-12)


def _fd(f, a, h=1e-6):
    g = np.zeros_like(a)
    it = np.nditer(a, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        old = a[i]
        a[i] = old + h
        fp = f()
        a[i] = old - h
        fm = f()
        a[i] = old
        g[i] = (fp - fm) / (2 * h)
    return g


def test_conv_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    V = int(np.prod(DIMS))
    x = rng.standard_normal((V, 2))
    W = rng.standard_normal((3, 3, 3, 3, 2, 2)) * 0.3
    b = rng.standard_normal(2)
    g = rng.standard_normal((V, 2))
    loss = lambda: float(np.sum(g * net.conv4d(x, W, b, DIMS)))  # noqa: E731
    dx, dW, db = net.conv4d_backward(x, W, g, DIMS)
    assert np.allclose(dx, _fd(loss, x), atol=1e-6)
    assert np.allclose(db, _fd(loss, b), atol=1e-6)
    Wsub = W[:, :, 1]        # a view: finite differences on a slice of the taps
    assert np.allclose(dW[:, :, 1], _fd(loss, Wsub), atol=1e-6)


def test_silu_grad_and_net_backward_match_finite_differences():
    z = np.linspace(-6, 6, 41)
    h = 1e-6
    assert np.allclose(net.silu_grad(z), (net.silu(z + h) - net.silu(z - h)) / (2 * h), atol=1e-8)
    rng = np.random.default_rng(4)
    dims = (2, 3, 2, 2)
    V = int(np.prod(dims))
    params = [(rng.standard_normal((3, 3, 3, 3, 3, 4)) * 0.2, rng.standard_normal(4) * 0.1),
              (rng.standard_normal((3, 3, 3, 3, 4, 2)) * 0.2, rng.standard_normal(2) * 0.1)]
    x = rng.standard_normal((V, 3))
    g = rng.standard_normal((V, 2))
    loss = lambda: float(np.sum(g * net.forward(params, x, dims)[0]))  # noqa: E731
    out, cache = net.forward(params, x, dims)
    grads = net.backward(params, cache, g, dims)
    assert np.allclose(grads[0][1], _fd(loss, params[0][1]), atol=1e-6)
    assert np.allclose(grads[1][1], _fd(loss, params[1][1]), atol=1e-6)
    assert np.allclose(grads[0][0][0, 2], _fd(loss, params[0][0][0, 2]), atol=1e-6)
    assert np.allclose(grads[1][0][1, 1], _fd(loss, params[1][0][1, 1]), atol=1e-6)


B = (2, 2, 2, 2)
LDIMS = (4, 4, 2, 2)


def _fields(seed, n):
    return latgen.random_field(LDIMS, seed, n=n)


def test_deficit_equals_gram_schmidt_projector_path():
    Psi = _fields(10, 3)
    T = _fields(11, 2)
    loss, _ = net.deficit_loss(Psi, T, LDIMS, B)
    Phi = oracle.block_gram_schmidt(Psi, LDIMS, B)
    ref = np.mean([oracle.deficit(Phi, t, LDIMS, B) for t in T])
    assert abs(loss - ref) < 1e-12


def test_deficit_limits_and_basis_invariance():
    rng = np.random.default_rng(12)
    Psi = _fields(12, 3)
    # targets in the block span: zero deficit
    Pb = oracle.to_blocks(Psi, LDIMS, B)
    coef = rng.standard_normal((2, 3, Pb.shape[1])) + 1j * rng.standard_normal((2, 3, Pb.shape[1]))
    T = oracle.from_blocks(np.einsum("kln,lnj->knj", coef, Pb), LDIMS, B)
    assert net.deficit_loss(Psi, T, LDIMS, B)[0] < 1e-12
    # targets orthogonal to the span on every block: deficit one
    Phi = oracle.block_gram_schmidt(Psi, LDIMS, B)
    R = _fields(13, 2)
    Q = R - np.stack([oracle.proj_P(Phi, r, LDIMS, B) for r in R])
    assert abs(net.deficit_loss(Psi, Q, LDIMS, B)[0] - 1.0) < 1e-12
    # a change of basis within the span leaves it unchanged
    M = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    Psi2 = np.einsum("lm,lvc->mvc", M, Psi)
    a, _ = net.deficit_loss(Psi, R, LDIMS, B)
    b, _ = net.deficit_loss(Psi2, R, LDIMS, B)
    assert abs(a - b) < 1e-12


def test_deficit_gradient_matches_finite_differences():
    Psi = _fields(14, 2)
    T = _fields(15, 2)
    _, g = net.deficit_loss(Psi, T, LDIMS, B)
    rng = np.random.default_rng(16)
    for _ in range(6):
        l, v, c = rng.integers(2), rng.integers(Psi.shape[1]), rng.integers(12)
        for unit, part in [(1.0, np.real), (1j, np.imag)]:
            h = 1e-6
            P1 = Psi.copy()
            P1[l, v, c] += unit * h
            P2 = Psi.copy()
            P2[l, v, c] -= unit * h
            fd = (net.deficit_loss(P1, T, LDIMS, B)[0] - net.deficit_loss(P2, T, LDIMS, B)[0]) / (2 * h)
            assert abs(fd - 2 * part(g[l, v, c])) < 1e-7


def test_output_field_maps_are_adjoint():
    rng = np.random.default_rng(17)
    V, Ns = 8, 2
    out = rng.standard_normal((V, 24 * Ns))
    G = rng.standard_normal((Ns, V, 12)) + 1j * rng.standard_normal((Ns, V, 12))
    F = net.outputs_to_fields(out, Ns)
    assert F.shape == (Ns, V, 12)
    assert F[1, 3, 5] == out[3, (1 * 12 + 5) * 2] + 1j * out[3, (1 * 12 + 5) * 2 + 1]
    # L = 2 Re <G, Psi>  has dL/dconj(Psi) = G, so dL/dout = fields_grad_to_outputs(G)
    d = rng.standard_normal(out.shape)
    h = 1e-6
    L = lambda o: 2 * np.vdot(G, net.outputs_to_fields(o, Ns)).real  # noqa: E731
    fd = (L(out + h * d) - L(out - h * d)) / (2 * h)
    assert abs(fd - np.sum(net.fields_grad_to_outputs(G) * d)) < 1e-6


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = net.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # t = 1: m_hat = g, v_hat = g^2, so the step is lr * g / (|g| + eps)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_generators():
    p = latgen.net_init(latgen.NET_CHANNELS, 5)
    assert [w.shape for w, _ in p] == [(3, 3, 3, 3, 96, 32), (3, 3, 3, 3, 32, 32), (3, 3, 3, 3, 32, 32),
                                        (3, 3, 3, 3, 32, 576)]
    assert abs(np.var(p[0][0]) * 81 * 96 - 1.0) < 0.05
    assert np.array_equal(latgen.net_noise((2, 2, 2, 2), 3), latgen.net_noise((2, 2, 2, 2), 3))
    U = latgen.make_links((2, 2, 2, 2), 0.4, 1)
    f = net.link_features(U)
    assert f[3, ((2 * 3 + 1) * 3 + 0) * 2 + 1] == U[3, 2, 1, 0].imag
