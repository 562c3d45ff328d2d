"""GPU parity of the start-field network kernels with the FP64 oracle
(oracle.net), and the gain of the trained network over random start fields.

Tolerances: FP32 convolutions relative 2e-5 of the largest entry (sums of
81*Cin products); deficit loss FP64 1e-12 relative, its gradient 1e-10; the
whole network's parameter gradients in FP32 1e-3 relative.
"""
import numpy as np
import pytest

import latgen
import oracle
from oracle import net as onet
from paper_0706_2298_amd import F32, Solver, binding
from paper_0706_2298_amd.learned import StartFieldNet, make_targets

pytestmark = pytest.mark.gpu

DIMS = (8, 8, 8, 8)
B = (4, 4, 4, 4)
V = int(np.prod(DIMS))


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def S():
    s = Solver(DIMS, Ns=24, nkv=8, m0=-0.2, m0_setup=-0.2, n_inviter=3, sap_prec=F32, link_prec=F32,
               little_prec=F32, nrhs_max=1)
    s.set_gauge(latgen.make_links(DIMS, 0.4, 6001))
    yield s
    s.close()


def dev(a, torch):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


@pytest.mark.parametrize("cin,cout", [(5, 7), (96, 37), (32, 576)])
def test_conv_forward_backward(S, cin, cout):
    say(f"conv {cin}->{cout}")
    torch = S.torch
    rng = np.random.default_rng(cin * 1000 + cout)
    x = rng.standard_normal((V, cin))
    W = rng.standard_normal((3, 3, 3, 3, cin, cout)) / np.sqrt(81 * cin)
    b = rng.standard_normal(cout)
    g = rng.standard_normal((V, cout))
    zin = rng.standard_normal((V, cin))
    xd, Wd, bd = dev(x.T, torch), dev(W.reshape(81, cin, cout), torch), dev(b, torch)
    z = torch.empty(cout * V, dtype=torch.float32, device="cuda")
    a = torch.empty_like(z)
    binding.conv4d_forward(S.ctx, xd, cin, Wd, bd, cout, z, a)
    zr = onet.conv4d(x, W, b, DIMS)
    assert rel(z.cpu().numpy().reshape(cout, V).T, zr) < 2e-5
    assert rel(a.cpu().numpy().reshape(cout, V).T, onet.silu(zr)) < 2e-5
    dW = torch.empty_like(Wd)
    db = torch.empty_like(bd)
    din = torch.empty_like(xd)
    binding.conv4d_backward(S.ctx, xd, cin, Wd, cout, dev(g.T, torch), dW, db, din, dev(zin.T, torch))
    dxr, dWr, dbr = onet.conv4d_backward(x, W, g, DIMS)
    assert rel(dW.cpu().numpy().reshape(W.shape), dWr) < 2e-5
    assert rel(db.cpu().numpy(), dbr) < 2e-5
    assert rel(din.cpu().numpy().reshape(cin, V).T, dxr * onet.silu_grad(zin)) < 2e-5


def test_features_and_field_maps(S):
    say("features and field maps")
    torch = S.torch
    U = latgen.make_links(DIMS, 0.4, 6001)
    noise = latgen.net_noise(DIMS, 6002)
    x = torch.empty(96 * V, dtype=torch.float32, device="cuda")
    binding.net_features(S.ctx, dev(noise, torch), x)
    ref = onet.net_inputs(U, noise).astype(np.float32)
    assert np.array_equal(x.cpu().numpy().reshape(96, V).T, ref)
    rng = np.random.default_rng(3)
    out = rng.standard_normal((V, 48)).astype(np.float32)
    f = S.field(2)
    binding.net_outputs_to_fields(S.ctx, dev(out.T, torch), 2, f)
    assert np.array_equal(S.unpack(f), onet.outputs_to_fields(out.astype(np.float64), 2))
    G = latgen.random_field(DIMS, 4, n=2)
    d = torch.empty(48 * V, dtype=torch.float32, device="cuda")
    binding.net_fields_grad_to_outputs(S.ctx, S.pack(G), 2, d)
    assert rel(d.cpu().numpy().reshape(48, V).T, onet.fields_grad_to_outputs(G)) < 1e-7


def test_deficit_loss(S):
    say("deficit loss")
    Psi = latgen.random_field(DIMS, 11, n=6)
    T = latgen.random_field(DIMS, 12, n=4)
    T[0] += 3.0 * Psi[1]  # a target close to the span
    g = S.field(6)
    loss = binding.deficit_loss(S.ctx, S.pack(Psi), 6, S.pack(T), 4, g)
    lr, gr = onet.deficit_loss(Psi, T, DIMS, B)
    assert abs(loss - lr) <= 1e-12 * abs(lr)
    assert rel(S.unpack(g), gr) < 1e-10
    # linearly dependent fields on a block are an error
    Psi[2] = Psi[0]
    with pytest.raises(binding.DflError):
        binding.deficit_loss(S.ctx, S.pack(Psi), 6, S.pack(T), 4, None)


def test_adam(S):
    say("adam")
    torch = S.torch
    rng = np.random.default_rng(5)
    th = rng.standard_normal(1000)
    m = np.zeros(1000)
    v = np.zeros(1000)
    thd, md, vd = dev(th, torch), dev(m, torch), dev(v, torch)
    for t in range(1, 4):
        g = rng.standard_normal(1000)
        binding.adam_update(S.ctx, thd, dev(g, torch), md, vd, t, lr=0.01)
        th, m, v = onet.adam(th, g, m, v, t, lr=0.01)
    assert np.abs(thd.cpu().numpy() - th).max() < 1e-6


def test_network_gradients(S):
    # the whole chain: features -> 3 convolutions -> fields -> deficit -> gradients
    say("network gradients")
    chans = (96, 8, 8, 48)
    weights = latgen.net_init(chans, 21)
    weights = [(W, np.random.default_rng(22 + i).standard_normal(b.shape) * 0.1) for i, (W, b) in enumerate(weights)]
    N = StartFieldNet(S, weights, chans)
    noise = latgen.net_noise(DIMS, 23)
    T = latgen.random_field(DIMS, 24, n=3)
    fields = N.forward(noise)
    loss, grad = N.loss(fields, S.pack(T), 3)
    grads = N.backward(grad)
    U = latgen.make_links(DIMS, 0.4, 6001)
    x = onet.net_inputs(U, noise)
    Wn = N.weights_numpy()
    out, cache = onet.forward(Wn, x, DIMS)
    Psi = onet.outputs_to_fields(out, 2)
    assert rel(S.unpack(fields), Psi) < 1e-4
    lr, gr = onet.deficit_loss(Psi, T, DIMS, B)
    assert abs(loss - lr) < 1e-4 * lr
    ref = onet.backward(Wn, cache, onet.fields_grad_to_outputs(gr), DIMS)
    for i, (dW, db) in enumerate(grads):
        assert rel(dW.cpu().numpy().reshape(ref[i][0].shape), ref[i][0]) < 1e-3, i
        assert rel(db.cpu().numpy(), ref[i][1]) < 1e-3, i


def test_inverse_iteration_matches_oracle():
    say("inverse iteration")
    from paper_0706_2298_amd import F64
    U = latgen.make_links(DIMS, 0.4, 6001)
    init = latgen.make_init_fields(DIMS, 3, 31)
    s = Solver(DIMS, Ns=3, m0=-0.2, m0_setup=-0.25, ncy=2, nmr=3, sap_prec=F64, link_prec=F64)
    s.set_gauge(U)
    f = make_targets(s, s.pack(init), 2)
    ref = oracle.inverse_iteration(U, init, -0.25, DIMS, B, 2, 3, 2)
    assert rel(s.unpack(f), ref) < 1e-12
    s.close()


def test_trained_network_beats_random_start(S):
    """Train on two gauge fields, then on a held-out field compare the deficit
    of its inverse-iteration low modes w.r.t. the block span of (a) the
    trained network's fields, (b) random Gaussian fields, (c) the untrained
    network, each after k = 0 and k = 1 inverse-iteration steps."""
    say("training")
    torch = S.torch
    K = 24
    train = []
    for seed in (6101, 6102):
        S.set_gauge(latgen.make_links(DIMS, 0.4, seed))
        tgt = make_targets(S, S.pack(latgen.make_init_fields(DIMS, K, seed + 1)), 3)
        train.append((seed, tgt))
    N = StartFieldNet(S, latgen.net_init(latgen.NET_CHANNELS, 6200))
    N0 = StartFieldNet(S, latgen.net_init(latgen.NET_CHANNELS, 6200))
    losses = []
    for step in range(120):
        seed, tgt = train[step % 2]
        S.set_gauge(latgen.make_links(DIMS, 0.4, seed))
        losses.append(N.train_step(latgen.net_noise(DIMS, 7000 + step), tgt, K, lr=3e-3))
    assert np.mean(losses[-10:]) < 0.8 * np.mean(losses[:10]), losses[::10]
    # held-out field
    S.set_gauge(latgen.make_links(DIMS, 0.4, 6301))
    tgt = make_targets(S, S.pack(latgen.make_init_fields(DIMS, K, 6302)), 3)
    res = {}
    for name, make in [("trained", lambda: N.forward(latgen.net_noise(DIMS, 6303))),
                       ("untrained", lambda: N0.forward(latgen.net_noise(DIMS, 6303))),
                       ("random", lambda: S.pack(latgen.make_init_fields(DIMS, 24, 6304)))]:
        for k in (0, 1):
            f = make()
            if k:
                make_targets(S, f, k)
            res[(name, k)] = binding.deficit_loss(S.ctx, f, 24, tgt, K, None)
    print("[deficits]", {f"{a}/k{b}": round(v, 4) for (a, b), v in res.items()}, flush=True)
    assert res[("trained", 0)] < res[("random", 0)]
    assert res[("trained", 0)] < res[("untrained", 0)]
    torch.cuda.synchronize()


@pytest.mark.parametrize("dims,blk", [((8, 8, 8, 16), (4, 4, 4, 4)), ((4, 4, 8, 32), (2, 2, 2, 4))])
@pytest.mark.parametrize("cin,cout", [(5, 7), (96, 37), (32, 576)])
def test_conv_both_paths(dims, blk, cin, cout):
    # a lattice whose x3 extent is a multiple of 32 runs the convolutions on
    # the matrix cores (32 sites per workgroup), one with L3 = 16 the vector
    # kernel: forward, activation and the input gradient against the oracle,
    # same tolerance as above
    say(f"conv {dims} {cin}->{cout}")
    s = Solver(dims, dfl_block=blk, sap_block=blk, Ns=2, nkv=2, little_nkv=2, m0=-0.2, nrhs_max=1)
    s.set_gauge(latgen.make_links(dims, 0.4, 6011))
    torch = s.torch
    V = int(np.prod(dims))
    rng = np.random.default_rng(cin * 7 + cout + dims[3])
    x = rng.standard_normal((V, cin))
    W = rng.standard_normal((3, 3, 3, 3, cin, cout)) / np.sqrt(81 * cin)
    b = rng.standard_normal(cout)
    g = rng.standard_normal((V, cout))
    zin = rng.standard_normal((V, cin))
    xd, Wd, bd = dev(x.T, torch), dev(W.reshape(81, cin, cout), torch), dev(b, torch)
    z = torch.empty(cout * V, dtype=torch.float32, device="cuda")
    a = torch.empty_like(z)
    binding.conv4d_forward(s.ctx, xd, cin, Wd, bd, cout, z, a)
    zr = onet.conv4d(x, W, b, dims)
    assert rel(z.cpu().numpy().reshape(cout, V).T, zr) < 2e-5
    assert rel(a.cpu().numpy().reshape(cout, V).T, onet.silu(zr)) < 2e-5
    dW = torch.empty_like(Wd)
    db = torch.empty_like(bd)
    din = torch.empty_like(xd)
    binding.conv4d_backward(s.ctx, xd, cin, Wd, cout, dev(g.T, torch), dW, db, din, dev(zin.T, torch))
    dxr, _, _ = onet.conv4d_backward(x, W, g, dims)
    assert rel(din.cpu().numpy().reshape(cin, V).T, dxr * onet.silu_grad(zin)) < 2e-5
    s.close()


def bf16_round(a):
    """Round to BF16 (nearest even) through FP32, as the device does with FP32 inputs."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("dims,blk", [((4, 4, 8, 32), (2, 2, 2, 4)), ((4, 4, 4, 64), (2, 2, 2, 4))])
@pytest.mark.parametrize("cin,cout", [(5, 7), (96, 37), (32, 576), (32, 32), (8, 33)])
def test_conv_forward_bf16(dims, blk, cin, cout):
    # BF16 operands, FP32 sums. Two checks per output:
    #  (1) against the exact FP64 map: |z - z_exact| <= (2u + u^2 + n 2^-24) sum|W||x| + 2^-24 |z|,
    #      u = 2^-8 the BF16 unit roundoff, n = 81 cin products (rounding of both operands,
    #      then FP32 summation in any order, then the FP32 bias add);
    #  (2) against the FP64 map of the BF16-rounded operands: only the FP32 summation error.
    say(f"conv bf16 {dims} {cin}->{cout}")
    s = Solver(dims, dfl_block=blk, sap_block=blk, Ns=2, nkv=2, little_nkv=2, m0=-0.2, nrhs_max=1)
    try:
        torch = s.torch
        V = int(np.prod(dims))
        rng = np.random.default_rng(cin * 11 + cout + dims[3])
        x = rng.standard_normal((V, cin))
        W = rng.standard_normal((3, 3, 3, 3, cin, cout)) / np.sqrt(81 * cin)
        b = rng.standard_normal(cout)
        xd, Wd, bd = dev(x.T, torch), dev(W.reshape(81, cin, cout), torch), dev(b, torch)
        z = torch.empty(cout * V, dtype=torch.float32, device="cuda")
        a = torch.empty_like(z)
        binding.conv4d_forward_bf16(s.ctx, xd, cin, Wd, bd, cout, z, a)
        zg = z.cpu().numpy().reshape(cout, V).T.astype(np.float64)
        ag = a.cpu().numpy().reshape(cout, V).T.astype(np.float64)
        x32, W32, b32 = (np.float32(v).astype(np.float64) for v in (x, W, b))
        n = 81 * cin
        scale = onet.conv4d(np.abs(x32), np.abs(W32), np.zeros(cout), dims)
        u = 2.0 ** -8
        exact = onet.conv4d(x32, W32, b32, dims)
        bound = (2 * u + u * u + n * 2.0 ** -24) * scale + 2.0 ** -24 * np.abs(exact) + 1e-30
        assert np.all(np.abs(zg - exact) <= bound), float(np.max(np.abs(zg - exact) / bound))
        rounded = onet.conv4d(bf16_round(x32), bf16_round(W32), b32, dims)
        tight = n * 2.0 ** -24 * scale * (1 + 2 * u) + 2.0 ** -24 * np.abs(rounded) + 1e-30
        assert np.all(np.abs(zg - rounded) <= tight), float(np.max(np.abs(zg - rounded) / tight))
        # the operands really are rounded (not an FP32 path)
        assert np.max(np.abs(zg - exact)) > 1e-5 * np.max(np.abs(exact))
        assert rel(ag, onet.silu(zg)) < 1e-6
    finally:
        s.close()


def test_conv_forward_bf16_refuses_other_lattices(S):
    say("conv bf16 lattice check")
    torch = S.torch
    x = torch.zeros(4 * V, dtype=torch.float32, device="cuda")
    W = torch.zeros(81 * 4 * 4, dtype=torch.float32, device="cuda")
    z = torch.empty(4 * V, dtype=torch.float32, device="cuda")
    with pytest.raises(binding.DflError):
        binding.conv4d_forward_bf16(S.ctx, x, 4, W, None, 4, z, None)  # L3 = 8
