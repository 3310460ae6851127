"""Pins of the FP64 warm-start network reference (oracle/wsnet.py) against
what the mathematics fixes: brute-force loops, exact special cases, adjoint
(dot-product) identities, exact reproduction of trilinear functions, central
finite differences of the whole network's loss, and Adam's closed form."""
import itertools

import numpy as np
import pytest

from oracle import wsnet as W


def rng(seed):
    return np.random.default_rng(seed)


def brute_conv(X, Wt):
    B, D, H, Wd, Ci = X.shape
    Co = Wt.shape[2]
    Z = np.zeros((B, D, H, Wd, Co))
    for b, z, y, x in itertools.product(range(B), range(D), range(H), range(Wd)):
        for kz, ky, kx in itertools.product(range(3), range(3), range(3)):
            zz, yy, xx = z + kz - 1, y + ky - 1, x + kx - 1
            if 0 <= zz < D and 0 <= yy < H and 0 <= xx < Wd:
                t = 9 * kz + 3 * ky + kx
                for ci in range(Ci):
                    Z[b, z, y, x, :] += X[b, zz, yy, xx, ci] * Wt[t, ci, :]
    return Z


def test_conv_matches_brute_force_loops():
    r = rng(1)
    X = r.standard_normal((2, 3, 4, 5, 3))
    Wt = r.standard_normal((27, 3, 2))
    assert np.allclose(W.conv3d(X, Wt), brute_conv(X, Wt), rtol=0, atol=1e-12)


def test_conv_special_cases_identity_and_shift():
    r = rng(2)
    X = r.standard_normal((1, 4, 5, 6, 2))
    Wt = np.zeros((27, 2, 2))
    Wt[13] = np.eye(2)                               # centre tap
    assert np.array_equal(W.conv3d(X, Wt), X)
    Wt = np.zeros((27, 2, 2))
    Wt[9 * 1 + 3 * 1 + 2] = np.eye(2)                # reads x + 1
    Z = W.conv3d(X, Wt)
    assert np.array_equal(Z[:, :, :, :-1], X[:, :, :, 1:])
    assert not Z[:, :, :, -1].any()
    Wt = np.zeros((27, 2, 2))
    Wt[0] = np.eye(2)                                # reads (z - 1, y - 1, x - 1)
    Z = W.conv3d(X, Wt)
    assert np.array_equal(Z[:, 1:, 1:, 1:], X[:, :-1, :-1, :-1])
    assert not Z[:, 0].any() and not Z[:, :, 0].any() and not Z[:, :, :, 0].any()


@pytest.mark.parametrize("shared", [False, True])
def test_conv_adjoints_dot_product_identity(shared):
    r = rng(3)
    B = 3
    X = r.standard_normal((1 if shared else B, 4, 3, 5, 4))
    Wt = r.standard_normal((27, 4, 6))
    G = r.standard_normal((B, 4, 3, 5, 6))
    Xb = np.broadcast_to(X, (B,) + X.shape[1:])
    lhs = np.sum(W.conv3d(Xb, Wt) * G)
    assert np.isclose(lhs, np.sum(Xb * W.conv3d_bwd_data(G, Wt)), rtol=1e-12)
    assert np.isclose(lhs, np.sum(Wt * W.conv3d_bwd_weight(X, G)), rtol=1e-12)


def test_bwd_data_matches_brute_force_transpose():
    """dX[u] = sum over outputs v reading u: built from the forward loop's
    transpose, one unit vector at a time."""
    r = rng(4)
    Wt = r.standard_normal((27, 2, 3))
    shp = (1, 3, 3, 4, 2)
    G = r.standard_normal((1, 3, 3, 4, 3))
    dX = W.conv3d_bwd_data(G, Wt)
    for idx in [(0, 0, 0, 0, 0), (0, 1, 2, 3, 1), (0, 2, 1, 0, 0), (0, 1, 1, 2, 1)]:
        e = np.zeros(shp)
        e[idx] = 1.0
        assert np.isclose(dX[idx], np.sum(brute_conv(e, Wt) * G), rtol=1e-12)


def test_prolong_reproduces_trilinear_functions_exactly():
    n = 5
    c = np.arange(n, dtype=np.float64)                 # coarse node i sits at fine 2i
    f = lambda z, y, x: 1.5 - 0.25 * x + 2 * y - z + 0.5 * x * y - 0.75 * y * z + 0.125 * x * y * z
    zc, yc, xc = np.meshgrid(2 * c, 2 * c, 2 * c, indexing="ij")
    coarse = f(zc, yc, xc)[None, ..., None]
    fz = np.arange(2 * n - 1, dtype=np.float64)
    zf, yf, xf = np.meshgrid(fz, fz, fz, indexing="ij")
    assert np.allclose(W.prolong(coarse)[0, ..., 0], f(zf, yf, xf), rtol=0, atol=1e-12)
    # and restriction picks the coarse nodes back
    assert np.array_equal(W.restrict(W.prolong(coarse)), coarse)


def test_level_maps_adjoint_identities():
    r = rng(5)
    fine = (2, 9, 9, 9, 3)
    coarse = (2, 5, 5, 5, 3)
    A, Gc = r.standard_normal(fine), r.standard_normal(coarse)
    assert np.isclose(np.sum(W.restrict(A) * Gc), np.sum(A * W.restrict_adj(Gc, fine)), rtol=1e-12)
    C, Gf = r.standard_normal(coarse), r.standard_normal(fine)
    assert np.isclose(np.sum(W.prolong(C) * Gf), np.sum(C * W.prolong_adj(Gf, coarse)), rtol=1e-12)


def test_silu_and_its_derivative():
    y = np.linspace(-6, 6, 97)
    h = 1e-6
    fd = (W.silu(y + h) - W.silu(y - h)) / (2 * h)
    assert np.allclose(W.silu_grad(y), fd, rtol=0, atol=1e-9)
    assert W.silu(0.0) == 0.0 and np.isclose(W.silu_grad(0.0), 0.5)
    assert np.allclose(W.silu(y) - W.silu(-y), y)   # silu(y) - silu(-y) = y


def test_features_and_condition():
    M = 5
    X = W.features(M)[0]
    assert X.shape == (M, M, M, W.N_IN)
    assert np.isclose(X[0, 0, 0, 6], 0.5 / M) and np.isclose(X[2, 2, 2, 6], 0.5)
    assert np.allclose(X[..., 0][2, 2], 2 * (np.arange(M) + 0.5) / M - 1)
    assert np.allclose(X[..., 3], X[..., 0] ** 2) and np.all(X[..., 7] == 1)
    assert np.allclose(W.condition([1e4, 1e7], [0.71, 7.0]), [[-1, -1], [1, 1]])


def small_net(seed, ch=(2, 3, 4), M=9, B=2):
    r = rng(seed)
    # weights at the He scale keep every pre-activation O(1), so the finite
    # differences are not swamped by rounding of a huge loss
    p = {name: (np.sqrt(2.0 / (27 * shp[1])) if name.endswith(".W") else 0.3)
         * r.standard_normal(shp) for name, shp in W.param_shapes(ch)}
    cond = r.uniform(-1, 1, (B, 2))
    target = 0.3 * r.standard_normal((B, M, M, M, W.N_FIELDS))
    return p, cond, target


def loss_of(p, cond, target, ch, M):
    out, _ = W.forward(p, cond, M, ch)
    return W.mse(out, target)[0]


def test_whole_network_gradient_matches_central_differences():
    ch, M = (2, 3, 4), 9
    p, cond, target = small_net(6, ch, M)
    out, cache = W.forward(p, cond, M, ch)
    L, dout = W.mse(out, target)
    g = W.backward(p, cache, dout, ch)
    assert set(g) == {name for name, _ in W.param_shapes(ch)}
    r = rng(7)
    h = 1e-5
    checked = 0
    for name, shp in W.param_shapes(ch):
        for _ in range(3):
            idx = tuple(r.integers(0, s) for s in shp)
            old = p[name][idx]
            p[name][idx] = old + h
            lp = loss_of(p, cond, target, ch, M)
            p[name][idx] = old - h
            lm = loss_of(p, cond, target, ch, M)
            p[name][idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(g[name][idx] - fd) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (name, idx, g[name][idx], fd)
            checked += 1
    assert checked == 3 * len(W.param_shapes(ch))


def test_flat_parameter_order_round_trips():
    ch = (2, 3, 4)
    p, _, _ = small_net(8, ch)
    flat = W.flatten(p, ch)
    assert flat.size == sum(int(np.prod(s)) for _, s in W.param_shapes(ch))
    q = W.unflatten(flat, ch)
    assert all(np.array_equal(p[k], q[k]) for k in p)


def test_adam_closed_form_first_two_steps():
    g1, g2 = np.array([0.5, -2.0, 1e-3]), np.array([-0.5, 1.0, 3e-3])
    p0 = np.array([1.0, 2.0, 3.0])
    lr, eps = 1e-2, 1e-8
    p1, m, v = W.adam(p0, g1, 0 * p0, 0 * p0, 1, lr, eps=eps)
    assert np.allclose(p1, p0 - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    p2, m, v = W.adam(p1, g2, m, v, 2, lr, eps=eps)
    mh = (0.9 * 0.1 * g1 + 0.1 * g2) / (1 - 0.81)
    vh = (0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2) / (1 - 0.999 ** 2)
    assert np.allclose(p2, p1 - lr * mh / (np.sqrt(vh) + eps), rtol=0, atol=1e-15)


def test_bf16_rounding_ties_to_even():
    one = 1.0
    vals = np.array([one, one + 2.0 ** -8, one + 3 * 2.0 ** -8, one + 2.0 ** -7, -3.0, 0.0,
                     one + 2.0 ** -8 + 2.0 ** -20])
    want = np.array([one, one, one + 2.0 ** -6, one + 2.0 ** -7, -3.0, 0.0, one + 2.0 ** -7])
    assert np.array_equal(W.bf16_round(vals), want)


def test_upsample_same_grid_is_identity_in_lattice_units():
    r = rng(9)
    M = 5
    pred = r.standard_normal((M, M, M, 8))
    out = W.upsample_fields(pred, M, M, 0, U=0.05, T_hot=0.5, T_cold=-0.5)
    assert np.allclose(out[:3], 0.05 * np.moveaxis(pred[..., :3], -1, 0), rtol=0, atol=1e-15)
    assert np.allclose(out[3], pred[..., 3], rtol=0, atol=1e-15)


def test_upsample_interior_reproduces_trilinear_and_walls_anchor():
    M, N = 6, 13
    c = (np.arange(M) + 0.5) / M
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    f = 0.3 + 0.2 * x - 0.1 * y + 0.4 * z + 0.7 * x * y * z
    pred = np.zeros((M, M, M, 4))
    pred[..., 0] = f
    pred[..., 3] = f
    out = W.upsample_fields(pred, M, N, 0, U=1.0, T_hot=0.5, T_cold=-0.5)
    q = (np.arange(N) + 0.5) / N
    inside = (q >= c[0]) & (q <= c[-1])
    zq, yq, xq = np.meshgrid(q, q, q, indexing="ij")
    fq = 0.3 + 0.2 * xq - 0.1 * yq + 0.4 * zq + 0.7 * xq * yq * zq
    m = np.ix_(inside, inside, inside)
    assert np.allclose(out[0][m], fq[m], rtol=0, atol=1e-13)
    assert np.allclose(out[3][m], fq[m], rtol=0, atol=1e-13)
    # the first lattice node of an M = 2 grid sampled at N = 4 sits halfway
    # between the wall and node 0: u is half the node value, T half the hot
    # wall's +1/2 plus half the node value along x, the node value along y
    pred = np.ones((2, 2, 2, 4))
    out = W.upsample_fields(pred, 2, 4, 0, U=1.0, T_hot=0.5, T_cold=-0.5)
    assert np.isclose(out[0][1, 1, 0], 0.5)                  # x wall only
    assert np.isclose(out[0][1, 0, 1], 0.5)                  # y wall only
    assert np.isclose(out[3][1, 1, 0], 0.5 * 0.5 + 0.5)      # isothermal x wall
    assert np.isclose(out[3][1, 1, 3], 0.5 * -0.5 + 0.5)     # cold wall
    assert np.isclose(out[3][1, 0, 1], 1.0)                  # adiabatic y wall
    # Rayleigh-Benard: z walls isothermal, x adiabatic
    out = W.upsample_fields(pred, 2, 4, 1, U=1.0, T_hot=0.5, T_cold=-0.5)
    assert np.isclose(out[3][0, 1, 1], 0.75) and np.isclose(out[3][1, 1, 0], 1.0)


def test_upsample_symmetrized_is_invariant_and_keeps_symmetric_fields():
    r = rng(10)
    M, N = 6, 11
    pred = r.standard_normal((M, M, M, 4))
    out = W.upsample_fields(pred, M, N, 0, U=1.0, T_hot=0.5, T_cold=-0.5, symmetrize=True)
    # invariant under the half-turn about y (T* odd) and the y mirror (v odd)
    turn = np.array([-1.0, 1.0, -1.0, -1.0])[:, None, None, None] * out[:, ::-1, :, ::-1]
    mirror = np.array([1.0, -1.0, 1.0, 1.0])[:, None, None, None] * out[:, :, ::-1, :]
    assert np.allclose(turn, out, rtol=0, atol=1e-14) and np.allclose(mirror, out, rtol=0, atol=1e-14)
    assert abs(out[3].mean()) < 1e-14                       # the mean temperature is removed
    # a prediction that already has the symmetries is left as it was
    p = pred.copy()
    p = 0.5 * (p + np.array([-1.0, 1.0, -1.0, -1.0]) * p[::-1, :, ::-1])
    p = 0.5 * (p + np.array([1.0, -1.0, 1.0, 1.0]) * p[:, ::-1, :])
    a = W.upsample_fields(p, M, N, 0, U=1.0, T_hot=0.5, T_cold=-0.5, symmetrize=True)
    b = W.upsample_fields(p, M, N, 0, U=1.0, T_hot=0.5, T_cold=-0.5)
    assert np.allclose(a, b, rtol=0, atol=1e-14)
