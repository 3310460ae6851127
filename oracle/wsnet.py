"""Plain FP64 reference of the warm-start network: a 3-D convolutional
encoder-decoder, conditioned on (log Ra, Pr), that maps a side-heated cavity's
parameters to its steady (u/U, v/U, w/U, T/dT) fields on an M^3 grid.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the reference the HIP
network kernels and their gradients are compared against.  Nothing here is
shared with the GPU library.  The network is not part of the paper; it is the
learned initial guess for runs whose convergence the paper's steady-state
criterion (Sec. 3) decides.  Every operation is its plain definition: zero-padded 3x3x3
cross-correlation as 27 shifted matrix products, FiLM as an affine map per
channel, SiLU, injection and linear interpolation between grid levels, the
mean squared error, and Adam (Kingma & Ba 2015, Algorithm 1).  Backward passes
are the adjoints of the forward maps, written out; ``tests/`` pins them against
brute-force loops, dot-product (adjoint) identities and central finite
differences.

Arrays are channels-last: activations [B, D, H, W, C] (z, y, x, channel);
weights [27, Cin, Cout] with tap t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1) reading
the input at (z + dz, y + dy, x + dx).
"""
import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
N_IN = 8        # input feature channels
N_OUT = 8       # output channels, the first 4 are (u/U, v/U, w/U, T/dT)
N_FIELDS = 4


# ---------------------------------------------------------------------------
# Convolution and its adjoints
# ---------------------------------------------------------------------------
def _pad(X):
    return np.pad(X, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))


def _window(P, dz, dy, dx, D, H, W):
    return P[:, 1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :]


def conv3d(X, Wt):
    """Z[b, v, co] = sum_t sum_ci X[b, v + off_t, ci] Wt[t, ci, co] (zero outside)."""
    B, D, H, W, _ = X.shape
    P = _pad(np.asarray(X, dtype=np.float64))
    Z = np.zeros((B, D, H, W, Wt.shape[2]))
    for t, (dz, dy, dx) in enumerate(TAPS):
        Z += _window(P, dz, dy, dx, D, H, W) @ Wt[t]
    return Z


def conv3d_bwd_data(dZ, Wt):
    """Adjoint of conv3d in X: dX[b, u, ci] = sum_t sum_co dZ[b, u - off_t, co] Wt[t, ci, co]."""
    B, D, H, W, _ = dZ.shape
    P = _pad(np.asarray(dZ, dtype=np.float64))
    dX = np.zeros((B, D, H, W, Wt.shape[1]))
    for t, (dz, dy, dx) in enumerate(TAPS):
        dX += _window(P, -dz, -dy, -dx, D, H, W) @ Wt[t].T
    return dX


def conv3d_bwd_weight(X, dZ):
    """Adjoint of conv3d in Wt: dWt[t, ci, co] = sum_b sum_v X[b, v + off_t, ci] dZ[b, v, co].
    X may have batch 1 and is then shared by every sample of dZ."""
    B, D, H, W, Co = dZ.shape
    X = np.broadcast_to(np.asarray(X, dtype=np.float64), (B, D, H, W, X.shape[-1]))
    P = _pad(X)
    dW = np.zeros((27, X.shape[-1], Co))
    G = dZ.reshape(-1, Co)
    for t, (dz, dy, dx) in enumerate(TAPS):
        dW[t] = _window(P, dz, dy, dx, D, H, W).reshape(-1, X.shape[-1]).T @ G
    return dW


# ---------------------------------------------------------------------------
# Grid levels: M -> (M + 1) / 2 by injection, back by linear interpolation
# ---------------------------------------------------------------------------
def restrict(X):
    """Coarse node i is fine node 2i (per axis)."""
    return X[:, ::2, ::2, ::2, :]


def restrict_adj(G, fine):
    out = np.zeros(fine[:4] + (G.shape[-1],))
    out[:, ::2, ::2, ::2, :] = G
    return out


def _interp_matrix(n):
    """(2n - 1) x n matrix of 1-D linear interpolation: fine 2i = coarse i,
    fine 2i + 1 = (coarse i + coarse i + 1) / 2."""
    P = np.zeros((2 * n - 1, n))
    for i in range(n):
        P[2 * i, i] = 1.0
    for i in range(n - 1):
        P[2 * i + 1, i] = 0.5
        P[2 * i + 1, i + 1] = 0.5
    return P


def prolong(X):
    """Trilinear (tensor-product linear) interpolation to 2n - 1 nodes per axis."""
    Pz, Py, Px = (_interp_matrix(n) for n in X.shape[1:4])
    return np.einsum("zk,yj,xi,bkjic->bzyxc", Pz, Py, Px, X)


def prolong_adj(G, coarse):
    Pz, Py, Px = (_interp_matrix(n) for n in coarse[1:4])
    return np.einsum("zk,yj,xi,bzyxc->bkjic", Pz, Py, Px, G)


# ---------------------------------------------------------------------------
# Pointwise pieces
# ---------------------------------------------------------------------------
def sigmoid(y):
    return 0.5 * (1.0 + np.tanh(0.5 * y))


def silu(y):
    return y * sigmoid(y)


def silu_grad(y):
    s = sigmoid(y)
    return s * (1.0 + y * (1.0 - s))


def film(cond, Gw, Gb, Bw, Bb):
    """Per-sample channel scale 1 + cond Gw^T + Gb and shift cond Bw^T + Bb."""
    return 1.0 + cond @ Gw.T + Gb, cond @ Bw.T + Bb


def features(M):
    """Input features on the node-centred M^3 grid, (i + 1/2) / M per axis:
    (2x - 1, 2y - 1, 2z - 1, its squares, distance to the nearest wall, 1)."""
    c = (np.arange(M) + 0.5) / M
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    d = np.minimum.reduce([x, 1 - x, y, 1 - y, z, 1 - z])
    X = np.stack([2 * x - 1, 2 * y - 1, 2 * z - 1, (2 * x - 1) ** 2, (2 * y - 1) ** 2,
                  (2 * z - 1) ** 2, d, np.ones_like(x)], axis=-1)
    return X[None]


def condition(Ra, Pr):
    """Conditioning vector: (log10 Ra - 5.5) / 1.5 and (Pr - 3.855) / 3.145,
    both in [-1, 1] over Ra in [1e4, 1e7] and Pr in [0.71, 7]."""
    Ra = np.atleast_1d(np.asarray(Ra, dtype=np.float64))
    Pr = np.atleast_1d(np.asarray(Pr, dtype=np.float64))
    return np.stack([(np.log10(Ra) - 5.5) / 1.5, (Pr - 3.855) / 3.145], axis=-1)


# ---------------------------------------------------------------------------
# The network
# ---------------------------------------------------------------------------
def layers(ch=(16, 32, 64)):
    """(name, Cin, Cout, level, film) of every convolution, in parameter order.
    Encoder: two convolutions per level, injection between levels.  Decoder:
    interpolate up, concatenate [upsampled, skip], one convolution per level.
    The output convolution has a bias and no FiLM or activation."""
    c1, c2, c3 = ch
    return [("E1a", N_IN, c1, 0, True), ("E1b", c1, c1, 0, True),
            ("E2a", c1, c2, 1, True), ("E2b", c2, c2, 1, True),
            ("E3a", c2, c3, 2, True), ("E3b", c3, c3, 2, True),
            ("D2", c3 + c2, c2, 1, True), ("D1", c2 + c1, c1, 0, True),
            ("OUT", c1, N_OUT, 0, False)]


def param_shapes(ch=(16, 32, 64)):
    """[(name, shape)] in the flat parameter order: per layer W [27, Cin, Cout],
    then Gw [Cout, 2], Gb [Cout], Bw [Cout, 2], Bb [Cout] (FiLM layers) or
    b [Cout] (the output layer)."""
    out = []
    for name, ci, co, _, fl in layers(ch):
        out.append((name + ".W", (27, ci, co)))
        if fl:
            out += [(name + ".Gw", (co, 2)), (name + ".Gb", (co,)),
                    (name + ".Bw", (co, 2)), (name + ".Bb", (co,))]
        else:
            out.append((name + ".b", (co,)))
    return out


def unflatten(flat, ch=(16, 32, 64)):
    p, o = {}, 0
    for name, shp in param_shapes(ch):
        n = int(np.prod(shp))
        p[name] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    assert o == len(flat)
    return p


def flatten(p, ch=(16, 32, 64)):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1)
                           for name, _ in param_shapes(ch)])


def forward(p, cond, M, ch=(16, 32, 64), X0=None, rnd=None):
    """Network output [B, M, M, M, 8] for conditioning rows cond [B, 2], and
    the cache the backward pass needs.  With rnd (e.g. bf16_round) every
    convolution operand (input activation and weights) and every stored
    activation is passed through rnd, as reduced-precision kernels store them;
    rnd=None is the exact network."""
    rnd = rnd or (lambda a: a)
    cond = np.atleast_2d(np.asarray(cond, dtype=np.float64))
    X0 = rnd(features(M) if X0 is None else X0)
    cache = {"cond": cond, "X0": X0, "rnd": rnd}

    def block(name, X):
        Z = conv3d(X, rnd(p[name + ".W"]))
        sc, sh = film(cond, p[name + ".Gw"], p[name + ".Gb"], p[name + ".Bw"], p[name + ".Bb"])
        Y = Z * sc[:, None, None, None, :] + sh[:, None, None, None, :]
        cache[name] = (X, Z, Y, sc)
        return rnd(silu(Y))

    a = block("E1a", X0)
    s1 = block("E1b", a)
    a = block("E2a", restrict(s1))
    s2 = block("E2b", a)
    a = block("E3a", restrict(s2))
    s3 = block("E3b", a)
    a = block("D2", np.concatenate([rnd(prolong(s3)), s2], axis=-1))
    a = block("D1", np.concatenate([rnd(prolong(a)), s1], axis=-1))
    out = conv3d(a, rnd(p["OUT.W"])) + p["OUT.b"]
    cache["OUT"] = a
    cache["shapes"] = (s1.shape, s2.shape, s3.shape)
    return out, cache


def backward(p, cache, dout, ch=(16, 32, 64)):
    """Gradients of a scalar loss with respect to every parameter, given the
    loss's gradient dout [B, M, M, M, 8] with respect to the output.  With the
    forward pass's rnd, the convolution operands of the backward pass (the
    output gradient, each dZ, the weights) are rounded the same way."""
    cond = cache["cond"]
    rnd = cache["rnd"]
    g = {}
    c1, c2, c3 = ch
    s1s, s2s, s3s = cache["shapes"]
    a = cache["OUT"]
    dr = rnd(dout)
    g["OUT.W"] = conv3d_bwd_weight(a, dr)
    g["OUT.b"] = dout.sum(axis=(0, 1, 2, 3))
    da = conv3d_bwd_data(dr, rnd(p["OUT.W"]))

    def block_bwd(name, da, need_dx=True):
        X, Z, Y, sc = cache[name]
        dY = da * silu_grad(Y)
        dsc = (dY * Z).sum(axis=(1, 2, 3))          # [B, Cout]
        dsh = dY.sum(axis=(1, 2, 3))
        g[name + ".Gw"] = dsc.T @ cond
        g[name + ".Gb"] = dsc.sum(axis=0)
        g[name + ".Bw"] = dsh.T @ cond
        g[name + ".Bb"] = dsh.sum(axis=0)
        dZ = rnd(dY * sc[:, None, None, None, :])
        g[name + ".W"] = conv3d_bwd_weight(X, dZ)
        return conv3d_bwd_data(dZ, rnd(p[name + ".W"])) if need_dx else None

    dX = block_bwd("D1", da)                        # [.., c2 + c1]
    ds1 = dX[..., c2:].copy()
    da = prolong_adj(dX[..., :c2], s2s)
    dX = block_bwd("D2", da)                        # [.., c3 + c2]
    ds2 = dX[..., c3:].copy()
    da = prolong_adj(dX[..., :c3], s3s)
    da = block_bwd("E3b", da)
    da = block_bwd("E3a", da)
    ds2 += restrict_adj(da, s2s)
    da = block_bwd("E2b", ds2)
    da = block_bwd("E2a", da)
    ds1 += restrict_adj(da, s1s)
    da = block_bwd("E1b", ds1)
    block_bwd("E1a", da, need_dx=False)
    return g


def mse(out, target):
    """Mean squared error over the 4 field channels and its gradient."""
    diff = out[..., :N_FIELDS] - target
    n = diff.size
    dout = np.zeros_like(out)
    dout[..., :N_FIELDS] = 2.0 * diff / n
    return float((diff ** 2).sum() / n), dout


def adam(param, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns the new (param, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return param - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a):
    """Round values to FP32, then to the nearest bfloat16 (ties to even),
    returned as FP64: the operands the MFMA kernels see."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def upsample_fields(pred, M, N, cell, U, T_hot, T_cold, symmetrize=False):
    """Fields on the node-centred M^3 grid (pred [M, M, M, >=4]: u/U, v/U, w/U,
    T*) trilinearly interpolated at the N^3 lattice nodes (i + 1/2)/N, in
    lattice units, [4, N, N, N].  Per axis the samples are the M nodes and,
    half a spacing beyond the outermost ones, the walls: velocity 0 on every
    wall; T* = +1/2 at the low and -1/2 at the high isothermal wall (axis x
    for side-heated, cell 0; z for Rayleigh-Benard), the nearest node's T*
    across an adiabatic wall.  With symmetrize (side-heated only) the result
    is averaged over the cell's symmetries: the half-turn about the y axis
    through the centre, (x, z) -> (1 - x, 1 - z) with (u, w, T*) -> -(u, w, T*),
    and the mirror y -> 1 - y with v -> -v."""
    ext = np.zeros((M + 2,) * 3 + (4,))
    ext[1:-1, 1:-1, 1:-1] = pred[..., :4]
    # temperature beyond adiabatic walls: the nearest node (edges and corners too)
    T = np.pad(pred[..., 3], 1, mode="edge")
    iso = 2 if cell == 0 else 0                   # array axis of the isothermal walls (z, y, x order)
    lo = [slice(None)] * 3
    hi = [slice(None)] * 3
    lo[iso], hi[iso] = 0, M + 1
    T[tuple(lo)] = 0.5
    T[tuple(hi)] = -0.5
    ext[..., 3] = T
    # sample positions in units of the node spacing, with the walls at -1/2 and M - 1/2
    pos = [-0.5] + list(range(M)) + [M - 0.5]
    s = (np.arange(N) + 0.5) / N * M - 0.5
    idx = np.clip(np.searchsorted(pos, s, side="right") - 1, 0, M)
    w = (s - np.take(pos, idx)) / (np.take(pos, idx + 1) - np.take(pos, idx))
    out = np.zeros((4, N, N, N))
    for cz in (0, 1):
        wz = w if cz else 1 - w
        for cy in (0, 1):
            wy = w if cy else 1 - w
            for cx in (0, 1):
                wx = w if cx else 1 - w
                vals = ext[np.ix_(idx + cz, idx + cy, idx + cx)]          # [N, N, N, 4]
                wt = wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
                out += np.moveaxis(vals, -1, 0) * wt[None]
    if symmetrize and cell == 0:
        turn = np.array([-1.0, 1.0, -1.0, -1.0])[:, None, None, None] * out[:, ::-1, :, ::-1]
        mirror = np.array([1.0, -1.0, 1.0, 1.0])[:, None, None, None] * out[:, :, ::-1, :]
        both = np.array([-1.0, -1.0, -1.0, -1.0])[:, None, None, None] * out[:, ::-1, ::-1, ::-1]
        out = 0.25 * (out + turn + mirror + both)
    Tm, dT = 0.5 * (T_hot + T_cold), T_hot - T_cold
    out[:3] *= U
    out[3] = Tm + dT * out[3]
    return out
