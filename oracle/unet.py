"""Network of the learned coarse-grid correction: plain FP64 forward and
backward passes (test infrastructure; only the tests and the benchmark's CPU
baseline use this package).

The network has no counterpart in the paper: it is the coarse-solver slot
of Alg. 2 filled by a learned map r_c -> e_c ~ A_c^{-1} r_c, trained on the
method's own exact coarse solves.  Definition (the one the library states):

  grid G^3 (G a multiple of 8), samples as arrays [B, z, y, x, c]
  (x fastest, channels last), 3x3x3 convolutions with zero padding, tap
  t = (dx+1) + 3 (dy+1) + 9 (dz+1) reads the point (x+dx, y+dy, z+dz);
  L0 2->16, L1 16->16 (G); pool; L2 16->32 (G/2); pool; L3 32->48 (G/4);
  pool; L4 48->48 (G/8); up + a3; L5 48->32; up + a2; L6 32->16;
  up + a1; L7 16->1 (linear); ReLU after L0..L6; pool = 2x2x2 mean;
  up = nearest-neighbour copy to the 8 children.
  Parameters packed per layer as w[cout][27][cin], then b[cout].
  Loss: mean over the points whose mask (input channel 1) is set of
  (out - target)^2, over all samples.

parity unpinned: the network itself is not in the paper; its oracle is pinned
by finite differences, adjointness and a library correlation instead.

round_bf16 emulates the BF16 rounding of the GPU kernels' matrix-core
operands (round to nearest even) so that both sides can be compared with the
same operand precision.
"""
import numpy as np

LAYERS = [(2, 16, 0, True), (16, 16, 0, True), (16, 32, 1, True), (32, 48, 2, True),
          (48, 48, 3, True), (48, 32, 2, True), (32, 16, 1, True), (16, 1, 0, False)]


def n_params():
    return sum(co * 27 * ci + co for ci, co, _, _ in LAYERS)


def unpack(theta):
    """Parameter vector -> list of (w [cout, 27, cin], b [cout])."""
    out, o = [], 0
    for ci, co, _, _ in LAYERS:
        w = np.asarray(theta[o:o + co * 27 * ci], dtype=np.float64).reshape(co, 27, ci)
        o += co * 27 * ci
        b = np.asarray(theta[o:o + co], dtype=np.float64)
        o += co
        out.append((w, b))
    return out


def pack(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def round_bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = np.where(nan, (u | 0x400000) & 0xFFFF0000, r).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _shift(x, dx, dy, dz):
    """x[b, z+dz, y+dy, x+dx, c] with zeros outside the grid."""
    B, g = x.shape[0], x.shape[1]
    p = np.zeros((B, g + 2, g + 2, g + 2, x.shape[4]))
    p[:, 1:-1, 1:-1, 1:-1] = x
    return p[:, 1 + dz:1 + dz + g, 1 + dy:1 + dy + g, 1 + dx:1 + dx + g]


def taps():
    for t in range(27):
        yield t, t % 3 - 1, (t // 3) % 3 - 1, t // 9 - 1


def conv(x, w, b=None, bf16=False):
    """y[.., co] = sum_t sum_ci x[neighbour t, ci] w[co, t, ci] + b[co]."""
    if bf16:
        x, w = round_bf16(x), round_bf16(w)
    y = np.zeros(x.shape[:4] + (w.shape[0],))
    for t, dx, dy, dz in taps():
        y += _shift(x, dx, dy, dz) @ w[:, t, :].T
    return y if b is None else y + b


def conv_grads(x, dz, w, need_dx=True, bf16=False):
    """Gradients of conv with respect to w, b and x for the upstream dz."""
    if bf16:
        xr, dzr, wr = round_bf16(x), round_bf16(dz), round_bf16(w)
    else:
        xr, dzr, wr = x, dz, w
    gw = np.zeros_like(w)
    dx = np.zeros_like(x) if need_dx else None
    D = dzr.reshape(-1, dz.shape[4])
    for t, ddx, ddy, ddz in taps():
        gw[:, t, :] = D.T @ _shift(xr, ddx, ddy, ddz).reshape(-1, x.shape[4])
        if need_dx:
            # d x[q] += sum_co dz[q - o_t, co] w[co, t, ci]
            dx += _shift(dzr, -ddx, -ddy, -ddz) @ wr[:, t, :]
    gb = dz.reshape(-1, dz.shape[4]).sum(axis=0)
    return gw, gb, dx


def pool(x):
    B, g, c = x.shape[0], x.shape[1], x.shape[4]
    return x.reshape(B, g // 2, 2, g // 2, 2, g // 2, 2, c).mean(axis=(2, 4, 6))


def pool_bwd(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, 1), 2, 2), 2, 3) / 8.0


def up(a):
    return np.repeat(np.repeat(np.repeat(a, 2, 1), 2, 2), 2, 3)


def up_bwd(du):
    B, g, c = du.shape[0], du.shape[1], du.shape[4]
    return du.reshape(B, g // 2, 2, g // 2, 2, g // 2, 2, c).sum(axis=(2, 4, 6))


def relu(x):
    return np.maximum(x, 0.0)


def forward(theta, inp, bf16=False):
    """inp [B, G, G, G, 2] -> (out [B, G, G, G], cache)."""
    P = unpack(theta)
    c = {"in": inp}
    c["a0"] = relu(conv(inp, *P[0], bf16=bf16))
    c["a1"] = relu(conv(c["a0"], *P[1], bf16=bf16))
    c["p1"] = pool(c["a1"])
    c["a2"] = relu(conv(c["p1"], *P[2], bf16=bf16))
    c["p2"] = pool(c["a2"])
    c["a3"] = relu(conv(c["p2"], *P[3], bf16=bf16))
    c["p3"] = pool(c["a3"])
    c["a4"] = relu(conv(c["p3"], *P[4], bf16=bf16))
    c["u3"] = up(c["a4"]) + c["a3"]
    c["a5"] = relu(conv(c["u3"], *P[5], bf16=bf16))
    c["u2"] = up(c["a5"]) + c["a2"]
    c["a6"] = relu(conv(c["u2"], *P[6], bf16=bf16))
    c["u1"] = up(c["a6"]) + c["a1"]
    out = conv(c["u1"], *P[7], bf16=bf16)[..., 0]
    return out, c


def loss(out, target, inp):
    m = inp[..., 1]
    d = m * (out - target)
    return float((d * d).sum() / m.astype(bool).sum())


def backward(theta, inp, target, bf16=False):
    """(loss, gradient vector packed like theta)."""
    P = unpack(theta)
    out, c = forward(theta, inp, bf16)
    m = inp[..., 1]
    count = m.astype(bool).sum()
    d = m * (out - target)
    L = float((d * d).sum() / count)
    g = [None] * 8
    dz = (2.0 * d / count)[..., None]
    g[7] = conv_grads(c["u1"], dz, P[7][0], bf16=bf16)
    du1 = g[7][2]
    da6 = up_bwd(du1) * (c["a6"] > 0)
    g[6] = conv_grads(c["u2"], da6, P[6][0], bf16=bf16)
    du2 = g[6][2]
    da5 = up_bwd(du2) * (c["a5"] > 0)
    g[5] = conv_grads(c["u3"], da5, P[5][0], bf16=bf16)
    du3 = g[5][2]
    da4 = up_bwd(du3) * (c["a4"] > 0)
    g[4] = conv_grads(c["p3"], da4, P[4][0], bf16=bf16)
    da3 = (du3 + pool_bwd(g[4][2])) * (c["a3"] > 0)
    g[3] = conv_grads(c["p2"], da3, P[3][0], bf16=bf16)
    da2 = (du2 + pool_bwd(g[3][2])) * (c["a2"] > 0)
    g[2] = conv_grads(c["p1"], da2, P[2][0], bf16=bf16)
    da1 = (du1 + pool_bwd(g[2][2])) * (c["a1"] > 0)
    g[1] = conv_grads(c["a0"], da1, P[1][0], bf16=bf16)
    da0 = g[1][2] * (c["a0"] > 0)
    g[0] = conv_grads(inp, da0, P[0][0], need_dx=False, bf16=bf16)
    return L, pack([(gw, gb) for gw, gb, _ in g])


def adam(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba 2015, Alg. 1, bias-corrected step size)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    lr_t = lr * np.sqrt(1 - b2 ** step) / (1 - b1 ** step)
    return theta - lr_t * m / (np.sqrt(v) + eps), m, v
