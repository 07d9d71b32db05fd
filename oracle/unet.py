"""FP64 reference of the convolutional neural operator of the learned warm start.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no network: this module writes out the plain definitions of the network that the
library trains and runs, so that its kernels can be checked element by element:
  * 3x3 convolution = cross-correlation with zero padding, y[p] = sum_tap W[tap] x[p + s(tap)] + b,
    tap = 3 (dy + 1) + (dx + 1), s(tap) = (dy, dx); the 1x1 head is the taps = 1 case;
  * ReLU; 2x2 mean pooling; nearest 2x upsampling; channel concatenation [upsampled, skip];
  * masked mean squared error L = sum_p m_p |out_p - t_p|^2 / (4 sum_p m_p);
  * Adam (Kingma and Ba, 2015) with bias correction and decoupled weight decay.
Topology: encoder levels with channels 32, 64, 128, 256 (two convolutions each, the second one
the skip), a bottleneck of 256 channels (two convolutions), decoder levels 3..0 (upsample,
concatenate, two convolutions), head 1x1 32 -> 4. Input 4 planes padded with 4 zero planes.
Flat parameter layout: per layer W [cout][taps][cin] then b [cout], in that order.

Activations are NHWC float64 arrays [B, H, W, C]. With emulate_bf16 the forward pass rounds
weights (not the head), the packed input, every convolution output, and every pooled value to
bfloat16 (round to nearest even), as the device stores them; the backward pass is exact FP64, or
with emulate_bf16 rounds the activation gradients where the device stores them.
The convolution is im2col followed by one matrix product; conv_brute is the loop definition.
Parity of this module is pinned by brute force, adjointness, finite differences and closed forms
in the tests, not by the paper.
"""
import numpy as np

LEVELS = 5
CH = (32, 64, 128, 256, 256)
CIN0 = 8
NIN = 4
NOUT = 4


def layer_shapes():
    """(cin, cout, taps) of every layer in parameter order."""
    L = []
    c = CIN0
    for l in range(LEVELS):
        L += [(c, CH[l], 9), (CH[l], CH[l], 9)]
        c = CH[l]
    for l in range(LEVELS - 2, -1, -1):
        L += [(CH[l + 1] + CH[l], CH[l], 9), (CH[l], CH[l], 9)]
    L.append((CH[0], NOUT, 1))
    return L


def param_count():
    return sum(co * t * ci + co for ci, co, t in layer_shapes())


def split_params(theta):
    """List of (W [cout, taps, cin], b [cout]) views into the flat vector."""
    out, off = [], 0
    for ci, co, t in layer_shapes():
        n = co * t * ci
        W = theta[off:off + n].reshape(co, t, ci)
        off += n
        b = theta[off:off + co]
        off += co
        out.append((W, b))
    return out


def bf16_round(x):
    """Round to bfloat16 (nearest, ties to even) through float32, returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _shift(t, taps):
    return (t // 3 - 1, t % 3 - 1) if taps == 9 else (0, 0)


def im2col(X, taps):
    B, H, W, C = X.shape
    if taps == 1:
        return X.copy()
    Xp = np.zeros((B, H + 2, W + 2, C))
    Xp[:, 1:H + 1, 1:W + 1, :] = X
    cols = np.empty((B, H, W, taps * C))
    for t in range(taps):
        dy, dx = _shift(t, taps)
        cols[..., t * C:(t + 1) * C] = Xp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :]
    return cols


def col2im(dcols, taps, C):
    B, H, W, _ = dcols.shape
    if taps == 1:
        return dcols.copy()
    dXp = np.zeros((B, H + 2, W + 2, C))
    for t in range(taps):
        dy, dx = _shift(t, taps)
        dXp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :] += dcols[..., t * C:(t + 1) * C]
    return dXp[:, 1:H + 1, 1:W + 1, :]


def conv(X, Wt, b, taps, relu, accum32=False):
    """Pre-activation z and output y of one convolution layer. accum32: the products are summed
    in float32 (any order), as a second valid accumulation beside the FP64 one."""
    cout = Wt.shape[0]
    if accum32:
        z = (im2col(X, taps).astype(np.float32) @ Wt.reshape(cout, -1).T.astype(np.float32)).astype(np.float64) + b
    else:
        z = im2col(X, taps) @ Wt.reshape(cout, -1).T + b
    return z, (np.maximum(z, 0.0) if relu else z)


def conv_brute(X, Wt, b, taps):
    """Loop definition of the convolution (no activation), for tiny inputs."""
    B, H, W, C = X.shape
    cout = Wt.shape[0]
    Y = np.zeros((B, H, W, cout))
    for n in range(B):
        for y in range(H):
            for x in range(W):
                for co in range(cout):
                    s = b[co]
                    for t in range(taps):
                        dy, dx = _shift(t, taps)
                        yy, xx = y + dy, x + dx
                        if 0 <= yy < H and 0 <= xx < W:
                            for ci in range(C):
                                s += Wt[co, t, ci] * X[n, yy, xx, ci]
                    Y[n, y, x, co] = s
    return Y


def pool(X):
    B, H, W, C = X.shape
    return X.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool_adjoint(G):
    return np.repeat(np.repeat(G, 2, axis=1), 2, axis=2) * 0.25


def up(X):
    return np.repeat(np.repeat(X, 2, axis=1), 2, axis=2)


def up_adjoint(G):
    B, H, W, C = G.shape
    return G.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def forward(theta, x_in, emulate_bf16=False, accum32=False):
    """Network output [B, H, W, 4] and the cache of the backward pass. accum32: float32 sums in
    the 3x3 convolutions; with bf16 storage emulated, the distance between the two accumulations
    is the floor that any FP32-accumulating implementation can be held to."""
    rb = bf16_round if emulate_bf16 else (lambda v: v)
    P = split_params(theta)
    nconv = len(P) - 1
    Ws = [(rb(W) if k < nconv else W, b) for k, (W, b) in enumerate(P)]
    B, H, W, _ = x_in.shape
    x = np.zeros((B, H, W, CIN0))
    x[..., :NIN] = x_in
    x = rb(x)
    cache = {'x0': x}
    k = 0
    skips = []
    for l in range(LEVELS):
        if l > 0:
            x = rb(pool(skips[-1]))
        cache[('in', k)] = x
        _, a = conv(x, *Ws[k], 9, True, accum32)
        a = rb(a)
        cache[('out', k)] = a
        k += 1
        cache[('in', k)] = a
        _, s = conv(a, *Ws[k], 9, True, accum32)
        s = rb(s)
        cache[('out', k)] = s
        k += 1
        skips.append(s)
    below = skips.pop()                     # bottleneck output
    for l in range(LEVELS - 2, -1, -1):
        cat = np.concatenate([up(below), skips[l]], axis=-1)
        cache[('in', k)] = cat
        _, a = conv(cat, *Ws[k], 9, True, accum32)
        a = rb(a)
        cache[('out', k)] = a
        k += 1
        cache[('in', k)] = a
        _, d = conv(a, *Ws[k], 9, True, accum32)
        d = rb(d)
        cache[('out', k)] = d
        k += 1
        below = d
    cache[('in', k)] = below
    _, out = conv(below, *Ws[k], 1, False)
    cache['Ws'] = Ws
    return out, cache


def loss(out, tgt, mask=None):
    m = np.ones(out.shape[:3]) if mask is None else mask
    cnt = NOUT * m.sum()
    return float((m[..., None] * (out - tgt) ** 2).sum() / cnt)


def backward(theta, cache, out, tgt, mask=None, emulate_bf16=False):
    """Gradient of the masked MSE with respect to the flat parameters, in FP64.

    Exact by default. With emulate_bf16 every activation gradient is rounded to bfloat16 where the
    device stores one: the data gradient of each convolution (the head's included), the adjoint of
    the upsampling (four values summed, then rounded) and the skip gradient once the pooling path
    has been added to it. The ReLU masks are exact; weight and bias gradients are sums of products
    of those stored values and stay unrounded.
    """
    rb = bf16_round if emulate_bf16 else (lambda v: v)
    Ws = cache['Ws']
    shapes = layer_shapes()
    grads = [None] * len(Ws)
    m = np.ones(out.shape[:3]) if mask is None else mask
    cnt = NOUT * m.sum()
    g = 2.0 * m[..., None] * (out - tgt) / cnt

    def conv_bwd(k, dZ):
        ci, co, t = shapes[k]
        X = cache[('in', k)]
        cols = im2col(X, t)
        dW = dZ.reshape(-1, co).T @ cols.reshape(-1, t * ci)
        grads[k] = (dW.reshape(co, t, ci), dZ.reshape(-1, co).sum(axis=0))
        dcols = dZ @ Ws[k][0].reshape(co, -1)
        return rb(col2im(dcols, t, ci))

    k = len(Ws) - 1
    dA = conv_bwd(k, g)                     # head (no activation)
    k -= 1
    d_skip = [None] * (LEVELS - 1)
    for l in range(LEVELS - 1):             # decoder, top level first
        dA = dA * (cache[('out', k)] > 0)
        dA = conv_bwd(k, dA)
        k -= 1
        dA = dA * (cache[('out', k)] > 0)
        dcat = conv_bwd(k, dA)
        k -= 1
        cu = CH[l + 1]
        d_skip[l] = dcat[..., cu:]
        dA = rb(up_adjoint(dcat[..., :cu]))
    dpool = None
    for l in range(LEVELS - 1, -1, -1):     # bottleneck and encoder
        if l == LEVELS - 1:
            dS = dA
        else:
            dS = rb(d_skip[l] + pool_adjoint(dpool))
        dS = dS * (cache[('out', k)] > 0)
        dA = conv_bwd(k, dS)
        k -= 1
        dA = dA * (cache[('out', k)] > 0)
        dpool = conv_bwd(k, dA)
        k -= 1
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return flat, loss(out, tgt, mask)


def clip_grad_norm(g, max_norm):
    """Gradient clipping by the global L2 norm: g min(1, max_norm / ||g||)."""
    norm = float(np.sqrt(np.sum(np.asarray(g, dtype=np.float64) ** 2)))
    return (g * (max_norm / norm) if norm > max_norm else g), norm


def adam_step(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * (mh / (np.sqrt(vh) + eps) + wd * theta), m, v
