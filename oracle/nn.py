"""Periodic 3x3x3 convolutions, their adjoints and Adam (oracle for the
warm-start network kernels).

TEST INFRASTRUCTURE ONLY: imported by tests and never by the library.

Fields are (C, nz, ny, nx); a filter bank is (cout, cin, 27) with tap
t = (dz+1)*9 + (dy+1)*3 + (dx+1), and out[co](v) = b[co] +
sum_{ci,t} w[co, ci, t] in[ci](v + (dz, dy, dx)), indices periodic. FP64.

Pinned by (``tests/test_oracle_nn.py``): explicit index loops on a tiny grid
(the tap convention, the 2x2x2 pooling and the nearest upsampling), the
adjoint identities <A x, y> = <x, A^T y> of the convolution, pooling and
upsampling, the weight gradient against the (linear) map at unit weights,
and Adam's bias correction (a constant gradient gives m_hat = g at every
step).
"""
import numpy as np

TAPS = [(t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1) for t in range(27)]


def _shift(x, off):
    """y(v) = x(v + off), periodic, for x of shape (..., nz, ny, nx)."""
    dz, dy, dx = off
    return np.roll(x, shift=(-dz, -dy, -dx), axis=(-3, -2, -1))


def conv3d(x, w, b=None):
    cout = w.shape[0]
    out = np.zeros((cout,) + x.shape[1:])
    for t, off in enumerate(TAPS):
        xs = _shift(x, off)
        out += np.einsum("oc,c...->o...", w[:, :, t], xs)
    if b is not None:
        out += np.asarray(b)[:, None, None, None]
    return out


def conv3d_backward_data(g, w):
    """The adjoint of conv3d (without bias) applied to g."""
    cin = w.shape[1]
    out = np.zeros((cin,) + g.shape[1:])
    for t, (dz, dy, dx) in enumerate(TAPS):
        gs = _shift(g, (-dz, -dy, -dx))
        out += np.einsum("oc,o...->c...", w[:, :, t], gs)
    return out


def conv3d_backward_weights(g, x):
    """d<g, conv3d(x; w)>/dw (cout, cin, 27) and d/db (cout,)."""
    gw = np.zeros((g.shape[0], x.shape[0], 27))
    for t, off in enumerate(TAPS):
        xs = _shift(x, off)
        gw[:, :, t] = np.einsum("ozyx,czyx->oc", g, xs)
    return gw, g.sum(axis=(1, 2, 3))


def relu(x):
    return np.maximum(x, 0.0)


def adam(w, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba): returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(x):
    """Round to BF16 (the upper 16 bits of binary32, ties to even), as float64."""
    a = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    a = (a + 0x7FFF + ((a >> 16) & 1)) >> 16 << 16
    return (a.astype(np.uint32)).view(np.float32).astype(np.float64)


def pool2(x):
    """Mean over 2x2x2 blocks (C, nz, ny, nx) -> (C, nz/2, ny/2, nx/2)."""
    C, nz, ny, nx = x.shape
    return x.reshape(C, nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(2, 4, 6))


def pool2_backward(g):
    """The adjoint of pool2: every child of a block gets g / 8."""
    return np.repeat(np.repeat(np.repeat(g, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def upsample2(x):
    """Nearest-neighbour doubling of every axis (C, nz, ny, nx) -> (C, 2nz, 2ny, 2nx)."""
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def upsample2_backward(g):
    """The adjoint of upsample2: the sum over the 8 children of a block."""
    C, nz, ny, nx = g.shape
    return g.reshape(C, nz // 2, 2, ny // 2, 2, nx // 2, 2).sum(axis=(2, 4, 6))


def unet_forward(x, params, levels, bf16=False):
    """The encoder-decoder of the warm start (levels resolutions, 2x2x2 mean
    pooling, nearest upsampling, the decoder's input = [encoder features,
    upsampled coarse features]; the channel counts follow the weights, so a
    level may widen); params = {"enc": [(w, b)] * levels,
    "dec": [(w, b)] * (levels - 1) (finest first), "out": (w, b)}. With bf16,
    every convolution input is rounded to BF16 first (as the kernels store
    activations). Returns the output and the intermediate values the backward
    pass needs."""
    rnd = bf16_round if bf16 else (lambda a: a)
    st = {"enc": [], "in": [], "dec": [None] * (levels - 1), "cat": [None] * (levels - 1)}
    h = x
    for l in range(levels):
        if l > 0:
            h = pool2(st["enc"][l - 1])
        w, b = params["enc"][l]
        hin = rnd(h)
        st["in"].append(hin)
        st["enc"].append(relu(conv3d(hin, w, b)))
    prev = st["enc"][levels - 1]
    for l in range(levels - 2, -1, -1):
        cat = np.concatenate([rnd(st["enc"][l]), rnd(upsample2(prev))], axis=0)
        st["cat"][l] = cat
        w, b = params["dec"][l]
        st["dec"][l] = relu(conv3d(cat, w, b))
        prev = st["dec"][l]
    w, b = params["out"]
    st["out_in"] = rnd(st["dec"][0])
    return conv3d(st["out_in"], w, b), st


def unet_backward(gy, params, st, levels):
    """Gradients of <gy, y> with respect to every (w, b), for the values `st`
    of unet_forward (the BF16 roundings of the forward pass are treated as
    identities). Returns a dict shaped like params. The channel counts may
    differ between levels (a widening network): the decoder input of level l
    is [encoder features of level l (C_l channels), upsampled coarse features]."""
    grads = {"enc": [None] * levels, "dec": [None] * (levels - 1)}
    w, _ = params["out"]
    grads["out"] = conv3d_backward_weights(gy, st["out_in"])
    g = conv3d_backward_data(gy, w)
    g_enc = [None] * levels
    for l in range(levels - 1):
        gm = np.where(st["dec"][l] > 0, g, 0.0)
        w, _ = params["dec"][l]
        grads["dec"][l] = conv3d_backward_weights(gm, st["cat"][l])
        gcat = conv3d_backward_data(gm, w)
        C = params["enc"][l][0].shape[0]
        g_enc[l] = gcat[:C]
        g = upsample2_backward(gcat[C:])
    for l in range(levels - 1, -1, -1):
        gm = np.where(st["enc"][l] > 0, g, 0.0)
        w, _ = params["enc"][l]
        grads["enc"][l] = conv3d_backward_weights(gm, st["in"][l])
        if l == 0:
            break
        g = g_enc[l - 1] + pool2_backward(conv3d_backward_data(gm, w))
    return grads
