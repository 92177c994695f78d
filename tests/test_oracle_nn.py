"""Pins of the convolution oracle used to check the warm-start kernels."""
import numpy as np
import pytest

from oracle import nn


def test_tap_convention_against_index_loops():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 4, 5))
    w = rng.normal(size=(3, 2, 27))
    b = rng.normal(size=3)
    out = nn.conv3d(x, w, b)
    nz, ny, nx = x.shape[1:]
    ref = np.zeros_like(out)
    for co in range(3):
        for z in range(nz):
            for y in range(ny):
                for xx in range(nx):
                    s = b[co]
                    for ci in range(2):
                        for dz in (-1, 0, 1):
                            for dy in (-1, 0, 1):
                                for dx in (-1, 0, 1):
                                    t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                                    s += w[co, ci, t] * x[ci, (z + dz) % nz, (y + dy) % ny,
                                                          (xx + dx) % nx]
                    ref[co, z, y, xx] = s
    assert np.abs(out - ref).max() < 1e-12


def test_adjoint_identity_and_weight_gradient():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 4, 5, 6))
    y = rng.normal(size=(2, 4, 5, 6))
    w = rng.normal(size=(2, 3, 27))
    lhs = np.sum(nn.conv3d(x, w) * y)
    rhs = np.sum(x * nn.conv3d_backward_data(y, w))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    gw, gb = nn.conv3d_backward_weights(y, x)
    # the map w -> <y, conv(x; w)> is linear: the gradient entry is the value
    # at the unit weight
    for (co, ci, t) in [(0, 0, 0), (1, 2, 13), (0, 1, 26)]:
        e = np.zeros_like(w)
        e[co, ci, t] = 1.0
        assert abs(np.sum(y * nn.conv3d(x, e)) - gw[co, ci, t]) < 1e-10
    assert np.allclose(gb, y.sum(axis=(1, 2, 3)))


def test_adam_bias_correction_with_a_constant_gradient():
    w = np.array([1.0, -2.0])
    g = np.array([0.5, -0.25])
    m = np.zeros(2)
    v = np.zeros(2)
    for step in range(1, 6):
        w_new, m, v = nn.adam(w, m, v, g, step, lr=0.1)
        # m_hat = g and v_hat = g^2 exactly: the step is lr * sign(g) (up to eps)
        assert np.allclose(w - w_new, 0.1 * np.sign(g), rtol=1e-6)
        w = w_new


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -3.14159])
    r = nn.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0          # tie to even
    assert r[2] == 1.0 + 2 ** -7
    assert r[3] == 1.0 + 2 ** -6                # tie to even (up)
    assert abs(r[4] + 3.140625) < 1e-12


def test_pool_and_upsample_against_index_loops_and_adjoints():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 4, 6, 2))
    p = nn.pool2(x)
    assert p.shape == (2, 2, 3, 1)
    for c in range(2):
        for z in range(2):
            for y in range(3):
                s = 0.0
                for dz in range(2):
                    for dy in range(2):
                        for dx in range(2):
                            s += x[c, 2 * z + dz, 2 * y + dy, dx]
                assert abs(p[c, z, y, 0] - s / 8) < 1e-14
    u = nn.upsample2(p)
    assert u.shape == x.shape
    for c in range(2):
        for z in range(4):
            for y in range(6):
                for xx in range(2):
                    assert u[c, z, y, xx] == p[c, z // 2, y // 2, xx // 2]
    g = rng.normal(size=p.shape)
    assert abs(np.sum(nn.pool2(x) * g) - np.sum(x * nn.pool2_backward(g))) < 1e-12
    h = rng.normal(size=x.shape)
    assert abs(np.sum(nn.upsample2(p) * h) - np.sum(p * nn.upsample2_backward(h))) < 1e-12


def _unet_params(rng, levels, cin=3, C=4, cout=2, widths=None):
    """Weights of a network with widths[l] channels at level l (all C by
    default): the decoder of level l takes [encoder features of level l,
    upsampled features of level l + 1]."""
    wd = list(widths) if widths is not None else [C] * levels
    p = {"enc": [], "dec": []}
    for l in range(levels):
        p["enc"].append((rng.normal(scale=0.3, size=(wd[l], cin if l == 0 else wd[l - 1], 27)),
                         rng.normal(scale=0.1, size=wd[l])))
    for l in range(levels - 1):
        p["dec"].append((rng.normal(scale=0.3, size=(wd[l], wd[l] + wd[l + 1], 27)),
                         rng.normal(scale=0.1, size=wd[l])))
    p["out"] = (rng.normal(scale=0.3, size=(cout, wd[0], 27)), rng.normal(scale=0.1, size=cout))
    return p


@pytest.mark.parametrize("levels,widths,shape", [(3, None, (3, 8, 8, 4)),
                                                 (4, (2, 3, 4, 5), (3, 16, 8, 8))])
def test_unet_backward_against_finite_differences(levels, widths, shape):
    """The encoder-decoder is piecewise linear in each weight (ReLU), so a
    central difference with a small step reproduces the gradient of <gy, y>
    away from the kinks; also for a network that widens level by level."""
    rng = np.random.default_rng(4)
    p = _unet_params(rng, levels, widths=widths)
    x = rng.normal(size=shape)
    y, st = nn.unet_forward(x, p, levels)
    gy = rng.normal(size=y.shape)
    g = nn.unet_backward(gy, p, st, levels)
    h = 1e-6
    parts = [("enc", l) for l in range(levels)] + [("dec", l) for l in range(levels - 1)] + \
        [("out", None)]
    for part, idx in parts:
        w, b = p[part] if idx is None else p[part][idx]
        gw, gb = g[part] if idx is None else g[part][idx]
        for k in range(3):
            pos = tuple(rng.integers(0, s) for s in w.shape)
            w0 = w[pos]
            w[pos] = w0 + h
            yp, _ = nn.unet_forward(x, p, levels)
            w[pos] = w0 - h
            ym, _ = nn.unet_forward(x, p, levels)
            w[pos] = w0
            fd = np.sum(gy * (yp - ym)) / (2 * h)
            assert abs(fd - gw[pos]) < 1e-6 * max(1.0, abs(fd)), (part, idx, pos, fd, gw[pos])
        j = int(rng.integers(0, b.shape[0]))
        b0 = b[j]
        b[j] = b0 + h
        yp, _ = nn.unet_forward(x, p, levels)
        b[j] = b0 - h
        ym, _ = nn.unet_forward(x, p, levels)
        b[j] = b0
        fd = np.sum(gy * (yp - ym)) / (2 * h)
        assert abs(fd - gb[j]) < 1e-6 * max(1.0, abs(fd)), (part, idx, "bias", fd, gb[j])
