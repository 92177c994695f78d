"""Learned warm start of a load increment.

Algorithm 2 starts each load increment from the previous fluctuation. Here a
small 3D convolutional network (periodic 3x3x3 convolutions, BF16
activations and weights, FP32 accumulation; the kernels are the hfe_nn_*
entry points of libhfe.so) predicts the increment of the fluctuation from the
cell's state, and the solve starts from the prediction instead; the solver
then refines it to the same tolerance, so the result does not depend on the
guess beyond the solver's own tolerance (and, for the damage law, which of
several equilibria is reached).

Inputs per voxel (6 channels): the two phase indicators, the committed damage
(mean over the points of the voxel) and the previous increment of the
fluctuation, scaled by 1 / (||dE|| n) for a cell of n voxels per side. The
network predicts a correction to that previous increment (the last layer
starts at zero, so an untrained network repeats the previous increment: the
linear-extrapolation guess). Only the target of converged increments is used
for training.

This module only arranges data and calls the kernels; every convolution, its
gradients and the optimiser run in the HIP kernels.
"""
import ctypes

import numpy as np

from .hfe import HfeError, load_library

CHANNELS = (6, 16, 16, 3)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class ConvNet:
    """Layers conv(6->16)+ReLU, conv(16->16)+ReLU, conv(16->3) on a periodic grid."""

    def __init__(self, channels=CHANNELS, seed=0, device="cuda:0"):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device)
        self.channels = tuple(channels)
        rng = np.random.default_rng(seed)
        self.w, self.b, self.w16 = [], [], []
        self.mw, self.vw, self.mb, self.vb = [], [], [], []
        L = len(channels) - 1
        for l in range(L):
            cin, cout = channels[l], channels[l + 1]
            std = np.sqrt(2.0 / (27 * cin))
            w = rng.normal(scale=std, size=(cout, cin, 27)) if l < L - 1 else np.zeros((cout, cin, 27))
            self.w.append(torch.tensor(w, dtype=torch.float32, device=self.device))
            self.b.append(torch.zeros(cout, dtype=torch.float32, device=self.device))
            self.w16.append(torch.empty(w.size, dtype=torch.int16, device=self.device))
            for lst, ref in ((self.mw, self.w[-1]), (self.vw, self.w[-1]), (self.mb, self.b[-1]),
                             (self.vb, self.b[-1])):
                lst.append(torch.zeros_like(ref))
            self._check(self.lib.hfe_nn_to_bf16(_ptr(self.w[-1]), self.w[-1].numel(),
                                                _ptr(self.w16[-1]), self._stream()))
        self.step = 0

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    @staticmethod
    def _check(st):
        if st != 0:
            raise HfeError(st, "warm-start kernel call failed")

    def to_bf16(self, x32):
        y = self.torch.empty(x32.shape, dtype=self.torch.int16, device=self.device)
        self._check(self.lib.hfe_nn_to_bf16(_ptr(x32), x32.numel(), _ptr(y), self._stream()))
        return y

    def forward(self, x16, shape):
        """x16: BF16 input (cin, nz, ny, nx) as int16; returns the FP32 output
        and the activations kept for the backward pass."""
        torch = self.torch
        n = (ctypes.c_int * 3)(shape[2], shape[1], shape[0])
        acts = []
        h16 = x16
        L = len(self.w)
        for l in range(L):
            cin, cout = self.channels[l], self.channels[l + 1]
            out = torch.empty((cout,) + tuple(shape), dtype=torch.float32, device=self.device)
            out16 = torch.empty((cout,) + tuple(shape), dtype=torch.int16, device=self.device)
            relu = 1 if l < L - 1 else 0
            self._check(self.lib.hfe_nn_conv3d(_ptr(h16), cin, _ptr(self.w16[l]), _ptr(self.b[l]),
                                               cout, n, relu, _ptr(out), _ptr(out16),
                                               self._stream()))
            acts.append((h16, out if relu else None))
            h16 = out16
        return out, acts

    def train_step(self, x16, target, shape, lr=1e-3):
        """One Adam step on the mean squared error; returns the loss (host)."""
        torch = self.torch
        pred, acts = self.forward(x16, shape)
        n = (ctypes.c_int * 3)(shape[2], shape[1], shape[0])
        N = pred.numel()
        grad = torch.empty_like(pred)
        partials = torch.empty(int(self.lib.hfe_nn_mse_partials(N)), dtype=torch.float64,
                               device=self.device)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        self._check(self.lib.hfe_nn_mse(_ptr(pred), _ptr(target), N, _ptr(grad), _ptr(partials),
                                        _ptr(loss), self._stream()))
        grads = []
        for l in reversed(range(len(self.w))):
            cin, cout = self.channels[l], self.channels[l + 1]
            in16, act = acts[l]
            act_p = _ptr(act) if act is not None else None
            gw = torch.empty_like(self.w[l])
            gb = torch.empty_like(self.b[l])
            self._check(self.lib.hfe_nn_conv3d_backward_weights(
                _ptr(grad), cout, act_p, _ptr(in16), cin, n, _ptr(gw), _ptr(gb), self._stream()))
            grads.append((l, gw, gb))
            if l > 0:
                gin = torch.empty((cin,) + tuple(shape), dtype=torch.float32, device=self.device)
                self._check(self.lib.hfe_nn_conv3d_backward_data(
                    _ptr(grad), cout, act_p, _ptr(self.w16[l]), cin, n, _ptr(gin), self._stream()))
                grad = gin
        self.step += 1
        for l, gw, gb in grads:
            self._check(self.lib.hfe_nn_adam(_ptr(self.w[l]), _ptr(self.mw[l]), _ptr(self.vw[l]),
                                             _ptr(gw), gw.numel(), lr, 0.9, 0.999, 1e-8, self.step,
                                             _ptr(self.w16[l]), self._stream()))
            self._check(self.lib.hfe_nn_adam(_ptr(self.b[l]), _ptr(self.mb[l]), _ptr(self.vb[l]),
                                             _ptr(gb), gb.numel(), lr, 0.9, 0.999, 1e-8, self.step,
                                             None, self._stream()))
        return float(loss.item())

    def predict(self, x16, shape):
        out, _ = self.forward(x16, shape)
        return out


class _Conv:
    """One 3x3x3 layer: FP32 master weights and bias, Adam moments, BF16 copy."""

    def __init__(self, net, cin, cout, rng, zero=False):
        torch = net.torch
        self.cin, self.cout = cin, cout
        std = np.sqrt(2.0 / (27 * cin))
        w = np.zeros((cout, cin, 27)) if zero else rng.normal(scale=std, size=(cout, cin, 27))
        self.w = torch.tensor(w, dtype=torch.float32, device=net.device)
        self.b = torch.zeros(cout, dtype=torch.float32, device=net.device)
        self.w16 = torch.empty(w.size, dtype=torch.int16, device=net.device)
        self.mw, self.vw = torch.zeros_like(self.w), torch.zeros_like(self.w)
        self.mb, self.vb = torch.zeros_like(self.b), torch.zeros_like(self.b)
        net._check(net.lib.hfe_nn_to_bf16(_ptr(self.w), self.w.numel(), _ptr(self.w16),
                                          net._stream()))


class UNet:
    """Encoder-decoder on the periodic grid (row f3): `levels` resolutions,
    each halving the grid by 2x2x2 mean pooling, with widths[l] channels at
    level l (16 at every level by default; the widening network of the
    scaled warm start uses 16, 32, 64, 64). The decoder of level l upsamples
    (nearest) the features of level l + 1 and convolves them side by side
    with the encoder's features of level l (widths[l] + widths[l + 1]
    channels in). conv(in->w0)+ReLU at the finest level, conv(w[l-1]->w[l])
    +ReLU after every pooling, conv(w[l]+w[l+1]->w[l])+ReLU at every decoder
    level, conv(w0->out) out (zero-initialised, so an untrained network
    predicts no correction). BF16 activations and weights, FP32 accumulation;
    every operation runs in the hfe_nn_* kernels."""

    C = 16

    def __init__(self, levels=3, seed=0, device="cuda:0", in_channels=6, out_channels=3,
                 widths=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device)
        self.levels = levels
        self.widths = tuple(int(c) for c in widths) if widths is not None else (self.C,) * levels
        if len(self.widths) != levels:
            raise ValueError("one width per level")
        rng = np.random.default_rng(seed)
        W = self.widths
        self.enc = [_Conv(self, in_channels, W[0], rng)] + \
            [_Conv(self, W[l - 1], W[l], rng) for l in range(1, levels)]
        self.dec = [_Conv(self, W[l] + W[l + 1], W[l], rng) for l in range(levels - 1)]
        self.out = _Conv(self, W[0], out_channels, rng, zero=True)
        self.step = 0

    _stream = ConvNet._stream
    _check = staticmethod(ConvNet._check)
    to_bf16 = ConvNet.to_bf16

    def _dims(self, shape, l):
        nz, ny, nx = (int(v) >> l for v in shape)
        return (ctypes.c_int * 3)(nx, ny, nz), (nz, ny, nx)

    def _conv(self, layer, in16, n, relu, out, out16):
        self._check(self.lib.hfe_nn_conv3d(_ptr(in16), layer.cin, _ptr(layer.w16), _ptr(layer.b),
                                           layer.cout, n, 1 if relu else 0, _ptr(out),
                                           _ptr(out16) if out16 is not None else None,
                                           self._stream()))

    def forward(self, x16, shape):
        """x16: BF16 input (in_channels, nz, ny, nx), every axis divisible by
        2^(levels-1)."""
        torch, W, L = self.torch, self.widths, self.levels
        f32 = dict(dtype=torch.float32, device=self.device)
        i16 = dict(dtype=torch.int16, device=self.device)
        st = {"enc": [], "cat": [], "pool16": [], "dec": []}
        # encoder
        inp = x16
        for l in range(L):
            n, dims = self._dims(shape, l)
            e = torch.empty((W[l],) + dims, **f32)
            cat = torch.empty((W[l] + W[l + 1],) + dims, **i16) if l < L - 1 else None
            if l > 0:
                nf, _ = self._dims(shape, l - 1)
                p16 = torch.empty((W[l - 1],) + dims, **i16)
                self._check(self.lib.hfe_nn_pool2(_ptr(st["enc"][l - 1]), W[l - 1], nf, None,
                                                  _ptr(p16), self._stream()))
                st["pool16"].append(p16)
                inp = p16
            # the encoder's BF16 copy is the first part of the decoder input
            self._conv(self.enc[l], inp, n, True, e, cat[:W[l]] if cat is not None else None)
            st["enc"].append(e)
            st["cat"].append(cat)
        # decoder, coarse to fine
        prev = st["enc"][L - 1]
        dec = [None] * (L - 1)
        for l in range(L - 2, -1, -1):
            n, dims = self._dims(shape, l)
            m, _ = self._dims(shape, l + 1)
            cat = st["cat"][l]
            self._check(self.lib.hfe_nn_upsample2(_ptr(prev), W[l + 1], m, None,
                                                  _ptr(cat[W[l]:]), self._stream()))
            d = torch.empty((W[l],) + dims, **f32)
            d16 = torch.empty((W[l],) + dims, **i16) if l == 0 else None
            self._conv(self.dec[l], cat, n, True, d, d16)
            dec[l] = (d, d16)
            prev = d
        st["dec"] = dec
        n, dims = self._dims(shape, 0)
        y = torch.empty((self.out.cout,) + dims, **f32)
        self._conv(self.out, dec[0][1], n, False, y, None)
        return y, st

    def _grads(self, layer, g, act, in16, n):
        gw = self.torch.empty_like(layer.w)
        gb = self.torch.empty_like(layer.b)
        self._check(self.lib.hfe_nn_conv3d_backward_weights(
            _ptr(g), layer.cout, _ptr(act) if act is not None else None, _ptr(in16), layer.cin, n,
            _ptr(gw), _ptr(gb), self._stream()))
        return gw, gb

    def _gin(self, layer, g, act, n, dims):
        gin = self.torch.empty((layer.cin,) + dims, dtype=self.torch.float32, device=self.device)
        self._check(self.lib.hfe_nn_conv3d_backward_data(
            _ptr(g), layer.cout, _ptr(act) if act is not None else None, _ptr(layer.w16),
            layer.cin, n, _ptr(gin), self._stream()))
        return gin

    def backward(self, gy, x16, st, shape):
        """Weight and bias gradients [(layer, gw, gb)] for dL/dy = gy."""
        torch, W, L = self.torch, self.widths, self.levels
        out = []
        n0, d0 = self._dims(shape, 0)
        dec0, dec0_16 = st["dec"][0]
        out.append((self.out,) + self._grads(self.out, gy, None, dec0_16, n0))
        g = self._gin(self.out, gy, None, n0, d0)          # d loss / d dec_0
        g_enc_part = [None] * L
        for l in range(L - 1):
            n, dims = self._dims(shape, l)
            m, mdims = self._dims(shape, l + 1)
            d = st["dec"][l][0]
            out.append((self.dec[l],) + self._grads(self.dec[l], g, d, st["cat"][l], n))
            gcat = self._gin(self.dec[l], g, d, n, dims)    # (W[l] + W[l+1], level l)
            g_enc_part[l] = gcat[:W[l]]
            gc = torch.empty((W[l + 1],) + mdims, dtype=torch.float32, device=self.device)
            self._check(self.lib.hfe_nn_upsample2_backward(_ptr(gcat[W[l]:].contiguous()),
                                                           W[l + 1], m, _ptr(gc), self._stream()))
            g = gc                                          # d loss / d (dec_{l+1} or enc_{L-1})
        # encoder, coarse to fine: g is d loss / d enc_{L-1}
        for l in range(L - 1, -1, -1):
            n, dims = self._dims(shape, l)
            e = st["enc"][l]
            inp = x16 if l == 0 else st["pool16"][l - 1]
            out.append((self.enc[l],) + self._grads(self.enc[l], g, e, inp, n))
            if l == 0:
                break
            gp = self._gin(self.enc[l], g, e, n, dims)      # d loss / d pooled input
            nf, _ = self._dims(shape, l - 1)
            ge = g_enc_part[l - 1].contiguous()
            self._check(self.lib.hfe_nn_pool2_backward(_ptr(gp), W[l - 1], nf, _ptr(ge),
                                                       self._stream()))
            g = ge
        return out

    def train_step(self, x16, target, shape, lr=1e-3):
        torch = self.torch
        y, st = self.forward(x16, shape)
        N = y.numel()
        gy = torch.empty_like(y)
        partials = torch.empty(int(self.lib.hfe_nn_mse_partials(N)), dtype=torch.float64,
                               device=self.device)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        self._check(self.lib.hfe_nn_mse(_ptr(y), _ptr(target), N, _ptr(gy), _ptr(partials),
                                        _ptr(loss), self._stream()))
        grads = self.backward(gy, x16, st, shape)
        self.step += 1
        for layer, gw, gb in grads:
            self._check(self.lib.hfe_nn_adam(_ptr(layer.w), _ptr(layer.mw), _ptr(layer.vw),
                                             _ptr(gw), gw.numel(), lr, 0.9, 0.999, 1e-8, self.step,
                                             _ptr(layer.w16), self._stream()))
            self._check(self.lib.hfe_nn_adam(_ptr(layer.b), _ptr(layer.mb), _ptr(layer.vb),
                                             _ptr(gb), gb.numel(), lr, 0.9, 0.999, 1e-8, self.step,
                                             None, self._stream()))
        return float(loss.item())

    def predict(self, x16, shape):
        y, _ = self.forward(x16, shape)
        return y


def features(phase, damage, du_prev, scale):
    """The 6 input channels (numpy float32, (6, nz, ny, nx)).

    phase (nz, ny, nx) with 0 = matrix, 1 = inclusion; damage (nz, ny, nx, nq)
    committed damage; du_prev (3, nz, ny, nx) the previous increment of the
    fluctuation; scale = ||dE|| n."""
    f = np.empty((6,) + phase.shape, dtype=np.float32)
    f[0] = phase == 0
    f[1] = phase == 1
    f[2] = damage.mean(axis=-1)
    f[3:6] = du_prev / scale
    return f


def strain_channels(u, E):
    """sym(grad u) + E at the element centres of the trilinear field u (3,
    nz, ny, nx) on the unit periodic grid (per direction, the mean of the
    element's 4 edge differences), Voigt order xx, yy, zz, yz, xz, xy:
    (6, nz, ny, nx)."""
    G = np.empty((3, 3) + u.shape[1:])
    for j, ax in enumerate((3, 2, 1)):          # x, y, z axes of u
        d = np.roll(u, -1, axis=ax) - u
        others = [a for a in (3, 2, 1) if a != ax]
        d = 0.5 * (d + np.roll(d, -1, axis=others[0]))
        d = 0.5 * (d + np.roll(d, -1, axis=others[1]))
        G[:, j] = d
    S = 0.5 * (G + G.transpose(1, 0, 2, 3, 4)) + np.asarray(E)[:, :, None, None, None]
    return np.stack([S[0, 0], S[1, 1], S[2, 2], S[1, 2], S[0, 2], S[0, 1]])


def features_full(phase, damage, du_prev, scale, u, E, dE):
    """The 18 input channels of the scaled warm start: the 6 of `features`,
    the current strain (6, over ||E|| + ||dE||) and the macroscopic increment
    dE (6 uniform channels, Voigt order, over ||dE||)."""
    dE = np.asarray(dE, dtype=np.float64)
    ndE = max(float(np.linalg.norm(dE)), 1e-300)
    f = np.empty((18,) + phase.shape, dtype=np.float32)
    f[:6] = features(phase, damage, du_prev, scale)
    f[6:12] = strain_channels(u, E) / (float(np.linalg.norm(E)) + ndE)
    for k, (i, j) in enumerate(((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))):
        f[12 + k] = dE[i, j] / ndE
    return f


class WarmStart:
    """Training data from solves, training, and the warm-started solve.

    full=False: the 3-level network of 16 channels on the 6 channels of
    `features`. full=True: the 4-level network widening 16, 32, 64, 64 on the
    18 channels of `features_full` (the current strain and the macroscopic
    increment as well)."""

    def __init__(self, net=None, seed=0, full=False):
        self.full = full
        if net is None:
            net = (UNet(levels=4, widths=(16, 32, 64, 64), in_channels=18, seed=seed) if full
                   else UNet(seed=seed))
        self.net = net
        self.samples = []      # (features, target, shape), target = du / scale - du_prev / scale

    def _x16(self, f):
        torch = self.net.torch
        return self.net.to_bf16(torch.tensor(f, device=self.net.device))

    def record(self, phase, damage, du_prev, du, scale):
        f = features(phase, damage, du_prev, scale)
        target = ((du - du_prev) / scale).astype(np.float32)
        self.samples.append((f, target, phase.shape))

    def train(self, epochs, lr=1e-3, seed=0):
        torch = self.net.torch
        rng = np.random.default_rng(seed)
        data = [(self._x16(f), torch.tensor(t, device=self.net.device), sh)
                for f, t, sh in self.samples]
        losses = []
        for _ in range(epochs):
            for i in rng.permutation(len(data)):
                x16, t, sh = data[i]
                losses.append(self.net.train_step(x16, t, sh, lr))
        return losses

    def predict(self, phase, damage, du_prev, scale):
        """Predicted increment of the fluctuation (3, nz, ny, nx), float64."""
        f = features(phase, damage, du_prev, scale)
        corr = self.net.predict(self._x16(f), phase.shape).double().cpu().numpy()
        return du_prev + scale * corr

    def state_features(self, solver, phase, u_prev, du_prev, scale, dE=None):
        """The network's input at the solver's current state (right after
        apply_load_step, before the solve)."""
        if not self.full:
            return features(phase, solver.damage(), du_prev, scale)
        return features_full(phase, solver.damage(), du_prev, scale, u_prev,
                             solver.get_state()["E"], dE)

    def record_sample(self, f, du_prev, du, scale, shape):
        """A training pair: the input f at the start of an increment and the
        increment du of the fluctuation that the solve reached."""
        self.samples.append((f, ((du - du_prev) / scale).astype(np.float32), tuple(shape)))

    def predict_from(self, f, du_prev, scale, shape):
        """Predicted increment of the fluctuation from the input f, float64."""
        corr = self.net.predict(self._x16(f), tuple(shape)).double().cpu().numpy()
        return du_prev + scale * corr

    def warm_start(self, solver, phase, u_prev, du_prev, scale, dE=None):
        """Set the solver's initial guess for the increment just applied
        (after apply_load_step): the learned one, u_prev + the predicted
        increment, if its equilibrium residual r_eq is below that of
        Algorithm 2's plain guess (the previous fluctuation u_prev, which the
        solver holds on entry); otherwise the plain guess is kept. Returns
        True if the learned guess was taken."""
        r_plain = solver.residual()
        if self.full:
            du = self.predict_from(self.state_features(solver, phase, u_prev, du_prev, scale, dE),
                                   du_prev, scale, phase.shape)
        else:
            du = self.predict(phase, solver.damage(), du_prev, scale)
        solver.set_displacement(u_prev + du)
        if solver.residual() < r_plain:
            return True
        solver.set_displacement(u_prev)
        return False
