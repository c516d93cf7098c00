"""Encoder-solver U-Nets (eq. 3.13, 3.14, 4.1 and Fig. 1) in FP64 NumPy -- oracle, test infrastructure only.

Tensors are NHWC float64 arrays [B][H][W][C].  Layer parameters:
  conv3x3  W[Cout][3][3][Cin], b[Cout]; zero padding 1; stride 1 or 2
           out[b,y,x,o] = b[o] + sum_{ky,kx,c} in[b, s*y+ky-1, s*x+kx-1, c] W[o,ky,kx,c]
  upconv   W[2][2][Cout][Cin], b[Cout]; transposed 2x2 convolution, stride 2
           out[b, 2y+a, 2x+d, o] = b[o] + sum_c in[b, y, x, c] W[a,d,o,c]
  resblock y = x + conv_2(ReLU(conv_1(x)))      (two 3x3 convs, C -> C)

The paper fixes the structure only in words (Fig. 1): the encoder coarsens the
squared slowness with a convolution followed by two ResNet layers per level,
up-samples with a learned convolution, concatenates the feature map of the
same size and applies a ResNet layer; the solver maps a residual to an error
and takes the encoder's features at every level.  Widths 32-256 over four
levels.  This module is this build's concrete reading of that description
(layer list `encoder_layers` / `solver_layers`); the GPU library builds the
same list from its own code, and the flat parameter order (layer by layer,
W then b) is the interface between the two.

Inputs and scaling (reading of eq. 4.1-4.2):
  encoder input  [omega^2 hx hz m, gamma]      (2 channels)
  solver input   s r,  s = sqrt(N) / ||r||      (2 channels: Re, Im)
  preconditioner e = hx hz * net(s r) / s       (so that M is 1-homogeneous)
  training target  s e_true / (hx hz)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

WIDTHS = (32, 64, 128, 256)


@dataclass(frozen=True)
class Layer:
    kind: str       # "conv" | "upconv"
    cin: int
    cout: int
    stride: int = 1
    name: str = ""

    def wshape(self):
        if self.kind == "conv":
            return (self.cout, 3, 3, self.cin)
        return (2, 2, self.cout, self.cin)


def encoder_layers(w=WIDTHS, cin=2, down_res=2):
    L = [Layer("conv", cin, w[0], 1, "e.in")]
    for r in range(down_res):
        L += [Layer("conv", w[0], w[0], 1, f"e.d0.rb{r}.1"), Layer("conv", w[0], w[0], 1, f"e.d0.rb{r}.2")]
    for l in range(1, len(w)):
        L.append(Layer("conv", w[l - 1], w[l], 2, f"e.d{l}.down"))
        for r in range(down_res):
            L += [Layer("conv", w[l], w[l], 1, f"e.d{l}.rb{r}.1"), Layer("conv", w[l], w[l], 1, f"e.d{l}.rb{r}.2")]
    for l in range(len(w) - 2, -1, -1):
        L.append(Layer("upconv", w[l + 1], w[l], 2, f"e.u{l}.up"))
        L.append(Layer("conv", 2 * w[l], w[l], 1, f"e.u{l}.merge"))
        L += [Layer("conv", w[l], w[l], 1, f"e.u{l}.rb.1"), Layer("conv", w[l], w[l], 1, f"e.u{l}.rb.2")]
    return L


def solver_layers(w=WIDTHS, cin=2, cout=2):
    L = [Layer("conv", cin, w[0], 1, "s.in"), Layer("conv", 2 * w[0], w[0], 1, "s.d0.ctx"),
         Layer("conv", w[0], w[0], 1, "s.d0.rb.1"), Layer("conv", w[0], w[0], 1, "s.d0.rb.2")]
    for l in range(1, len(w)):
        L += [Layer("conv", w[l - 1], w[l], 2, f"s.d{l}.down"), Layer("conv", 2 * w[l], w[l], 1, f"s.d{l}.ctx"),
              Layer("conv", w[l], w[l], 1, f"s.d{l}.rb.1"), Layer("conv", w[l], w[l], 1, f"s.d{l}.rb.2")]
    for l in range(len(w) - 2, -1, -1):
        L += [Layer("upconv", w[l + 1], w[l], 2, f"s.u{l}.up"), Layer("conv", 2 * w[l], w[l], 1, f"s.u{l}.merge"),
              Layer("conv", w[l], w[l], 1, f"s.u{l}.rb.1"), Layer("conv", w[l], w[l], 1, f"s.u{l}.rb.2")]
    L.append(Layer("conv", w[0], cout, 1, "s.out"))
    return L


def all_layers(w=WIDTHS, down_res=2):
    return encoder_layers(w, down_res=down_res) + solver_layers(w)


def n_params(layers):
    return sum(int(np.prod(l.wshape())) + l.cout for l in layers)


def unflatten(theta, layers):
    out, o = [], 0
    for l in layers:
        nw = int(np.prod(l.wshape()))
        W = theta[o:o + nw].reshape(l.wshape())
        o += nw
        b = theta[o:o + l.cout]
        o += l.cout
        out.append((W, b))
    assert o == theta.size
    return out


def init_params(layers, rng, small_residual=False):
    """He-normal weights, zero biases (flat FP64 vector).  small_residual: the
    second convolution of every residual block at 0.1x and the output layer at
    0.01x (a network that starts close to the zero map)."""
    parts = []
    for l in layers:
        fan_in = (9 if l.kind == "conv" else 1) * l.cin
        g = 1.0
        if small_residual and (l.name.endswith(".2") or l.name == "s.out"):
            g = 0.01 if l.name == "s.out" else 0.1
        parts.append(rng.standard_normal(int(np.prod(l.wshape()))) * np.sqrt(2.0 / fan_in) * g)
        parts.append(np.zeros(l.cout))
    return np.concatenate(parts)


# ---------------------------------------------------------------- primitive ops
def conv3x3(x, W, b, stride=1):
    B, H, Wd, C = x.shape
    Ho, Wo = (H + stride - 1) // stride, (Wd + stride - 1) // stride
    xp = np.zeros((B, H + 2, Wd + 2, C))
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((B, Ho, Wo, W.shape[0])) + b
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + stride * Ho:stride, kx:kx + stride * Wo:stride, :]
            out += patch @ W[:, ky, kx, :].T
    return out


def conv3x3_backward(x, W, g, stride=1):
    """Gradients of conv3x3 w.r.t. x, W, b for upstream gradient g."""
    B, H, Wd, C = x.shape
    Ho, Wo = g.shape[1:3]
    xp = np.zeros((B, H + 2, Wd + 2, C))
    xp[:, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(None), slice(ky, ky + stride * Ho, stride), slice(kx, kx + stride * Wo, stride), slice(None))
            dW[:, ky, kx, :] = np.einsum("bhwo,bhwc->oc", g, xp[sl])
            gxp[sl] += g @ W[:, ky, kx, :]
    return gxp[:, 1:-1, 1:-1], dW, g.sum(axis=(0, 1, 2))


def upconv(x, W, b):
    B, H, Wd, C = x.shape
    out = np.zeros((B, 2 * H, 2 * Wd, W.shape[2])) + b
    for a in range(2):
        for d in range(2):
            out[:, a::2, d::2, :] += x @ W[a, d].T
    return out


def upconv_backward(x, W, g):
    gx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for a in range(2):
        for d in range(2):
            ga = g[:, a::2, d::2, :]
            gx += ga @ W[a, d]
            dW[a, d] = np.einsum("bhwo,bhwc->oc", ga, x)
    return gx, dW, g.sum(axis=(0, 1, 2))


def relu(x):
    return np.maximum(x, 0.0)


# ---------------------------------------------------------------- layers with caches
class Net:
    """Forward with cached activations and the mirrored hand-written backward.
    params: list of (W, b) in layer order; grads accumulate in self.d."""

    def __init__(self, params):
        self.p = params
        self.d = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]

    def _acc(self, i, dW, db):
        self.d[i][0][...] += dW
        self.d[i][1][...] += db

    # conv (+ReLU)
    def conv_f(self, i, x, stride=1, act=True):
        W, b = self.p[i]
        y = conv3x3(x, W, b, stride)
        out = relu(y) if act else y
        return out, (i, x, out, stride, act)

    def conv_b(self, c, g):
        i, x, out, stride, act = c
        if act:
            g = g * (out > 0)
        gx, dW, db = conv3x3_backward(x, self.p[i][0], g, stride)
        self._acc(i, dW, db)
        return gx

    def up_f(self, i, x):
        W, b = self.p[i]
        out = relu(upconv(x, W, b))
        return out, (i, x, out)

    def up_b(self, c, g):
        i, x, out = c
        gx, dW, db = upconv_backward(x, self.p[i][0], g * (out > 0))
        self._acc(i, dW, db)
        return gx

    # residual block y = x + conv2(relu(conv1(x)))
    def res_f(self, i, x):
        h, c1 = self.conv_f(i, x, 1, True)
        y, c2 = self.conv_f(i + 1, h, 1, False)
        return x + y, (c1, c2)

    def res_b(self, c, g):
        c1, c2 = c
        gh = self.conv_b(c2, g)
        return g + self.conv_b(c1, gh)


def encoder_forward(net, x, w=WIDTHS, down_res=2):
    """{z_l} = EncoderNet(x) for x [1][H][W][2]; returns (z list, cache)."""
    cache = []
    i = 0
    skips = [None] * len(w)
    h, c = net.conv_f(i, x); cache.append(("c", c)); i += 1
    for _ in range(down_res):
        h, c = net.res_f(i, h); cache.append(("r", c)); i += 2
    skips[0] = h
    for l in range(1, len(w)):
        h, c = net.conv_f(i, h, 2); cache.append(("c", c)); i += 1
        for _ in range(down_res):
            h, c = net.res_f(i, h); cache.append(("r", c)); i += 2
        skips[l] = h
    z = [None] * len(w)
    z[-1] = h
    for l in range(len(w) - 2, -1, -1):
        u, c = net.up_f(i, h); cache.append(("u", c)); i += 1
        h, c = net.conv_f(i, np.concatenate([u, skips[l]], axis=-1)); cache.append(("m", c, w[l])); i += 1
        h, c = net.res_f(i, h); cache.append(("r", c)); i += 2
        z[l] = h
    return z, cache


def encoder_backward(net, cache, gz, w=WIDTHS, down_res=2):
    """Backward of encoder_forward given dL/dz_l (list); returns dL/dx."""
    gskip = [None] * len(w)
    ops = list(cache)
    # up path, reversed: for l = 0 .. L-2: (u, m, r) groups, last group first in reverse
    n_up = len(w) - 1
    up_ops = ops[len(ops) - 3 * n_up:]
    down_ops = ops[:len(ops) - 3 * n_up]
    g = gz[0].copy()
    for k in range(n_up):                     # l = 0, 1, ..., L-2 (reverse of forward order)
        l = k
        grp = up_ops[3 * (n_up - 1 - k): 3 * (n_up - k)]
        (_, cu), (_, cm, cl), (_, cr) = grp
        g = net.res_b(cr, g)
        gcat = net.conv_b(cm, g)
        gu, gs = gcat[..., :cl], gcat[..., cl:]
        gskip[l] = gs if gskip[l] is None else gskip[l] + gs
        g = net.up_b(cu, gu) + gz[l + 1]
    # g is now dL/d(h at the bottom) = dL/d skips[L-1] (z[L-1] gradient included above)
    # down path reversed
    idx = len(down_ops)
    for l in range(len(w) - 1, -1, -1):
        if l < len(w) - 1 and gskip[l] is not None:
            g = g + gskip[l]
        for _ in range(down_res):
            idx -= 1
            g = net.res_b(down_ops[idx][1], g)
        idx -= 1
        g = net.conv_b(down_ops[idx][1], g)
    return g


def solver_forward(net, r, z, w=WIDTHS, offset=0):
    """e = SolverNet(r; {z_l}) for r [B][H][W][2]; z_l [1][h][w][C] broadcast."""
    B = r.shape[0]
    zb = [np.broadcast_to(zl, (B,) + zl.shape[1:]) for zl in z]
    cache = []
    i = offset
    skips = [None] * len(w)
    h, c = net.conv_f(i, r); cache.append(c); i += 1
    for l in range(len(w)):
        if l > 0:
            h, c = net.conv_f(i, h, 2); cache.append(c); i += 1
        h, c = net.conv_f(i, np.concatenate([h, zb[l]], axis=-1)); cache.append(c); i += 1
        h, c = net.res_f(i, h); cache.append(c); i += 2
        skips[l] = h
    for l in range(len(w) - 2, -1, -1):
        u, c = net.up_f(i, h); cache.append(c); i += 1
        h, c = net.conv_f(i, np.concatenate([u, skips[l]], axis=-1)); cache.append(c); i += 1
        h, c = net.res_f(i, h); cache.append(c); i += 2
    out, c = net.conv_f(i, h, 1, act=False); cache.append(c)
    return out, cache


def solver_backward(net, cache, g, w=WIDTHS):
    """Backward of solver_forward; returns (dL/dr, [dL/dz_l summed over the batch])."""
    L = len(w)
    ops = list(cache)
    g = net.conv_b(ops.pop(), g)
    gskip = [None] * L
    for l in range(L - 1):                       # up path reversed: l = 0 .. L-2
        cr = ops.pop(); cm = ops.pop(); cu = ops.pop()
        g = net.res_b(cr, g)
        gcat = net.conv_b(cm, g)
        gu, gs = gcat[..., :w[l]], gcat[..., w[l]:]
        gskip[l] = gs
        g = net.up_b(cu, gu)
    gz = [None] * L
    for l in range(L - 1, -1, -1):
        if gskip[l] is not None:
            g = g + gskip[l]
        cr = ops.pop(); cc = ops.pop()
        g = net.res_b(cr, g)
        gcat = net.conv_b(cc, g)
        g = gcat[..., :w[l]]
        gz[l] = gcat[..., w[l]:].sum(axis=0, keepdims=True)
        if l > 0:
            g = net.conv_b(ops.pop(), g)
    g = net.conv_b(ops.pop(), g)
    assert not ops
    return g, gz


def network_forward(theta, enc_in, res_in, w=WIDTHS, down_res=2):
    """e_net = SolverNet(r; EncoderNet(m)) (eq. 4.1); one medium per batch."""
    layers = all_layers(w, down_res)
    net = Net(unflatten(theta, layers))
    z, ce = encoder_forward(net, enc_in, w, down_res)
    out, cs = solver_forward(net, res_in, z, w, offset=len(encoder_layers(w, down_res=down_res)))
    return out, (net, ce, cs, down_res)


def network_backward(state, g_out, w=WIDTHS):
    """Gradient of a scalar loss w.r.t. all parameters (flat) given dL/d out."""
    net, ce, cs, down_res = state
    _, gz = solver_backward(net, cs, g_out, w)
    encoder_backward(net, ce, gz, w, down_res)
    return np.concatenate([np.concatenate([dW.ravel(), db.ravel()]) for dW, db in net.d])


# ---------------------------------------------------------------- preconditioner application
def encoder_input(kappa2, gamma, omega, hx, hz):
    return np.stack([omega ** 2 * hx * hz * np.asarray(kappa2, np.float64), np.asarray(gamma, np.float64)],
                    axis=-1)[None]


def cnn_precond(theta, kappa2, gamma, omega, hx, hz, r, w=WIDTHS, down_res=2):
    """e = hx hz * net(s r) / s, s = sqrt(N)/||r|| per sample; r complex [B][H][W]."""
    r = np.asarray(r, np.complex128)
    B = r.shape[0]
    N = r[0].size
    nr = np.linalg.norm(r.reshape(B, -1), axis=1)
    s = np.where(nr > 0, np.sqrt(N) / np.where(nr > 0, nr, 1.0), 0.0)
    rin = np.stack([r.real, r.imag], axis=-1) * s[:, None, None, None]
    out, _ = network_forward(theta, encoder_input(kappa2, gamma, omega, hx, hz), rin, w, down_res)
    e = out[..., 0] + 1j * out[..., 1]
    scale = np.where(s > 0, hx * hz / np.where(s > 0, s, 1.0), 0.0)
    return e * scale[:, None, None]
