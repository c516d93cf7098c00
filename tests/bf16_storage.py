"""The FP64 network oracle with its stored tensors rounded to BF16 where the
GPU kernels store BF16: weights, every layer's input activations, and the
masked output gradients that enter the backward convolutions (round to
nearest even).  Arithmetic stays FP64.  Test infrastructure: it measures how
far BF16 storage alone moves the network's output and loss gradient from the
plain FP64 oracle, the floor under the GPU-vs-oracle tolerances."""
from __future__ import annotations

import numpy as np

from oracle import train as T
from oracle import unet as U


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    b = a.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


class Bf16Net(U.Net):
    def __init__(self, params):
        super().__init__([(bf16(W), b) for W, b in params])

    def conv_f(self, i, x, stride=1, act=True):
        W, b = self.p[i]
        x = bf16(x)
        y = U.conv3x3(x, W, b, stride)
        out = U.relu(y) if act else y
        return out, (i, x, out, stride, act)

    def conv_b(self, c, g):
        i, x, out, stride, act = c
        if act:
            g = g * (out > 0)
        gx, dW, db = U.conv3x3_backward(x, self.p[i][0], bf16(g), stride)
        self._acc(i, dW, db)
        return gx

    def up_f(self, i, x):
        W, b = self.p[i]
        x = bf16(x)
        out = U.relu(U.upconv(x, W, b))
        return out, (i, x, out)

    def up_b(self, c, g):
        i, x, out = c
        gx, dW, db = U.upconv_backward(x, self.p[i][0], bf16(g * (out > 0)))
        self._acc(i, dW, db)
        return gx


def _with_net(cls, fn, *args):
    orig = U.Net
    U.Net = cls
    try:
        return fn(*args)
    finally:
        U.Net = orig


def network_forward(theta, enc_in, res_in, w, down_res):
    out, _ = _with_net(Bf16Net, U.network_forward, theta, enc_in, res_in, w, down_res)
    return out


def loss_and_grad(theta, enc, r, e, hx, hz, w, down_res):
    return _with_net(Bf16Net, T.loss_and_grad, theta, enc, r, e, hx, hz, w, down_res)
