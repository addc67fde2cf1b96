"""Learned warm start part of the FP64 oracle (test infrastructure only).

The network is not part of the paper's method: it predicts, per marker, the
error of the linear extrapolation 2 f_{k-1} - f_{k-2} of the boundary force so
that the Lagrange-multiplier solve of Sec. 3.1 (Eq. force_schur) can start
near its answer.  Architecture:
nin -> nh -> nh -> nout with tanh hidden layers, shared by all markers,

    xh = (x - in_shift) / in_scale
    h1 = tanh(xh W1^T + b1),  h2 = tanh(h1 W2^T + b2),  o = h2 W3^T + b3
    y  = out_shift + out_scale * o

and the training loss is 0.5/M sum_m ||o_m - (t_m - out_shift)/out_scale||^2.
Parameters are one flat vector in the order W1 [nh][nin], b1, W2 [nh][nh], b2,
W3 [nout][nh], b3 (row-major).

``bf16=True`` rounds both operands of every matrix product to bfloat16 (round
to nearest, ties to even) and keeps everything else in FP64; that is the
arithmetic a matrix-core implementation with BF16 operands and wide
accumulation performs, up to the order of its sums.
"""
from __future__ import annotations

import numpy as np

__all__ = ["bf16_round", "mlp_param_count", "mlp_unpack", "mlp_init", "mlp_forward", "mlp_loss_grad",
           "adam_step", "warm_features", "warm_start"]


def bf16_round(a) -> np.ndarray:
    """Round FP64 values to the nearest bfloat16 (ties to even) in two steps of
    exact arithmetic: FP64 -> nearest FP32 is not used, because double rounding
    could move a value that lies just beside a bfloat16 midpoint.  Instead the
    FP64 significand is rounded directly to 8 significant bits; the FP32
    exponent range is honoured for normal numbers (the network never produces
    bfloat16 subnormals; they are flushed to zero here)."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)                    # a = m 2^e, 0.5 <= |m| < 1
    scaled = np.ldexp(m, 8)               # 8 significant bits before the point
    r = np.round(scaled)                  # numpy rounds half to even
    out = np.ldexp(r, e - 8)
    out = np.where(np.abs(out) < 2.0 ** -126, 0.0, out)
    return out


def mlp_param_count(nin: int, nh: int, nout: int) -> int:
    return nh * nin + nh + nh * nh + nh + nout * nh + nout


def mlp_unpack(p, nin, nh, nout):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    out = []
    for shape in ((nh, nin), (nh,), (nh, nh), (nh,), (nout, nh), (nout,)):
        n = int(np.prod(shape))
        out.append(p[o:o + n].reshape(shape))
        o += n
    return out


def mlp_init(nin, nh, nout, seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fo, fi in ((nh, nin), (nh, nh), (nout, nh)):
        lim = 1.0 / np.sqrt(fi)
        parts.append(g.uniform(-lim, lim, size=fo * fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts)


def _mm(a, b, bf16):
    if bf16:
        a, b = bf16_round(a), bf16_round(b)
    return a @ b


def mlp_forward(p, x, nin, nh, nout, in_shift, in_scale, out_shift, out_scale, bf16=False, cache=False):
    """Network output y (physical units) for inputs x [M][nin]."""
    W1, b1, W2, b2, W3, b3 = mlp_unpack(p, nin, nh, nout)
    xh = (np.asarray(x, np.float64) - in_shift) / in_scale
    h1 = np.tanh(_mm(xh, W1.T, bf16) + b1)
    h2 = np.tanh(_mm(h1, W2.T, bf16) + b2)
    o = _mm(h2, W3.T, bf16) + b3
    y = out_shift + out_scale * o
    if cache:
        return y, (xh, h1, h2, o)
    return y


def mlp_loss_grad(p, x, t, nin, nh, nout, in_shift, in_scale, out_shift, out_scale, bf16=False):
    """Loss 0.5/M sum ||o - that||^2 and its gradient by reverse-mode
    differentiation of the forward pass above (chain rule written out layer by
    layer; d tanh(z)/dz = 1 - tanh(z)^2)."""
    W1, b1, W2, b2, W3, b3 = mlp_unpack(p, nin, nh, nout)
    _, (xh, h1, h2, o) = mlp_forward(p, x, nin, nh, nout, in_shift, in_scale, out_shift, out_scale, bf16, True)
    M = xh.shape[0]
    that = (np.asarray(t, np.float64) - out_shift) / out_scale
    d = o - that
    loss = 0.5 * float(np.sum(d * d)) / M
    dO = d / M
    gW3 = _mm(dO.T, h2, bf16)
    gb3 = dO.sum(axis=0)
    dZ2 = _mm(dO, W3, bf16) * (1.0 - h2 * h2)
    gW2 = _mm(dZ2.T, h1, bf16)
    gb2 = dZ2.sum(axis=0)
    dZ1 = _mm(dZ2, W2, bf16) * (1.0 - h1 * h1)
    gW1 = _mm(dZ1.T, xh, bf16)
    gb1 = dZ1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(p, g, m1, m2, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Kingma & Ba (2015) Adam with bias correction; ``step`` counts from 1.
    Returns the new (p, m1, m2)."""
    m1 = b1 * m1 + (1.0 - b1) * g
    m2 = b2 * m2 + (1.0 - b2) * g * g
    mh = m1 / (1.0 - b1 ** step)
    vh = m2 / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m1, m2


def warm_features(normals, ustate, f1, f2):
    """Per-marker features for the solve of step k: the outward normal, the
    body velocity increments U_{k+1} - U_k, U_k - U_{k-1}, U_{k-1} - U_{k-2}
    (ustate = (U_{k+1}, U_k, U_{k-1}, U_{k-2})), the marker's previous force
    and its last increment f_{k-1} - f_{k-2} -> [NL][12]."""
    nl = normals.shape[0]
    us = np.asarray(ustate, np.float64)
    du = np.broadcast_to(us[:3] - us[1:], (nl, 3))
    return np.concatenate([normals, du, f1, f1 - f2], axis=1)


def warm_start(y, f1, f2):
    """x0 = 2 f_{k-1} - f_{k-2} + y: the linear extrapolation of the force
    history plus the network's correction y."""
    return 2.0 * np.asarray(f1, np.float64) - np.asarray(f2, np.float64) + y
