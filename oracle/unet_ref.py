"""CPU oracle of the dose denoiser (test infrastructure only).

A 3-level 3D U-Net that maps (low-history dose, density) to a high-history
dose, written out in plain numpy, FP64, channels-first [C, D, H, W]:

  enc1: conv3 2->16, ReLU, conv3 16->16, ReLU                 (full res)
  pool: 2x2x2 average
  enc2: conv3 16->32, ReLU, conv3 32->32, ReLU                (1/2)
  pool
  mid : conv3 32->64, ReLU, conv3 64->64, ReLU                (1/4)
  up2 : transposed conv 2x2x2 stride 2, 64->32; concat [up2, enc2]
  dec2: conv3 64->32, ReLU, conv3 32->32, ReLU                (1/2)
  up1 : transposed conv 32->16; concat [up1, enc1]
  dec1: conv3 32->16, ReLU, conv3 16->16, ReLU                (full res)
  head: conv1 16->1;  output = input dose channel + head      (residual)
  loss: mean squared error against the target dose.

conv3 is a 3x3x3 cross-correlation with zero padding 1.  Every convolution is
the plain sum over kernel offsets of (weights x shifted input).  Backward is
the analytic adjoint of each step.  `bf16=True` rounds to bfloat16 (round to
nearest even) exactly where the GPU kernels store bfloat16: the weights, every
activation a convolution reads, and every activation gradient a convolution
reads; accumulation stays FP64 here (FP32 on the GPU).
"""
from __future__ import annotations

import itertools

import numpy as np

# (name, kind, cin, cout)
LAYERS = [
    ("enc1a", "conv3", 2, 16), ("enc1b", "conv3", 16, 16),
    ("enc2a", "conv3", 16, 32), ("enc2b", "conv3", 32, 32),
    ("mida", "conv3", 32, 64), ("midb", "conv3", 64, 64),
    ("up2", "tconv", 64, 32),
    ("dec2a", "conv3", 64, 32), ("dec2b", "conv3", 32, 32),
    ("up1", "tconv", 32, 16),
    ("dec1a", "conv3", 32, 16), ("dec1b", "conv3", 16, 16),
    ("head", "conv1", 16, 1),
]


def weight_shape(kind, cin, cout):
    if kind == "conv3":
        return (cout, cin, 3, 3, 3)
    if kind == "tconv":
        return (cin, cout, 2, 2, 2)
    return (cout, cin, 1, 1, 1)


def n_params():
    return sum(int(np.prod(weight_shape(k, ci, co))) + co for _, k, ci, co in LAYERS)


def init_params(seed=0):
    """He-normal weights, zero biases (float64 dict name -> (w, b))."""
    rng = np.random.default_rng(seed)
    P = {}
    for name, kind, ci, co in LAYERS:
        shp = weight_shape(kind, ci, co)
        fan_in = ci * (27 if kind == "conv3" else 8 if kind == "tconv" else 1)
        w = rng.standard_normal(shp) * np.sqrt(2.0 / fan_in)
        if name == "head":
            w *= 0.1
        P[name] = (w, np.zeros(co))
    return P


def flatten(P):
    """Canonical flat order: for each layer in LAYERS, weights (C order of
    weight_shape) then biases."""
    return np.concatenate([np.concatenate([P[n][0].ravel(), P[n][1]]) for n, *_ in LAYERS])


def unflatten(v):
    P, o = {}, 0
    for name, kind, ci, co in LAYERS:
        shp = weight_shape(kind, ci, co)
        k = int(np.prod(shp))
        P[name] = (np.asarray(v[o:o + k], np.float64).reshape(shp), np.asarray(v[o + k:o + k + co], np.float64))
        o += k + co
    return P


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


# --------------------------------------------------------------- primitives --
def conv3(x, w, b):
    """3x3x3 cross-correlation, zero padding 1: x [Ci,D,H,W], w [Co,Ci,3,3,3]."""
    ci, D, H, W = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))
    out = np.zeros((w.shape[0], D, H, W))
    for dz, dy, dx in itertools.product(range(3), repeat=3):
        out += np.tensordot(w[:, :, dz, dy, dx], xp[:, dz:dz + D, dy:dy + H, dx:dx + W], axes=(1, 0))
    return out + b[:, None, None, None]


def conv3_backward(x, w, g):
    """Gradients of conv3 wrt x, w and b, given the output gradient g."""
    ci, D, H, W = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dz, dy, dx in itertools.product(range(3), repeat=3):
        sl = (slice(None), slice(dz, dz + D), slice(dy, dy + H), slice(dx, dx + W))
        gxp[sl] += np.tensordot(w[:, :, dz, dy, dx], g, axes=(0, 0))
        gw[:, :, dz, dy, dx] = np.tensordot(g, xp[sl], axes=([1, 2, 3], [1, 2, 3]))
    return gxp[:, 1:-1, 1:-1, 1:-1], gw, g.sum(axis=(1, 2, 3))


def conv1(x, w, b):
    return np.tensordot(w[:, :, 0, 0, 0], x, axes=(1, 0)) + b[:, None, None, None]


def conv1_backward(x, w, g):
    return (np.tensordot(w[:, :, 0, 0, 0], g, axes=(0, 0)),
            np.tensordot(g, x, axes=([1, 2, 3], [1, 2, 3]))[:, :, None, None, None], g.sum(axis=(1, 2, 3)))


def tconv(x, w, b):
    """Transposed conv 2x2x2 stride 2: out[o, 2z+a, 2y+c, 2x+e] = sum_i w[i,o,a,c,e] x[i,z,y,x] + b[o]."""
    ci, D, H, W = x.shape
    out = np.zeros((w.shape[1], 2 * D, 2 * H, 2 * W))
    for a, c, e in itertools.product(range(2), repeat=3):
        out[:, a::2, c::2, e::2] = np.tensordot(w[:, :, a, c, e], x, axes=(0, 0))
    return out + b[:, None, None, None]


def tconv_backward(x, w, g):
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for a, c, e in itertools.product(range(2), repeat=3):
        gs = g[:, a::2, c::2, e::2]
        gx += np.tensordot(w[:, :, a, c, e], gs, axes=(1, 0))
        gw[:, :, a, c, e] = np.tensordot(x, gs, axes=([1, 2, 3], [1, 2, 3]))
    return gx, gw, g.sum(axis=(1, 2, 3))


def pool(x):
    C, D, H, W = x.shape
    return x.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).mean(axis=(2, 4, 6))


def pool_backward(g):
    return np.repeat(np.repeat(np.repeat(g, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


# ------------------------------------------------------------------ network --
def forward(P, x, bf16=False):
    """x [2, D, H, W] (dose, density); D, H, W multiples of 4.  Returns (y, cache)."""
    r = bf16_round if bf16 else (lambda a: a)
    W_ = {n: (r(w), b) for n, (w, b) in P.items()}
    c = {"x": r(x)}
    relu = lambda a: np.maximum(a, 0.0)
    c["e1a"] = r(relu(conv3(c["x"], *W_["enc1a"])))
    c["e1"] = r(relu(conv3(c["e1a"], *W_["enc1b"])))
    c["p1"] = r(pool(c["e1"]))
    c["e2a"] = r(relu(conv3(c["p1"], *W_["enc2a"])))
    c["e2"] = r(relu(conv3(c["e2a"], *W_["enc2b"])))
    c["p2"] = r(pool(c["e2"]))
    c["ma"] = r(relu(conv3(c["p2"], *W_["mida"])))
    c["m"] = r(relu(conv3(c["ma"], *W_["midb"])))
    c["u2"] = r(tconv(c["m"], *W_["up2"]))
    c["c2"] = np.concatenate([c["u2"], c["e2"]])
    c["d2a"] = r(relu(conv3(c["c2"], *W_["dec2a"])))
    c["d2"] = r(relu(conv3(c["d2a"], *W_["dec2b"])))
    c["u1"] = r(tconv(c["d2"], *W_["up1"]))
    c["c1"] = np.concatenate([c["u1"], c["e1"]])
    c["d1a"] = r(relu(conv3(c["c1"], *W_["dec1a"])))
    c["d1"] = r(relu(conv3(c["d1a"], *W_["dec1b"])))
    y = conv1(c["d1"], *W_["head"])[0] + x[0]
    c["W"] = W_
    return y, c


def backward(c, gy, bf16=False, acts=None):
    """Gradients (dict name -> (gw, gb)) of a scalar whose gradient wrt the
    output y is gy.  With a dict `acts`, it also receives the activation
    gradients (gd1 ... ge1a, as stored: masked by the ReLU, rounded)."""
    r = bf16_round if bf16 else (lambda a: a)
    W_ = c["W"]
    G = {}
    g = gy[None]
    gd1, *G["head"] = conv1_backward(c["d1"], W_["head"][0], g)
    gd1 = r(gd1 * (c["d1"] > 0))
    gd1a, *G["dec1b"] = conv3_backward(c["d1a"], W_["dec1b"][0], gd1)
    gd1a = r(gd1a * (c["d1a"] > 0))
    gc1, *G["dec1a"] = conv3_backward(c["c1"], W_["dec1a"][0], gd1a)
    gc1 = r(gc1)
    gu1, ge1_skip = gc1[:16], gc1[16:]
    gd2, *G["up1"] = tconv_backward(c["d2"], W_["up1"][0], gu1)
    gd2 = r(gd2 * (c["d2"] > 0))
    gd2a, *G["dec2b"] = conv3_backward(c["d2a"], W_["dec2b"][0], gd2)
    gd2a = r(gd2a * (c["d2a"] > 0))
    gc2, *G["dec2a"] = conv3_backward(c["c2"], W_["dec2a"][0], gd2a)
    gc2 = r(gc2)
    gu2, ge2_skip = gc2[:32], gc2[32:]
    gm, *G["up2"] = tconv_backward(c["m"], W_["up2"][0], gu2)
    gm = r(gm * (c["m"] > 0))
    gma, *G["midb"] = conv3_backward(c["ma"], W_["midb"][0], gm)
    gma = r(gma * (c["ma"] > 0))
    gp2, *G["mida"] = conv3_backward(c["p2"], W_["mida"][0], gma)
    ge2 = r((r(pool_backward(gp2)) + ge2_skip) * (c["e2"] > 0))
    ge2a, *G["enc2b"] = conv3_backward(c["e2a"], W_["enc2b"][0], ge2)
    ge2a = r(ge2a * (c["e2a"] > 0))
    gp1, *G["enc2a"] = conv3_backward(c["p1"], W_["enc2a"][0], ge2a)
    ge1 = r((r(pool_backward(gp1)) + ge1_skip) * (c["e1"] > 0))
    ge1a, *G["enc1b"] = conv3_backward(c["e1a"], W_["enc1b"][0], ge1)
    ge1a = r(ge1a * (c["e1a"] > 0))
    _, *G["enc1a"] = conv3_backward(c["x"], W_["enc1a"][0], ge1a)
    if acts is not None:
        acts.update(gd1=gd1, gd1a=gd1a, gc1=gc1, gd2=gd2, gd2a=gd2a, gc2=gc2, gm=gm, gma=gma, gp2=r(gp2),
                    ge2=ge2, ge2a=ge2a, gp1=r(gp1), ge1=ge1, ge1a=ge1a)
    return {k: (gw, gb) for k, (gw, gb) in G.items()}


def loss_and_grad(P, x, target, bf16=False):
    y, c = forward(P, x, bf16)
    d = y - target
    loss = float(np.mean(d * d))
    gy = 2.0 * d / d.size
    return loss, backward(c, gy, bf16), y


def adam(v, g, m, s, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015) on flat arrays; returns new (v, m, s)."""
    m = b1 * m + (1 - b1) * g
    s = b2 * s + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    sh = s / (1 - b2 ** t)
    return v - lr * mh / (np.sqrt(sh) + eps), m, s
