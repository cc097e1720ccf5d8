"""Pins of the denoiser oracle: brute-force loops, PyTorch CPU operators (an
independent implementation, run only), finite differences, bfloat16 rounding
and Adam closed forms."""
import itertools

import numpy as np
import pytest
import torch
import torch.nn.functional as TF

from oracle import unet_ref as U


def test_parameter_count():
    assert U.n_params() == 339_681
    P = U.init_params(1)
    assert U.flatten(P).size == 339_681
    v = U.flatten(P)
    assert np.array_equal(U.flatten(U.unflatten(v)), v)


def test_conv3_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 4, 5))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    y = U.conv3(x, w, b)
    for o, z, yy, xx in itertools.product(range(3), range(3), range(4), range(5)):
        s = b[o]
        for i, dz, dy, dx in itertools.product(range(2), range(3), range(3), range(3)):
            zz, y2, x2 = z + dz - 1, yy + dy - 1, xx + dx - 1
            if 0 <= zz < 3 and 0 <= y2 < 4 and 0 <= x2 < 5:
                s += w[o, i, dz, dy, dx] * x[i, zz, y2, x2]
        assert abs(y[o, z, yy, xx] - s) < 1e-12


def test_primitives_match_torch_cpu():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 6, 4, 8))
    w3 = rng.standard_normal((5, 4, 3, 3, 3))
    b5 = rng.standard_normal(5)
    ref = TF.conv3d(torch.tensor(x)[None], torch.tensor(w3), torch.tensor(b5), padding=1)[0].numpy()
    assert np.allclose(U.conv3(x, w3, b5), ref, atol=1e-12)
    wt = rng.standard_normal((4, 3, 2, 2, 2))
    b3 = rng.standard_normal(3)
    ref = TF.conv_transpose3d(torch.tensor(x)[None], torch.tensor(wt), torch.tensor(b3), stride=2)[0].numpy()
    assert np.allclose(U.tconv(x, wt, b3), ref, atol=1e-12)
    assert np.allclose(U.pool(x), TF.avg_pool3d(torch.tensor(x)[None], 2)[0].numpy(), atol=1e-14)
    w1 = rng.standard_normal((2, 4, 1, 1, 1))
    ref = TF.conv3d(torch.tensor(x)[None], torch.tensor(w1), torch.tensor(b5[:2]))[0].numpy()
    assert np.allclose(U.conv1(x, w1, b5[:2]), ref, atol=1e-12)


def _fd_check(f, args, grads, idx_list, h=1e-6):
    """central differences of the scalar f(*args) against analytic grads"""
    for a_i, idx in idx_list:
        a = args[a_i]
        old = a[idx]
        a[idx] = old + h
        fp = f(*args)
        a[idx] = old - h
        fm = f(*args)
        a[idx] = old
        num = (fp - fm) / (2 * h)
        assert abs(num - grads[a_i][idx]) <= 1e-6 * max(1.0, abs(num)), (a_i, idx, num, grads[a_i][idx])


def test_primitive_backward_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 4, 4, 4))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    g = rng.standard_normal((2, 4, 4, 4))
    f = lambda x, w: float(np.sum(U.conv3(x, w, b) * g))
    gx, gw, gb = U.conv3_backward(x, w, g)
    assert np.allclose(gb, g.sum(axis=(1, 2, 3)))
    picks = [(0, tuple(rng.integers(0, s) for s in x.shape)) for _ in range(12)]
    picks += [(1, tuple(rng.integers(0, s) for s in w.shape)) for _ in range(12)]
    _fd_check(f, [x, w], [gx, gw], picks)
    wt = rng.standard_normal((3, 2, 2, 2, 2))
    gt = rng.standard_normal((2, 8, 8, 8))
    f = lambda x, wt: float(np.sum(U.tconv(x, wt, b) * gt))
    gx, gw, _ = U.tconv_backward(x, wt, gt)
    picks = [(0, tuple(rng.integers(0, s) for s in x.shape)) for _ in range(8)]
    picks += [(1, tuple(rng.integers(0, s) for s in wt.shape)) for _ in range(8)]
    _fd_check(f, [x, wt], [gx, gw], picks)
    gp = rng.standard_normal((3, 2, 2, 2))
    assert np.isclose(np.sum(U.pool(x) * gp), np.sum(x * U.pool_backward(gp)))


def test_network_gradient_finite_differences():
    """Whole U-Net in FP64 (no rounding), 8^3 input, random parameters."""
    rng = np.random.default_rng(3)
    P = U.init_params(3)
    for n in P:                                  # non-zero biases exercise every term
        P[n] = (P[n][0], 0.1 * rng.standard_normal(P[n][1].shape))
    x = rng.random((2, 8, 8, 8))
    t = rng.random((8, 8, 8))
    loss, G, _ = U.loss_and_grad(P, x, t)
    v = U.flatten(P)
    gv = U.flatten(G)
    h = 1e-6
    for k in rng.choice(v.size, 40, replace=False):
        vp, vm = v.copy(), v.copy()
        vp[k] += h
        vm[k] -= h
        lp = U.loss_and_grad(U.unflatten(vp), x, t)[0]
        lm = U.loss_and_grad(U.unflatten(vm), x, t)[0]
        num = (lp - lm) / (2 * h)
        assert abs(num - gv[k]) <= 1e-5 * max(1e-3, abs(num)) + 1e-9, (k, num, gv[k])


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7, -2.5, 3.14159, 1e-30, 65504.0])
    exp = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.bf16_round(vals), exp)
    assert U.bf16_round(np.array([1.0 + 2 ** -8]))[0] == 1.0          # tie -> even
    assert U.bf16_round(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6   # tie -> even (up)
    r = np.random.default_rng(5).standard_normal(10000) * 100
    exp = torch.tensor(r, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.bf16_round(r), exp)


def test_adam_step():
    rng = np.random.default_rng(6)
    v = rng.standard_normal(50)
    g = rng.standard_normal(50)
    m = np.zeros(50)
    s = np.zeros(50)
    v1, m1, s1 = U.adam(v, g, m, s, 1, lr=1e-3)
    # first step: m_hat = g, s_hat = g^2 -> step = lr * g / (|g| + eps)
    assert np.allclose(v1, v - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    t = torch.tensor(v, requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    vv, mm, ss = v.copy(), m, s
    for step in range(1, 4):
        gg = rng.standard_normal(50)
        t.grad = torch.tensor(gg)
        opt.step()
        vv, mm, ss = U.adam(vv, gg, mm, ss, step, lr=1e-3)
    assert np.allclose(vv, t.detach().numpy(), rtol=0, atol=1e-12)
