"""The denoiser's BF16-MFMA kernels against the oracle (oracle/unet_ref.py),
element by element, on a crop of 20 x 24 x 136 voxels (z, y, x): at the
coarsest level (5 x 6 x 34) every layer still has several 16 x 4 x 4 output
tiles along each axis with partial tiles at the far edges, the 64-channel
layers stage their input in two phases, and the full-resolution layers run
hundreds of tiles.

Two comparisons, for every activation, every activation gradient and every
parameter gradient:
  * layer by layer: the oracle's primitive (conv3, its adjoint, the transposed
    convolution, the pool) applied to the bf16 operands the GPU layer actually
    read, rounded to bf16 where the GPU stores bf16 - the GPU value must agree
    within 2^-7 of itself plus 1e-5 of the buffer's RMS (a bf16 value may land
    one unit of the last place away after FP32 accumulation in another order),
    parameter gradients within 1e-3 of themselves plus 1e-4 of the RMS;
  * end to end: the oracle's whole forward and backward pass from the same
    input.  A bf16 value one unit in the last place apart upstream (FP32
    accumulation in another order lands on the other side of a rounding
    boundary) moves every value computed from it downstream, and such flips
    multiply from layer to layer (an output depends on 27 x C rounded inputs),
    so after a few layers most values differ by some units in the last place.
    The tolerance is therefore the oracle's own spread: a second oracle pass in
    which every stored activation and gradient is perturbed by a relative
    2^-24 N(0, 1) before its bf16 rounding (FP32's unit roundoff; the spread
    it produces downstream hardly depends on that size, since the flips
    saturate) gives the differences its arithmetic admits.  A
    buffer passes if 99.9% of its elements are within 2^-7 of themselves plus
    1e-3 of the RMS and all within 2^-7 of themselves plus 1e-2 of the RMS (no
    cascade), or if its differences from the oracle are no larger than the
    perturbed pass's: RMS and 99.9th percentile within 2x, largest within 4x
    (plus 1e-4 of the buffer's RMS).
The 2 x 2 x 2 average pools are exact: bf16 of the FP32 mean of the eight
bf16 children."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import unet_ref as U  # noqa: E402
from paper_1011_2188_amd import fdc as F  # noqa: E402

SHAPE = (20, 24, 136)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


def _rms(a):
    return float(np.sqrt(np.mean(np.square(a))))


def _levels():
    return [SHAPE, tuple(s // 2 for s in SHAPE), tuple(s // 4 for s in SHAPE)]


@pytest.fixture(scope="module")
def run():
    rng = np.random.default_rng(23)
    P = U.init_params(23)
    for n in P:                                   # biases that move the ReLU thresholds
        P[n] = (P[n][0], 0.05 * rng.standard_normal(P[n][1].shape))
    flat = U.flatten(P).astype(np.float32)
    x = np.stack([rng.random(SHAPE) * 2.0, 0.5 + rng.random(SHAPE)]).astype(np.float32)
    t = (x[0] + 0.1 * rng.standard_normal(SHAPE)).astype(np.float32)
    net = F.UNet(SHAPE)
    net.set_params(flat)
    xin = torch.tensor(x, device="cuda")
    y = torch.empty(SHAPE, device="cuda")
    net.forward(xin, y)
    torch.cuda.synchronize()
    out = {"y": y.cpu().numpy().astype(np.float64)}
    for name in F.UNET_BUFFERS[:13]:
        out[name] = net.debug_buffer(name).astype(np.float64)
    net.backward(xin, torch.tensor(t, device="cuda"), want_loss=False)
    torch.cuda.synchronize()
    for name in F.UNET_BUFFERS[13:]:
        out[name] = net.debug_buffer(name).astype(np.float64)
    out["grads"] = net.get_grads().astype(np.float64)
    net.close()
    Wf = U.unflatten(flat.astype(np.float64))
    xo = x.astype(np.float64)
    yo, cache = U.forward(Wf, xo, bf16=True)
    d = yo - t.astype(np.float64)
    acts = {}
    G = U.backward(cache, 2.0 * d / d.size, bf16=True, acts=acts)
    pert = _perturbed_pass(Wf, xo, t.astype(np.float64))
    return dict(gpu=out, W=cache["W"], cache=cache, yo=yo, G=G, acts=acts, x=xo, t=t.astype(np.float64), pert=pert)


def _perturbed_pass(Wf, xo, t):
    """The oracle's forward and backward pass with every value it stores as
    bf16 first perturbed by a relative 2^-24 N(0, 1) (FP32's unit roundoff).
    Weights and input are rounded beforehand, so the perturbation (far below
    half a unit in the last place) leaves them as they are."""
    rng = np.random.default_rng(77)
    exact = U.bf16_round
    Wr = {n: (exact(w), b) for n, (w, b) in Wf.items()}
    xr = np.stack([exact(xo[0]), exact(xo[1])])

    def noisy(a):
        a = np.asarray(a, np.float64)
        return exact(a * (1.0 + 2.0 ** -24 * rng.standard_normal(a.shape)))
    U.bf16_round = noisy
    try:
        yp, cp = U.forward(Wr, xr, bf16=True)
        yp = yp - xr[0] + xo[0]                        # the residual adds the unrounded input
        dp = yp - t
        acts = {}
        G = U.backward(cp, 2.0 * dp / dp.size, bf16=True, acts=acts)
    finally:
        U.bf16_round = exact
    return dict(cache=cp, yo=yp, acts=acts, G=G)


def _cf(buf, lvl, c0, c1):
    """GPU channels-last buffer [voxels, pitch] -> channels-first [C, D, H, W]."""
    nz, ny, nx = _levels()[lvl]
    return buf[:, c0:c1].T.reshape(c1 - c0, nz, ny, nx)


def _check(name, got, want, rel, abs_frac):
    bound = rel * np.abs(want) + abs_frac * _rms(want) + 1e-30
    worst = float(np.max(np.abs(got - want) / bound))
    print(f"{name}: worst at {worst:.3f} of the bound (rms {_rms(want):.3e})")
    assert worst <= 1.0, name


def _check_cascade(name, got, want, pert, failures):
    """End to end (see the module notes): within one unit in the last place
    (99.9% within 2^-7 |x| + 1e-3 RMS, all within 2^-7 |x| + 1e-2 RMS), or no
    larger than the perturbed oracle pass's differences (`pert`): RMS and
    99.9th percentile within 2x, largest within 4x, plus 1e-4 RMS."""
    r = np.abs(got - want)
    rp = np.abs(pert - want)
    rms = _rms(want)
    tight = 2.0 ** -7 * np.abs(want) + 1e-3 * rms + 1e-30
    loose = 2.0 ** -7 * np.abs(want) + 1e-2 * rms + 1e-30
    frac = float(np.mean(r <= tight))
    worst_l = float(np.max(r / loose))
    stats = [(_rms(r), _rms(rp)), (float(np.quantile(r, 0.999)), float(np.quantile(rp, 0.999))),
             (float(r.max()), float(rp.max()))]
    ratios = [a / (b + 1e-4 * rms + 1e-300) for a, b in stats]
    print(f"{name}: {frac:.6f} within one ulp, worst at {worst_l:.3f} of the loose bound; against the "
          f"perturbed oracle: rms {stats[0][0]:.3e}/{stats[0][1]:.3e}, q99.9 {stats[1][0]:.3e}/{stats[1][1]:.3e}, "
          f"max {stats[2][0]:.3e}/{stats[2][1]:.3e}")
    one_ulp = frac >= 0.999 and worst_l <= 1.0
    spread = ratios[0] <= 2.0 and ratios[1] <= 2.0 and ratios[2] <= 4.0
    if not (one_ulp or spread):
        failures.append(name)


# the GPU buffer, level and channels of each forward activation
ACT = {"e1a": ("e1a", 0, 0, 16), "e1": ("c1", 0, 16, 32), "p1": ("p1", 1, 0, 16), "e2a": ("e2a", 1, 0, 32),
       "e2": ("c2", 1, 32, 64), "p2": ("p2", 2, 0, 32), "ma": ("ma", 2, 0, 64), "m": ("m", 2, 0, 64),
       "u2": ("c2", 1, 0, 32), "d2a": ("d2a", 1, 0, 32), "d2": ("d2", 1, 0, 32), "u1": ("c1", 0, 0, 16),
       "d1a": ("d1a", 0, 0, 16), "d1": ("d1", 0, 0, 16)}
# activation gradients: GPU buffer, level, channels, the oracle's name
GRAD = {"gd1": (0, 16), "gd1a": (0, 16), "gc1": (0, 32), "gd2": (1, 32), "gd2a": (1, 32), "gc2": (1, 64),
        "gm": (2, 64), "gma": (2, 64), "gp2": (2, 32), "ge2": (1, 32), "ge2a": (1, 32), "gp1": (1, 16),
        "ge1": (0, 16), "ge1a": (0, 16)}


def act(g, name):
    buf, lvl, c0, c1 = ACT[name]
    return _cf(g[buf], lvl, c0, c1)


def grad(g, name):
    lvl, ch = GRAD[name]
    return _cf(g[name], lvl, 0, ch)


def test_pools_exact(run):
    g = run["gpu"]
    for child, coarse in (("e1", "p1"), ("e2", "p2")):
        c = act(g, child)
        C, D, H, W = c.shape
        s = c.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).sum(axis=(2, 4, 6))   # exact in FP64
        want = U.bf16_round(np.float32(0.125) * s.astype(np.float32))
        assert np.array_equal(act(g, coarse), want), coarse


def test_forward_layer_by_layer(run):
    g, W = run["gpu"], run["W"]
    x = _cf(g["x"], 0, 0, 2)
    relu = lambda a: np.maximum(a, 0.0)
    r = U.bf16_round
    steps = [("e1a", U.conv3, x, "enc1a", True), ("e1", U.conv3, act(g, "e1a"), "enc1b", True),
             ("e2a", U.conv3, act(g, "p1"), "enc2a", True), ("e2", U.conv3, act(g, "e2a"), "enc2b", True),
             ("ma", U.conv3, act(g, "p2"), "mida", True), ("m", U.conv3, act(g, "ma"), "midb", True),
             ("u2", U.tconv, act(g, "m"), "up2", False),
             ("d2a", U.conv3, np.concatenate([act(g, "u2"), act(g, "e2")]), "dec2a", True),
             ("d2", U.conv3, act(g, "d2a"), "dec2b", True), ("u1", U.tconv, act(g, "d2"), "up1", False),
             ("d1a", U.conv3, np.concatenate([act(g, "u1"), act(g, "e1")]), "dec1a", True),
             ("d1", U.conv3, act(g, "d1a"), "dec1b", True)]
    for name, op, inp, layer, has_relu in steps:
        want = op(inp, *W[layer])
        want = r(relu(want) if has_relu else want)
        _check(f"{name} (layer)", act(g, name), want, 2.0 ** -7, 1e-5)
    head = U.conv1(act(g, "d1"), *W["head"])[0] + run["x"][0]
    _check("y (layer)", g["y"], head, 1e-5, 1e-5)


def test_forward_end_to_end(run):
    g, c, pc = run["gpu"], run["cache"], run["pert"]["cache"]
    bad = []
    for name in ACT:
        _check_cascade(f"{name} (end to end)", act(g, name), c[name], pc[name], bad)
    _check_cascade("y (end to end)", g["y"] - run["x"][0], run["yo"] - run["x"][0],
                   run["pert"]["yo"] - run["x"][0], bad)
    assert not bad, bad


def _backward_layers(g, W, gy):
    """Each activation gradient from the GPU's own upstream gradient and
    activations, with the oracle's adjoints (mask, bf16 rounding as stored)."""
    r = U.bf16_round
    out = {}
    gd1 = U.conv1_backward(act(g, "d1"), W["head"][0], gy[None])[0]
    out["gd1"] = r(gd1 * (act(g, "d1") > 0))
    out["gd1a"] = r(U.conv3_backward(act(g, "d1a"), W["dec1b"][0], grad(g, "gd1"))[0] * (act(g, "d1a") > 0))
    c1 = np.concatenate([act(g, "u1"), act(g, "e1")])
    out["gc1"] = r(U.conv3_backward(c1, W["dec1a"][0], grad(g, "gd1a"))[0])
    gc1 = grad(g, "gc1")
    out["gd2"] = r(U.tconv_backward(act(g, "d2"), W["up1"][0], gc1[:16])[0] * (act(g, "d2") > 0))
    out["gd2a"] = r(U.conv3_backward(act(g, "d2a"), W["dec2b"][0], grad(g, "gd2"))[0] * (act(g, "d2a") > 0))
    c2 = np.concatenate([act(g, "u2"), act(g, "e2")])
    out["gc2"] = r(U.conv3_backward(c2, W["dec2a"][0], grad(g, "gd2a"))[0])
    gc2 = grad(g, "gc2")
    out["gm"] = r(U.tconv_backward(act(g, "m"), W["up2"][0], gc2[:32])[0] * (act(g, "m") > 0))
    out["gma"] = r(U.conv3_backward(act(g, "ma"), W["midb"][0], grad(g, "gm"))[0] * (act(g, "ma") > 0))
    out["gp2"] = r(U.conv3_backward(act(g, "p2"), W["mida"][0], grad(g, "gma"))[0])
    out["ge2"] = r((r(U.pool_backward(grad(g, "gp2"))) + gc2[32:]) * (act(g, "e2") > 0))
    out["ge2a"] = r(U.conv3_backward(act(g, "e2a"), W["enc2b"][0], grad(g, "ge2"))[0] * (act(g, "e2a") > 0))
    out["gp1"] = r(U.conv3_backward(act(g, "p1"), W["enc2a"][0], grad(g, "ge2a"))[0])
    out["ge1"] = r((r(U.pool_backward(grad(g, "gp1"))) + gc1[16:]) * (act(g, "e1") > 0))
    out["ge1a"] = r(U.conv3_backward(act(g, "e1a"), W["enc1b"][0], grad(g, "ge1"))[0] * (act(g, "e1a") > 0))
    return out


def test_backward_data_layer_by_layer(run):
    g = run["gpu"]
    d = g["y"] - run["t"]
    want = _backward_layers(g, run["W"], 2.0 * d / d.size)
    for name in GRAD:
        _check(f"{name} (layer)", grad(g, name), want[name], 2.0 ** -7, 1e-5)


def test_backward_data_end_to_end(run):
    """Every activation gradient against the oracle's own backward pass."""
    g = run["gpu"]
    bad = []
    for name in GRAD:
        _check_cascade(f"{name} (end to end)", grad(g, name), run["acts"][name], run["pert"]["acts"][name], bad)
    assert not bad, bad


def _offsets():
    offs, off = {}, 0
    for name, kind, ci, co in U.LAYERS:
        nw = int(np.prod(U.weight_shape(kind, ci, co)))
        offs[name] = (off, nw, co)
        off += nw + co
    return offs


def test_parameter_gradients_layer_by_layer(run):
    """Every weight and bias gradient from the GPU's own operands (its bf16
    activations and activation gradients) with the oracle's adjoints."""
    g, W = run["gpu"], run["W"]
    d = g["y"] - run["t"]
    gy = (2.0 * d / d.size)[None]
    ins = {"enc1a": _cf(g["x"], 0, 0, 2), "enc1b": act(g, "e1a"), "enc2a": act(g, "p1"), "enc2b": act(g, "e2a"),
           "mida": act(g, "p2"), "midb": act(g, "ma"), "up2": act(g, "m"),
           "dec2a": np.concatenate([act(g, "u2"), act(g, "e2")]), "dec2b": act(g, "d2a"), "up1": act(g, "d2"),
           "dec1a": np.concatenate([act(g, "u1"), act(g, "e1")]), "dec1b": act(g, "d1a"), "head": act(g, "d1")}
    gout = {"enc1a": grad(g, "ge1a"), "enc1b": grad(g, "ge1"), "enc2a": grad(g, "ge2a"), "enc2b": grad(g, "ge2"),
            "mida": grad(g, "gma"), "midb": grad(g, "gm"), "up2": grad(g, "gc2")[:32], "dec2a": grad(g, "gd2a"),
            "dec2b": grad(g, "gd2"), "up1": grad(g, "gc1")[:16], "dec1a": grad(g, "gd1a"), "dec1b": grad(g, "gd1"),
            "head": gy}
    offs = _offsets()
    for name, kind, ci, co in U.LAYERS:
        op = {"conv3": U.conv3_backward, "tconv": U.tconv_backward, "conv1": U.conv1_backward}[kind]
        _, gw, gb = op(ins[name], W[name][0], gout[name])
        o, nw, _ = offs[name]
        _check(f"{name} weights (layer)", run["gpu"]["grads"][o:o + nw].reshape(gw.shape), gw, 1e-3, 1e-4)
        _check(f"{name} biases (layer)", run["gpu"]["grads"][o + nw:o + nw + co], gb, 1e-3, 1e-4)


def test_parameter_gradients_end_to_end(run):
    offs = _offsets()
    bad = []
    for name, kind, ci, co in U.LAYERS:
        gw, gb = run["G"][name]
        pw, pb = run["pert"]["G"][name]
        o, nw, _ = offs[name]
        _check_cascade(f"{name} weights (end to end)", run["gpu"]["grads"][o:o + nw].reshape(gw.shape), gw, pw, bad)
        _check_cascade(f"{name} biases (end to end)", run["gpu"]["grads"][o + nw:o + nw + co], gb, pb, bad)
    assert not bad, bad
