"""The BF16-MFMA denoiser kernels (through the C ABI) against the FP64 oracle
that rounds to bfloat16 at the same storage points.  Criteria: prediction and
per-layer parameter gradients within 1e-2 (2e-2 for gradients) of the oracle's
RMS; Adam exact to FP32 rounding; a single crop can be over-fitted."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import unet_ref as U  # noqa: E402
from paper_1011_2188_amd import fdc as F  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


def _case(shape, seed):
    rng = np.random.default_rng(seed)
    P = U.init_params(seed)
    for n in P:
        P[n] = (P[n][0], 0.05 * rng.standard_normal(P[n][1].shape))
    nz, ny, nx = shape
    x = np.stack([rng.random(shape) * 2.0, 0.5 + rng.random(shape)])
    t = x[0] + 0.1 * rng.standard_normal(shape)
    return P, x, t


def _rms(a):
    return float(np.sqrt(np.mean(np.square(a))))


def test_unet_parameter_count():
    assert F.lib().fdc_unet_num_params() == U.n_params() == 339_681


@pytest.mark.parametrize("shape", [(8, 8, 16), (16, 12, 8)])
def test_unet_forward_matches_oracle(shape):
    P, x, _ = _case(shape, 1)
    net = F.UNet(shape)
    flat = U.flatten(P).astype(np.float32)
    net.set_params(flat)
    xin = torch.tensor(x, dtype=torch.float32, device="cuda")
    y = torch.empty(shape, dtype=torch.float32, device="cuda")
    net.forward(xin, y)
    torch.cuda.synchronize()
    yo, cache = U.forward(U.unflatten(flat.astype(np.float64)), x.astype(np.float32).astype(np.float64), bf16=True)
    # layer by layer (channels-last buffers vs channels-first oracle)
    for name, key, ch in [("e1a", "e1a", 16), ("d1", "d1", 16), ("m", "m", 64)]:
        g = net.debug_buffer(name)[:, :ch]
        o = cache[key].reshape(ch, -1).T
        assert _rms(g - o) <= 1e-2 * _rms(o), name
    h_g = y.cpu().numpy() - x[0]
    h_o = yo - x[0]
    assert _rms(h_g - h_o) <= 1e-2 * _rms(h_o)


def test_unet_gradients_match_oracle():
    shape = (8, 8, 8)
    P, x, t = _case(shape, 2)
    net = F.UNet(shape)
    flat = U.flatten(P).astype(np.float32)
    net.set_params(flat)
    xin = torch.tensor(x, dtype=torch.float32, device="cuda")
    tt = torch.tensor(t, dtype=torch.float32, device="cuda")
    loss = net.backward(xin, tt)
    gg = net.get_grads()
    lo, G, _ = U.loss_and_grad(U.unflatten(flat.astype(np.float64)), x.astype(np.float32).astype(np.float64),
                               t.astype(np.float32).astype(np.float64), bf16=True)
    assert abs(loss / lo - 1) < 1e-3
    go = U.flatten(G)
    off = 0
    for name, kind, ci, co in U.LAYERS:
        nw = int(np.prod(U.weight_shape(kind, ci, co)))
        for a, b, what in [(off, off + nw, "w"), (off + nw, off + nw + co, "b")]:
            assert _rms(gg[a:b] - go[a:b]) <= 2e-2 * _rms(go[a:b]) + 1e-12, (name, what)
        off += nw + co


def test_unet_adam_matches_oracle():
    shape = (8, 8, 8)
    P, x, t = _case(shape, 3)
    net = F.UNet(shape)
    flat = U.flatten(P).astype(np.float32)
    net.set_params(flat)
    xin = torch.tensor(x, dtype=torch.float32, device="cuda")
    tt = torch.tensor(t, dtype=torch.float32, device="cuda")
    v, m, s = flat.astype(np.float64), np.zeros(flat.size), np.zeros(flat.size)
    for step in (1, 2):
        net.backward(xin, tt, want_loss=False)
        g = net.get_grads().astype(np.float64)
        net.adam(1e-3)
        v, m, s = U.adam(v, g, m, s, step, lr=1e-3)
        got = net.get_params()
        assert np.max(np.abs(got - v)) <= 1e-6 * max(1.0, np.max(np.abs(v)))


def test_unet_overfits_one_crop():
    shape = (16, 16, 16)
    P, x, t = _case(shape, 4)
    net = F.UNet(shape)
    net.set_params(U.flatten(P).astype(np.float32))
    xin = torch.tensor(x, dtype=torch.float32, device="cuda")
    tt = torch.tensor(t, dtype=torch.float32, device="cuda")
    first = net.backward(xin, tt)
    net.adam(3e-3)
    for _ in range(150):
        net.backward(xin, tt, want_loss=False)
        net.adam(3e-3)
    last = net.backward(xin, tt)
    assert last < 0.2 * first


def _wgrad3_fp64(gout, inp, shape):
    """dW[co, ci, dz, dy, dx] = sum over voxels v of gout[v, co] * inp[v + (dz, dy, dx) - 1, ci]
    (zero outside), in FP64 from the bf16 values the kernels contracted."""
    nz, ny, nx = shape
    co, ci = gout.shape[1], inp.shape[1]
    g = gout.astype(np.float64)
    xp = np.pad(inp.astype(np.float64).reshape(nz, ny, nx, ci), ((1, 1), (1, 1), (1, 1), (0, 0)))
    dw = np.zeros((co, ci, 3, 3, 3))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                dw[:, :, dz, dy, dx] = g.T @ xp[dz:dz + nz, dy:dy + ny, dx:dx + nx].reshape(-1, ci)
    return dw


def test_unet_weight_gradients_multi_tile():
    """Weight gradients of one 3x3x3 layer per kernel shape (16, 16 x 32, 32 and
    64 channels) and of both transposed convolutions on a 64 x 128 x 128 crop,
    where every workgroup walks several tiles or row slabs, against an FP64
    contraction of the same bf16 operands."""
    shape = (64, 128, 128)
    rng = np.random.default_rng(7)
    P = U.init_params(7)
    flat = U.flatten(P).astype(np.float32)
    x = np.stack([rng.random(shape) * 2.0, 0.5 + rng.random(shape)]).astype(np.float32)
    t = (x[0] + 0.1 * rng.standard_normal(shape)).astype(np.float32)
    net = F.UNet(shape)
    net.set_params(flat)
    net.backward(torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda"), want_loss=False)
    gg = net.get_grads()
    offs, off = {}, 0
    for name, kind, ci, co in U.LAYERS:
        offs[name] = off
        off += int(np.prod(U.weight_shape(kind, ci, co))) + co
    levels = [shape, tuple(s // 2 for s in shape), tuple(s // 4 for s in shape)]
    for layer, gname, iname, lvl, ci, co in [("enc1b", "ge1", "e1a", 0, 16, 16), ("dec1a", "gd1a", "c1", 0, 32, 16),
                                             ("enc2b", "ge2", "e2a", 1, 32, 32), ("midb", "gm", "ma", 2, 64, 64)]:
        want = _wgrad3_fp64(net.debug_buffer(gname)[:, :co], net.debug_buffer(iname)[:, :ci], levels[lvl])
        got = gg[offs[layer]:offs[layer] + want.size].reshape(want.shape)
        err = float(np.max(np.abs(got - want))) / _rms(want)
        print(f"{layer}: max |GPU - FP64| = {err:.2e} of the RMS gradient")
        assert err <= 1e-4, layer
    # transposed convolutions (2x2x2, stride 2): dW[ci, co, a, b, c] = sum over coarse
    # voxels v of input[v, ci] * output gradient[2 v + (a, b, c), co]; the gradient of
    # up1 (up2) is the first 16 (32) channels of the level-0 (level-1) concatenation's
    for layer, iname, gname, lvl, ci, co in [("up1", "d2", "gc1", 1, 32, 16), ("up2", "m", "gc2", 2, 64, 32)]:
        cz, cy, cx = levels[lvl]
        x_in = net.debug_buffer(iname)[:, :ci].astype(np.float64)
        g_f = net.debug_buffer(gname)[:, :co].astype(np.float64).reshape(2 * cz, 2 * cy, 2 * cx, co)
        want = np.zeros((ci, co, 2, 2, 2))
        for a in range(2):
            for b in range(2):
                for c in range(2):
                    want[:, :, a, b, c] = x_in.T @ g_f[a::2, b::2, c::2].reshape(-1, co)
        got = gg[offs[layer]:offs[layer] + want.size].reshape(want.shape)
        err = float(np.max(np.abs(got - want))) / _rms(want)
        print(f"{layer}: max |GPU - FP64| = {err:.2e} of the RMS gradient")
        assert err <= 1e-4, layer
    net.close()


def test_unet_forward_full_volume_sampled():
    """The full 128 x 256 x 256 (z, y, x) volume the denoiser is timed on: three
    3x3x3 layers (2 -> 16, 16 -> 16, and 64 -> 32 at half resolution, whose 64
    input channels are staged 32 at a time) recomputed in FP64 at sampled voxels
    (random, corners and tile edges) from the kernels' own bf16 inputs and the
    bf16-rounded weights; the GPU output is bf16, so each value must agree within
    2^-7 of itself plus 1e-3 of the layer's RMS."""
    shape = (128, 256, 256)
    rng = np.random.default_rng(11)
    flat = U.flatten(U.init_params(11)).astype(np.float32)
    W = U.unflatten(flat.astype(np.float64))
    net = F.UNet(shape)
    net.set_params(flat)
    g = torch.Generator(device="cuda").manual_seed(11)
    x = torch.rand((2,) + shape, device="cuda", generator=g)
    y = torch.empty(shape, device="cuda")
    net.forward(x, y)
    torch.cuda.synchronize()
    for layer, src, s_ch, dst, d_off, d_ch, div in [("enc1a", "x", 2, "e1a", 0, 16, 1),
                                                    ("enc1b", "e1a", 16, "c1", 16, 16, 1),
                                                    ("dec2a", "c2", 64, "d2a", 0, 32, 2)]:
        nz, ny, nx = (s // div for s in shape)
        xin = net.debug_buffer(src)[:, :s_ch].reshape(nz, ny, nx, s_ch).astype(np.float64)
        out = net.debug_buffer(dst)[:, d_off:d_off + d_ch].reshape(nz, ny, nx, d_ch).astype(np.float64)
        w = U.bf16_round(W[layer][0])                      # [co, ci, dz, dy, dx]
        b = W[layer][1]
        pts = [tuple(int(rng.integers(0, n)) for n in (nz, ny, nx)) for _ in range(240)]
        pts += [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (3, 3, 15), (4, 4, 16), (nz - 1, 0, nx - 1), (7, ny - 1, 31)]
        ref, got = [], []
        for z, yy, xx in pts:
            acc = b.copy()
            for dz in range(3):
                for dy in range(3):
                    for dx in range(3):
                        zz, y2, x2 = z + dz - 1, yy + dy - 1, xx + dx - 1
                        if 0 <= zz < nz and 0 <= y2 < ny and 0 <= x2 < nx:
                            acc += w[:, :, dz, dy, dx] @ xin[zz, y2, x2]
            ref.append(np.maximum(acc, 0.0))
            got.append(out[z, yy, xx])
        ref, got = np.array(ref), np.array(got)
        bound = 2.0 ** -7 * np.abs(ref) + 1e-3 * _rms(ref)
        worst = float(np.max(np.abs(got - ref) / bound))
        print(f"{layer}: {len(pts)} voxels x {d_ch} channels, worst |GPU - FP64| at {worst:.2f} of the bound")
        assert worst <= 1.0, layer
    net.close()
