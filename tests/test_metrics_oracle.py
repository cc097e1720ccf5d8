"""Pins of the oracle's dose metrics: the gamma index against brute force,
constant-field and linear-ramp closed forms; Eq. (1) and the mean
uncertainty are pinned in test_oracle_pins.py."""
import itertools
import math

import numpy as np

from oracle import oracle as O
from paper_1011_2188_amd import inputs as I


def _field(n=(12, 10, 8), seed=0):
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = np.exp(-((x - nx / 2) ** 2 + (y - ny / 2) ** 2) / 8.0) * (1 + 0.05 * z) + 0.01 * rng.random((nz, ny, nx))
    return d


def test_gamma_identical_is_zero():
    ph = I.water_phantom((12, 10, 8), 0.2)
    d = _field()
    g, rate = O.gamma_index(d, d, ph)
    assert rate == 1.0 and np.all(g[g >= 0] == 0.0)


def test_gamma_constant_field_scaled():
    """Every point of a constant field differs by the same amount: gamma =
    (scale - 1) / dose_frac exactly, whatever the distance."""
    ph = I.water_phantom((6, 6, 6), 0.2)
    d = np.full((6, 6, 6), 2.0)
    g, rate = O.gamma_index(d, 1.03 * d, ph, dose_frac=0.02)
    assert np.allclose(g, 1.5, rtol=1e-12) and rate == 0.0
    g, rate = O.gamma_index(d, 1.019 * d, ph, dose_frac=0.02)
    assert np.allclose(g, 0.95, rtol=1e-12) and rate == 1.0


def test_gamma_linear_ramp_bounds():
    """Ramp D = k x shifted by s: the continuous minimum over the distance t of
    t^2/dta^2 + (k (t - s))^2/dd^2 is s^2 / (dta^2 + dd^2 / k^2); the discrete
    half-voxel search can only be above it, and by a bounded amount."""
    vox = 0.1
    ph = I.water_phantom((40, 3, 3), vox)
    x = (np.arange(40) + 0.5) * vox
    k = 2.0
    ref = np.broadcast_to(k * x, (3, 3, 40)).copy() + 1.0
    s = 0.15
    ev = np.broadcast_to(k * (x - s), (3, 3, 40)).copy() + 1.0
    g, _ = O.gamma_index(ref, ev, ph, dose_frac=0.02, dta_cm=0.2, cutoff_frac=0.0, search_cm=0.6)
    dd = 0.02 * ref.max()
    cont = math.sqrt(s ** 2 / (0.2 ** 2 + dd ** 2 / k ** 2))
    inner = g[1, 1, 10:30]
    assert np.all(inner >= cont - 1e-12)
    # the grid step is 0.05 cm: the discrete minimum is within half a step of the optimum t
    assert np.all(inner <= math.sqrt(cont ** 2 + (0.025 / 0.2) ** 2 + (k * 0.025 / dd) ** 2) + 1e-12)


def test_gamma_brute_force_tiny():
    """Pure-Python brute force on a 5x4x3 grid with anisotropic voxels."""
    rng = np.random.default_rng(4)
    ph = I.Phantom(np.zeros((3, 4, 5), np.int16), np.array([0.1, 0.15, 0.25], np.float32),
                   np.zeros(3, np.float32))
    ref = rng.random((3, 4, 5)) + 0.5
    ev = ref * (1 + 0.05 * rng.standard_normal((3, 4, 5)))
    g, _ = O.gamma_index(ref, ev, ph, dose_frac=0.03, dta_cm=0.3, cutoff_frac=0.2, search_cm=0.5)
    vx, vy, vz = (float(v) for v in ph.voxel_cm)      # as stored (float32)
    pos = lambda i, j, k: np.array([i * vx, j * vy, k * vz])

    def e_at(px, py, pz):      # half-voxel coordinates -> trilinear evaluated dose
        val = 0.0
        for cx, cy, cz in itertools.product((0, 1), repeat=3):
            ix = px // 2 + (cx if px % 2 else 0)
            iy = py // 2 + (cy if py % 2 else 0)
            iz = pz // 2 + (cz if pz % 2 else 0)
            val += ev[iz, iy, ix] / 8.0
        return val
    dmax = ref.max()
    for k, j, i in itertools.product(range(3), range(4), range(5)):
        if ref[k, j, i] < 0.2 * dmax:
            assert g[k, j, i] == -1.0
            continue
        best = math.inf
        for pz, py, px in itertools.product(range(5), range(7), range(9)):
            r = np.linalg.norm(pos(px / 2, py / 2, pz / 2) - pos(i, j, k))
            if r > 0.5 + 1e-12:
                continue
            best = min(best, r ** 2 / 0.3 ** 2 + (e_at(px, py, pz) - ref[k, j, i]) ** 2 / (0.03 * dmax) ** 2)
        assert math.isclose(g[k, j, i], math.sqrt(best), rel_tol=1e-12, abs_tol=1e-12)


def test_gamma_rigid_shift_one_dta():
    """A field shifted by exactly one DTA (one voxel here) passes everywhere the
    shifted partner exists."""
    ph = I.water_phantom((16, 8, 8), 0.2)
    d = _field((16, 8, 8))
    ev = np.zeros_like(d)
    ev[:, :, 1:] = d[:, :, :-1]
    g, _ = O.gamma_index(d, ev, ph, dose_frac=0.02, dta_cm=float(ph.voxel_cm[0]), cutoff_frac=0.0)
    assert np.all(g[:, :, :-1][g[:, :, :-1] >= 0] <= 1.0 + 1e-12)
