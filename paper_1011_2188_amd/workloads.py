"""The benchmark and parity workloads, built from the seeded generators in
`inputs`.  Each returns plain numpy inputs: (phantom(s), spot list(s), track DB).

  water_pencil  64^3 water of 2 mm, one 150 MeV pencil beam (sigma 3 mm),
                1e5 histories, DB of 1e4 tracks at 150 MeV.
  slab          128^3 of 1 mm, bone slab z in [4,6) cm, lung slab z in [8,12) cm,
                25 spots on a 5x5 grid at 70 + 20 i / 3 MeV, 4e5 histories each
                (1e7 total), DB of 1e4 tracks per 5 MeV bin from 70 to 230 MeV.
  thorax        256x256x128 of 2 mm synthetic thorax, 3 coplanar fields (gantry
                0/90/180 deg) x 2000 spots on an 8x8 cm square at the right-lung
                centre, E ~ U[70,230], 1e8 histories total.
  batched       64 thorax-like plans of varying size, 1 field each, 50-3000
                spots, log-uniform 1e5-1e7 histories per plan.
"""
from __future__ import annotations

import functools
import math

import numpy as np

from . import inputs as I

DB_BINS_FULL = np.arange(70.0, 230.0 + 1e-9, 5.0)   # 33 bins


@functools.lru_cache(maxsize=4)
def water_db(n_tracks=10_000, seed=1011, energy=150.0):
    return I.make_water_track_db([energy], n_tracks, seed)


@functools.lru_cache(maxsize=4)
def multi_bin_db(n_tracks=10_000, seed=2188, bins=tuple(DB_BINS_FULL), secondaries=False):
    return I.make_water_track_db(list(bins), n_tracks, seed, secondaries=secondaries)


def water_pencil(n_histories=100_000, n_tracks=10_000, depth_vox=64):
    ph = I.water_phantom((64, 64, depth_vox), 0.2, origin=(-6.4, -6.4, 0.0))
    sp = I.spots([[0.0, 0.0, -1.0]], [[0.0, 0.0, 1.0]], [150.0], 0.3, n_histories)
    return ph, sp, water_db(n_tracks)


def slab_spots(per_spot=400_000):
    E = 70.0 + 20.0 * np.arange(25) / 3.0
    col = np.arange(25) % 5
    row = np.arange(25) // 5
    pos = np.stack([-2.0 + col, -2.0 + row, np.full(25, -1.0)], axis=1)
    dirs = np.tile([0.0, 0.0, 1.0], (25, 1))
    return I.spots(pos, dirs, E, 0.3, per_spot)


def slab(per_spot=400_000, n_tracks=10_000):
    return I.slab_phantom(128, 0.1), slab_spots(per_spot), multi_bin_db(n_tracks)


THORAX_ISO = (7.0, -1.0, 0.0)


def thorax_spots(total=100_000_000, spots_per_field=2000, seed=2188, gantries=(0.0, 90.0, 180.0)):
    rng = np.random.default_rng([int(seed), 7])
    sp = np.concatenate([I.field_spots(THORAX_ISO, g, spots_per_field, rng) for g in gantries])
    n = sp.size
    base, extra = divmod(int(total), n)
    h = np.full(n, base, np.uint64)
    h[:extra] += 1
    sp["n_histories"] = h
    return sp


def thorax(total=100_000_000, n_tracks=10_000, n=(256, 256, 128)):
    return I.thorax_phantom(n, 0.2, seed=2188), thorax_spots(total), multi_bin_db(n_tracks)


def batched_plans(n_plans=64, seed=2188, hist_scale=1.0):
    """64 independent thorax-like plans: list of (phantom, spots)."""
    rng = np.random.default_rng([int(seed), 64])
    plans = []
    for p in range(n_plans):
        nxy = int(rng.choice(np.arange(96, 257, 16)))
        nz = int(rng.choice([96, 112, 128]))
        scale = (nxy * 0.2 / 51.2, nxy * 0.2 / 51.2, nz * 0.2 / 25.6)
        ph = I.thorax_phantom((nxy, nxy, nz), 0.2, seed=int(seed) * 1000 + p, scale=scale)
        gantry = float(rng.choice([0.0, 90.0, 180.0, 270.0]))
        n_spots = int(round(math.exp(rng.uniform(math.log(50), math.log(3000)))))
        n_hist = int(round(math.exp(rng.uniform(math.log(1e5), math.log(1e7))) * hist_scale))
        iso = (7.0 * scale[0], -1.0 * scale[1], 0.0)
        sp = I.field_spots(iso, gantry, n_spots, rng, half_width_cm=4.0 * scale[0])
        base, extra = divmod(max(n_hist, n_spots), n_spots)
        h = np.full(n_spots, base, np.uint64)
        h[:extra] += 1
        sp["n_histories"] = h
        plans.append((ph, sp))
    return plans


PAPER_ISO = (7.0, -1.0, 0.0)


def paper_field(total=10_000_000, n_tracks=100_000, n=(352, 240, 72), voxel_cm=(0.1, 0.1, 0.25)):
    """The paper's test case (Section 2.5) with synthetic anatomy: a thorax of
    1 x 1 x 2.5 mm voxels (352 x 240 x 72 = 6.08e6 voxels, against the CT's
    6.06e6), a mono-energetic 121 MeV field of circular cross-section (radius
    4 cm, uniform) aimed through the right lung along -y, and a database of
    1e5 tracks at 121 MeV (the paper's database size)."""
    ph = I.thorax_phantom(n, voxel_cm, seed=2188)
    d = I.gantry_direction(0.0)
    pos = np.asarray(PAPER_ISO) - 30.0 * d
    sp = I.disk_field(pos, d, 121.0, 4.0, np.uint64(total))
    return ph, sp, water_db(n_tracks, 2188, 121.0)
