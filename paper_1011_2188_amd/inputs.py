"""Seeded synthetic inputs for track-repeating dose calculation.

This module builds the *inputs* of the method and nothing else: voxel phantoms
(int16 Hounsfield units), pencil-beam spot lists, and the synthetic water track
database that stands in for the GEANT4 water database of Section 2.2 (the
paper's database itself is not available).  It holds none of the replay
arithmetic (scaling, voxel walk, deflection, tallying, dose): both the HIP path
and the CPU oracle read what this module produces and nothing else.

Water track database (stand-in for Section 2.1/2.2):
  * mean energy loss per step from the Bragg-Kleeman range-energy relation
    R(E) = ALPHA * E**P_BK (cm, MeV);
  * Gaussian energy straggling with Bohr's variance (the variance model named
    in Section 2.1);
  * Highland multiple-scattering angle, sampled once per step (condensed
    history: the angular effect of a segment applied at its end, Section 2.1).
  Each step record is (dx [cm of water], dE [MeV], theta [rad], phi [rad]) as
  float32, contiguous per track, tracks grouped by energy bin.

Units: cm, MeV, rad, g/cm^3.  Arrays are x-fastest: hu[z, y, x].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# --- physics constants of the synthetic water database ---------------------
ALPHA = 0.0022          # Bragg-Kleeman prefactor, cm / MeV**P_BK
P_BK = 1.77             # Bragg-Kleeman exponent
K_BOHR = 0.1569         # 4*pi*N_A*r_e^2*(m_e c^2)^2, MeV^2 cm^2 / g
Z_OVER_A_WATER = 0.5551
X0_WATER = 36.08        # radiation length of water, cm
M_PROTON = 938.272      # MeV
STEP_CM = 0.1           # database step length (about the 1 mm depth segmentation of Section 2.2)

# numpy structured dtype matching the C struct fdc_spot (40 bytes)
SPOT_DTYPE = np.dtype([("pos_cm", "<f4", (3,)), ("dir", "<f4", (3,)),
                       ("energy_MeV", "<f4"), ("sigma_cm", "<f4"),
                       ("n_histories", "<u8")])
assert SPOT_DTYPE.itemsize == 40

# one listed incident proton (the C struct fdc_particle, 32 bytes)
PARTICLE_DTYPE = np.dtype([("pos_cm", "<f4", (3,)), ("dir", "<f4", (3,)), ("energy_MeV", "<f4"),
                           ("reserved", "<f4")])
assert PARTICLE_DTYPE.itemsize == 32
PHASE_SPACE_MAGIC = b"FDCPHSP1"

# Default HU -> (density, relative stopping power, relative scattering power)
# table: synthetic constants (not clinical data), piecewise linear.
HU_TABLE_DEFAULT = {
    "hu":   np.array([-1000.0, 0.0, 1000.0, 3071.0]),
    "rho":  np.array([0.0012, 1.0, 1.6, 2.84]),
    "rsp":  np.array([0.0011, 1.0, 1.5, 2.64]),
    "rscp": np.array([0.0012, 1.0, 2.16, 3.834]),
    "vacuum_below_hu": -990.0,
}


@dataclasses.dataclass
class Phantom:
    hu: np.ndarray            # int16 [nz, ny, nx]
    voxel_cm: np.ndarray      # float32 [3] (x, y, z)
    origin_cm: np.ndarray     # float32 [3] corner of voxel (0,0,0)

    @property
    def shape_xyz(self):
        nz, ny, nx = self.hu.shape
        return nx, ny, nz


@dataclasses.dataclass
class Secondaries:
    """Secondary trajectories of a track database (Section 2.2: each particle
    trajectory of a stored history is broken into steps): trajectory j of
    track t (sec_first[t] <= j < sec_first[t+1]) starts at the end of the
    track's primary step `branch[j]` (counted from the track's first step),
    leaving at polar angle emit[j, 0] and azimuth emit[j, 1] from the
    primary's direction there, and replays its own steps
    steps[off[j] : off[j+1]] = (dx, dE, theta, phi)."""
    sec_first: np.ndarray     # uint32 [n_tracks + 1]
    off: np.ndarray           # uint64 [n_sec + 1]
    steps: np.ndarray         # float32 [n_sec_steps, 4]
    branch: np.ndarray        # uint32 [n_sec]
    emit: np.ndarray          # float32 [n_sec, 2]

    @property
    def n(self):
        return int(self.branch.size)


@dataclasses.dataclass
class TrackDB:
    steps: np.ndarray         # float32 [n_steps, 4] = (dx, dE, theta, phi)
    track_off: np.ndarray     # uint64 [n_tracks + 1]
    bin_E: np.ndarray         # float32 [n_bins]
    bin_first: np.ndarray     # uint32 [n_bins + 1]
    sec: Secondaries = None   # secondary trajectories, if any

    @property
    def n_tracks(self):
        return int(self.track_off.size - 1)

    @property
    def n_bins(self):
        return int(self.bin_E.size)


# --------------------------------------------------------------------------
# water track database
# --------------------------------------------------------------------------
def _beta2(E):
    g = (E + M_PROTON) / M_PROTON
    return 1.0 - 1.0 / (g * g)


def highland_theta0(E, x_cm):
    """Highland width (rad) for a proton of kinetic energy E (MeV) over x_cm of water."""
    b2 = _beta2(E)
    bcp = b2 * (E + M_PROTON)                 # beta * c * p = beta^2 * total energy
    arg = np.maximum(x_cm, 1e-30) / (X0_WATER * b2)
    th = 13.6 / bcp * np.sqrt(x_cm / X0_WATER) * (1.0 + 0.038 * np.log(arg))
    return np.maximum(th, 0.0)


def bohr_sigma(E, x_cm):
    """Bohr straggling width (MeV) in water over x_cm at kinetic energy E."""
    b2 = _beta2(E)
    return np.sqrt(K_BOHR * Z_OVER_A_WATER * x_cm * (1.0 - 0.5 * b2) / (1.0 - b2))


def csda_range(E):
    return ALPHA * np.power(E, P_BK)


def energy_at_range(R):
    return np.power(np.maximum(R, 0.0) / ALPHA, 1.0 / P_BK)


def _gen_bin(Eb, n_tracks, rng, step_cm, nuc=None):
    """All tracks of one energy bin (Eb a scalar, or one start energy per
    track); returns (records [n_steps,4] f32, steps per track).  With nuc =
    (rng, rate per cm, max per track, list), a regular step of a track with
    more than NUC_MIN_MEV left ends with a nuclear interaction with probability
    rate * step length: a secondary proton takes a fraction U(0.2, 0.5) of the
    energy left after the step, leaving at polar angle U(0.05, 0.4) rad and a
    uniform azimuth, and the primary goes on with the rest; each interaction
    is appended to the list as (track, step, energy, theta, phi)."""
    E = np.broadcast_to(np.asarray(Eb, np.float64), (n_tracks,)).copy()
    alive = np.ones(n_tracks, bool)
    n_sec = np.zeros(n_tracks, np.int64)
    cols = []     # per step: (n_tracks, 4) float32, valid where mask
    masks = []
    while alive.any():
        z = rng.standard_normal((n_tracks, 3))
        R = csda_range(E)
        final = alive & (R <= step_cm)
        normal = alive & ~final
        rec = np.zeros((n_tracks, 4))
        # regular step of length step_cm
        Rn = np.where(normal, R, 2.0 * step_cm)
        E_mid = energy_at_range(Rn - 0.5 * step_cm)
        dE_mean = E - energy_at_range(Rn - step_cm)
        sig = bohr_sigma(E_mid, step_cm)
        dE = np.clip(dE_mean + sig * z[:, 0], 0.0, E)
        th0 = highland_theta0(E_mid, step_cm)
        # final step: the residual range, all residual energy, angle at E/2
        Ef = np.where(final, E, 1.0)
        th0f = highland_theta0(0.5 * Ef, np.where(final, R, step_cm))
        th0 = np.where(final, th0f, th0)
        dx = np.where(final, R, step_cm)
        dE = np.where(final, E, dE)
        tx = th0 * z[:, 1]
        ty = th0 * z[:, 2]
        rec[:, 0] = dx
        rec[:, 1] = dE
        rec[:, 2] = np.hypot(tx, ty)
        rec[:, 3] = np.arctan2(ty, tx)
        cols.append(rec.astype(np.float32))
        masks.append(alive.copy())
        E = np.where(alive, E - dE, E)
        if nuc is not None:
            nrng, rate, max_sec, out = nuc
            u = nrng.random((n_tracks, 4))
            hit = normal & (E > NUC_MIN_MEV) & (n_sec < max_sec) & (u[:, 0] < rate * step_cm)
            for t in np.flatnonzero(hit):
                Es = float(np.float32(E[t] * (0.2 + 0.3 * u[t, 1])))
                out.append((int(t), len(cols) - 1, Es, 0.05 + 0.35 * u[t, 2], 2.0 * math.pi * u[t, 3]))
                E[t] -= Es
                n_sec[t] += 1
        alive = normal & (E > 0.0)
    recs = np.stack(cols, axis=1)            # [n_tracks, n_steps_max, 4]
    mask = np.stack(masks, axis=1)           # [n_tracks, n_steps_max]
    return recs[mask], mask.sum(axis=1)


NUC_PER_CM = 0.012        # non-elastic nuclear interactions of protons in water, per cm (about 1%/cm)
NUC_MIN_MEV = 20.0        # no interaction below this energy left
NUC_MAX_PER_TRACK = 2


def make_water_track_db(bin_energies_MeV, n_tracks_per_bin, seed, step_cm=STEP_CM, secondaries=False,
                        nuc_per_cm=NUC_PER_CM):
    """Synthetic water track database: `n_tracks_per_bin` tracks at each bin energy.

    Deterministic in (seed, bin index).  Bins must be strictly increasing.
    With secondaries, nuclear interactions along the primary (see _gen_bin)
    each start a secondary proton trajectory generated the same way (from its
    own energy, no interactions of its own); interactions and secondaries draw
    from streams of their own, so a track without an interaction is the same
    as in the database without secondaries."""
    bins = np.asarray(bin_energies_MeV, np.float32)
    if bins.ndim != 1 or bins.size == 0 or np.any(np.diff(bins) <= 0):
        raise ValueError("bin energies must be a non-empty increasing list")
    recs, counts = [], []
    sec_recs, sec_counts, sec_branch, sec_emit, sec_per_track = [], [], [], [], []
    for b, Eb in enumerate(bins):
        rng = np.random.default_rng([int(seed), b])
        inter = []
        nuc = (np.random.default_rng([int(seed), b, 7]), nuc_per_cm, NUC_MAX_PER_TRACK, inter) if secondaries else None
        r, c = _gen_bin(float(Eb), int(n_tracks_per_bin), rng, step_cm, nuc)
        recs.append(r)
        counts.append(c)
        if secondaries:
            inter.sort(key=lambda x: (x[0], x[1]))
            per = np.zeros(int(n_tracks_per_bin), np.int64)
            for t, *_ in inter:
                per[t] += 1
            sec_per_track.append(per)
            if inter:
                srng = np.random.default_rng([int(seed), b, 8])
                sr, sc = _gen_bin(np.array([x[2] for x in inter]), len(inter), srng, step_cm)
                sec_recs.append(sr)
                sec_counts.append(sc)
                sec_branch.append(np.array([x[1] for x in inter], np.uint32))
                sec_emit.append(np.array([[x[3], x[4]] for x in inter], np.float32))
    counts = np.concatenate(counts).astype(np.uint64)
    track_off = np.zeros(counts.size + 1, np.uint64)
    np.cumsum(counts, out=track_off[1:])
    bin_first = (np.arange(bins.size + 1, dtype=np.uint64) * int(n_tracks_per_bin)).astype(np.uint32)
    sec = None
    if secondaries:
        per = np.concatenate(sec_per_track)
        sec_first = np.zeros(per.size + 1, np.uint32)
        np.cumsum(per, out=sec_first[1:])
        sc = np.concatenate(sec_counts).astype(np.uint64) if sec_counts else np.zeros(0, np.uint64)
        off = np.zeros(sc.size + 1, np.uint64)
        np.cumsum(sc, out=off[1:])
        sec = Secondaries(sec_first, off,
                          np.ascontiguousarray(np.concatenate(sec_recs, axis=0) if sec_recs else np.zeros((0, 4)),
                                               np.float32),
                          np.concatenate(sec_branch) if sec_branch else np.zeros(0, np.uint32),
                          np.concatenate(sec_emit) if sec_emit else np.zeros((0, 2), np.float32))
    return TrackDB(np.ascontiguousarray(np.concatenate(recs, axis=0), np.float32),
                   track_off, bins, bin_first, sec)


DB_FILE_MAGIC = b"FDCTRKDB"
_DB_HEADER = np.dtype([("magic", "S8"), ("version", "<u4"), ("n_bins", "<u4"), ("n_tracks", "<u4"),
                       ("n_sec", "<u4"), ("n_steps", "<u8"), ("db_seed", "<u8"), ("physics", "<f8", (8,))])
assert _DB_HEADER.itemsize == 104


def write_track_db_file(path, db, db_seed=0):
    """Write a track database in the library's file layout: a 104-byte
    little-endian header, then bin_E, bin_first, track_off and the step
    records, packed.  A database with secondary trajectories is version 2:
    the header's n_sec, and after the primary steps the secondaries' step
    count (u64), sec_first, sec_off, branch, emit and their steps."""
    h = np.zeros(1, _DB_HEADER)
    h["magic"] = DB_FILE_MAGIC
    h["version"] = 1 if db.sec is None else 2
    h["n_bins"] = db.n_bins
    h["n_tracks"] = db.n_tracks
    h["n_sec"] = 0 if db.sec is None else db.sec.n
    h["n_steps"] = db.steps.shape[0]
    h["db_seed"] = int(db_seed)
    h["physics"] = [ALPHA, P_BK, K_BOHR, Z_OVER_A_WATER, X0_WATER, M_PROTON, STEP_CM, 0.0]
    with open(path, "wb") as f:
        f.write(h.tobytes())
        f.write(np.ascontiguousarray(db.bin_E, "<f4").tobytes())
        f.write(np.ascontiguousarray(db.bin_first, "<u4").tobytes())
        f.write(np.ascontiguousarray(db.track_off, "<u8").tobytes())
        f.write(np.ascontiguousarray(db.steps, "<f4").tobytes())
        if db.sec is not None:
            s = db.sec
            st = np.ascontiguousarray(s.steps, "<f4").reshape(-1, 4)
            f.write(np.array([st.shape[0]], "<u8").tobytes())
            f.write(np.ascontiguousarray(s.sec_first, "<u4").tobytes())
            f.write(np.ascontiguousarray(s.off, "<u8").tobytes())
            f.write(np.ascontiguousarray(s.branch, "<u4").tobytes())
            f.write(np.ascontiguousarray(s.emit, "<f4").tobytes())
            f.write(st.tobytes())


def read_track_db_file(path):
    """Read a file written by write_track_db_file back into a TrackDB."""
    raw = np.fromfile(path, np.uint8)
    h = raw[:_DB_HEADER.itemsize].view(_DB_HEADER)[0]
    if bytes(h["magic"]) != DB_FILE_MAGIC or int(h["version"]) not in (1, 2):
        raise ValueError("not a track database file")
    nb, nt, ns = int(h["n_bins"]), int(h["n_tracks"]), int(h["n_steps"])
    o = _DB_HEADER.itemsize

    def take(dt, n):
        nonlocal o
        size = np.dtype(dt).itemsize * n
        a = raw[o:o + size].view(dt).copy()
        o += size
        return a
    parts = [take(dt, n) for dt, n in (("<f4", nb), ("<u4", nb + 1), ("<u8", nt + 1), ("<f4", 4 * ns))]
    sec = None
    if int(h["version"]) == 2:
        n_sec = int(h["n_sec"])
        nss = int(take("<u8", 1)[0])
        first, off, branch = take("<u4", nt + 1), take("<u8", n_sec + 1), take("<u4", n_sec)
        emit = take("<f4", 2 * n_sec).reshape(n_sec, 2)
        sec = Secondaries(first, off, take("<f4", 4 * nss).reshape(nss, 4), branch, emit)
    if o != raw.size:
        raise ValueError("track database file size does not match its header")
    return TrackDB(parts[3].reshape(ns, 4), parts[2], parts[0], parts[1], sec)


def write_phase_space_file(path, particles):
    """A phase-space file: 32-byte header (magic, version 1, record size 32,
    count, 0) then the fdc_particle records."""
    q = np.ascontiguousarray(particles, PARTICLE_DTYPE)
    h = np.zeros(1, np.dtype([("magic", "S8"), ("version", "<u4"), ("rec", "<u4"), ("n", "<u8"), ("res", "<u8")]))
    h["magic"] = PHASE_SPACE_MAGIC
    h["version"] = 1
    h["rec"] = PARTICLE_DTYPE.itemsize
    h["n"] = q.size
    with open(path, "wb") as f:
        f.write(h.tobytes())
        f.write(q.tobytes())


def read_phase_space_file(path):
    raw = np.fromfile(path, np.uint8)
    if raw[:8].tobytes() != PHASE_SPACE_MAGIC:
        raise ValueError("not a phase-space file")
    n = int(raw[16:24].view("<u8")[0])
    q = raw[32:].view(PARTICLE_DTYPE)
    if q.size != n:
        raise ValueError("phase-space file size does not match its header")
    return q.copy()


def synthetic_phase_space(n, seed, e_mean=121.0, e_sigma=0.8, tail_fraction=0.05, tail_min=100.0,
                          radius_cm=4.0, source_cm=(7.0, -31.0, 0.0), direction=(0.0, 1.0, 0.0),
                          sad_cm=200.0, divergence_rad=0.002):
    """A stand-in for a phase-space file scored at the exit of a beam line: a
    field of circular cross-section (start points uniform over a disk of
    radius_cm in the plane through source_cm perpendicular to `direction`),
    directions diverging from a virtual source sad_cm upstream plus a small
    Gaussian angular spread, energies Gaussian around e_mean with a
    low-energy tail (protons that lost energy in the beam line), uniform from
    tail_min to e_mean.  Deterministic in seed."""
    rng = np.random.default_rng([int(seed), 31])
    d = np.asarray(direction, np.float64)
    d /= np.linalg.norm(d)
    e1, e2 = field_frame(d)
    r = radius_cm * np.sqrt(rng.random(n))
    a = 2.0 * np.pi * rng.random(n)
    off = (r * np.cos(a))[:, None] * e1 + (r * np.sin(a))[:, None] * e2
    pos = np.asarray(source_cm, np.float64) + off
    dirs = d * sad_cm + off + divergence_rad * sad_cm * (rng.standard_normal((n, 1)) * e1
                                                          + rng.standard_normal((n, 1)) * e2)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    E = rng.normal(e_mean, e_sigma, n)
    tail = rng.random(n) < tail_fraction
    E[tail] = rng.uniform(tail_min, e_mean, int(tail.sum()))
    q = np.zeros(n, PARTICLE_DTYPE)
    q["pos_cm"] = pos
    q["dir"] = dirs
    q["energy_MeV"] = E
    return q


# --------------------------------------------------------------------------
# phantoms
# --------------------------------------------------------------------------
def water_phantom(n=(64, 64, 64), voxel_cm=0.2, origin=None):
    nx, ny, nz = n
    hu = np.zeros((nz, ny, nx), np.int16)
    vox = np.full(3, voxel_cm, np.float32)
    if origin is None:
        origin = (-0.5 * nx * voxel_cm, -0.5 * ny * voxel_cm, 0.0)
    return Phantom(hu, vox, np.asarray(origin, np.float32))


def slab_phantom(n=128, voxel_cm=0.1):
    """Water with a bone slab (HU +1000) at z in [4,6) cm and a lung slab
    (HU -800) at z in [8,12) cm, slabs perpendicular to the beam (+z)."""
    ph = water_phantom((n, n, n), voxel_cm)
    zc = (np.arange(n) + 0.5) * voxel_cm
    ph.hu[(zc >= 4.0) & (zc < 6.0)] = 1000
    ph.hu[(zc >= 8.0) & (zc < 12.0)] = -800
    return ph


def thorax_phantom(n=(256, 256, 128), voxel_cm=0.2, seed=2188, scale=(1.0, 1.0, 1.0),
                   body_axes=(17.0, 11.0), lung_centre_x=7.0, lung_centre_y=-1.0,
                   lung_axes=(5.0, 7.0, 10.0), spine_centre_y=-8.0, spine_radius=1.5):
    """Synthetic thorax: air (-1000) around an elliptic body cylinder along z
    (HU ~ N(40,20)), two lung ellipsoids (HU ~ N(-800,50)) and a spine cylinder
    (HU ~ N(1000,100)); i.i.d. HU per voxel, rounded to int16.  Centred on 0.
    voxel_cm: one size, or (x, y, z) sizes for anisotropic voxels."""
    nx, ny, nz = n
    sx, sy, sz = scale
    vx, vy, vz = (voxel_cm,) * 3 if np.ndim(voxel_cm) == 0 else tuple(float(v) for v in voxel_cm)
    rng = np.random.default_rng(int(seed))
    x = (np.arange(nx) + 0.5) * vx - 0.5 * nx * vx
    y = (np.arange(ny) + 0.5) * vy - 0.5 * ny * vy
    z = (np.arange(nz) + 0.5) * vz - 0.5 * nz * vz
    X, Y = x[None, :], y[:, None]              # cylinders along z: masks on the (y, x) plane
    shape = (nz, ny, nx)
    hu = np.full(shape, -1000.0)
    body = np.broadcast_to((X / (body_axes[0] * sx)) ** 2 + (Y / (body_axes[1] * sy)) ** 2 <= 1.0, shape)
    hu[body] = rng.normal(40.0, 20.0, int(body.sum()))
    lungs = np.zeros(shape, bool)
    tz = ((z / (lung_axes[2] * sz)) ** 2)[:, None, None]
    for cx in (-lung_centre_x, lung_centre_x):
        txy = (((X - cx * sx) / (lung_axes[0] * sx)) ** 2 + ((Y - lung_centre_y * sy) / (lung_axes[1] * sy)) ** 2)
        lungs |= (txy[None] + tz) <= 1.0
    hu[lungs] = rng.normal(-800.0, 50.0, int(lungs.sum()))
    spine = np.broadcast_to(X ** 2 + (Y - spine_centre_y * sy) ** 2 <= (spine_radius * min(sx, sy)) ** 2, shape)
    hu[spine] = rng.normal(1000.0, 100.0, int(spine.sum()))
    hu = np.clip(np.rint(hu), -32768, 32767).astype(np.int16)
    vox = np.array([vx, vy, vz], np.float32)
    origin = np.array([-0.5 * nx * vx, -0.5 * ny * vy, -0.5 * nz * vz], np.float32)
    return Phantom(hu, vox, origin)


# --------------------------------------------------------------------------
# beam spots
# --------------------------------------------------------------------------
def spots(pos, dirs, energies, sigmas, n_histories):
    k = len(energies)
    s = np.zeros(k, SPOT_DTYPE)
    s["pos_cm"] = np.asarray(pos, np.float32).reshape(k, 3)
    s["dir"] = np.asarray(dirs, np.float32).reshape(k, 3)
    s["energy_MeV"] = np.asarray(energies, np.float32)
    s["sigma_cm"] = np.broadcast_to(np.asarray(sigmas, np.float32), (k,))
    s["n_histories"] = np.broadcast_to(np.asarray(n_histories, np.uint64), (k,))
    return s


def disk_field(pos, direction, energy_MeV, radius_cm, n_histories):
    """One mono-energetic field of circular cross-section: start points uniform
    over a disk of radius_cm around pos, perpendicular to direction (Section
    2.5's test field); encoded as a spot with sigma = -radius."""
    return spots([pos], [direction], [energy_MeV], -float(radius_cm), n_histories)


def beam_device(origin_cm, direction, pitch_cm, pixels, rsp=1.0, rscp=1.0):
    """A beam-line device upstream of the phantom: an aperture and a range
    compensator on one pixel grid in the plane through origin_cm (the centre
    of its upstream face) perpendicular to direction (along the beam).
    pixels[j][i] (i along e1, fastest; j along e2; (e1, e2) the lateral axes of
    direction as for a spot, the grid centred on origin_cm, pitch_cm per
    axis): < 0 closed, else the compensator thickness in cm along direction
    (0: open, no material).  rsp, rscp: the compensator material's relative
    stopping and scattering powers."""
    pix = np.ascontiguousarray(np.asarray(pixels, np.float32))
    assert pix.ndim == 2
    return dict(origin_cm=np.asarray(origin_cm, np.float32).reshape(3), dir=np.asarray(direction, np.float32).reshape(3),
                pitch_cm=np.asarray(pitch_cm, np.float32).reshape(2), n=np.array([pix.shape[1], pix.shape[0]], np.uint32),
                rsp=float(rsp), rscp=float(rscp), pixels=pix)


def aperture_compensator(origin_cm, direction, radius_cm, ramp_cm=(0.0, 0.0), pitch_cm=0.1, half_width_cm=None,
                         rsp=1.19, rscp=1.35):
    """A circular aperture of radius radius_cm with a wedge-shaped compensator
    behind it (thickness ramp_cm[0] at e1 = -radius rising linearly to
    ramp_cm[1] at e1 = +radius), on a square grid of pitch pitch_cm; the
    default material resembles PMMA (RSP 1.19)."""
    hw = radius_cm * 1.25 if half_width_cm is None else half_width_cm
    n = int(math.ceil(2 * hw / pitch_cm))
    c = (np.arange(n) + 0.5 - n / 2) * pitch_cm
    a, b = np.meshgrid(c, c)                                    # a along e1 (columns), b along e2 (rows)
    t = ramp_cm[0] + (ramp_cm[1] - ramp_cm[0]) * (a + radius_cm) / (2 * radius_cm)
    pix = np.where(a * a + b * b <= radius_cm * radius_cm, np.maximum(t, 0.0), -1.0)
    return beam_device(origin_cm, direction, (pitch_cm, pitch_cm), pix, rsp, rscp)


def gantry_direction(gantry_deg):
    """Beam direction in the x-y plane for a coplanar gantry angle:
    0 deg points along -y, 90 deg along -x, 180 deg along +y."""
    g = math.radians(gantry_deg)
    return np.array([-math.sin(g), -math.cos(g), 0.0])


def field_frame(d):
    """Lateral unit vectors (e1, e2) of a beam with unit direction d, such that
    (e1, e2, d) is right-handed and d = +z gives (x, y)."""
    d = np.asarray(d, np.float64)
    a = np.array([1.0, 0.0, 0.0]) if abs(d[2]) >= 0.9 else np.array([0.0, 0.0, 1.0])
    e2 = np.cross(d, a)
    e2 /= np.linalg.norm(e2)
    e1 = np.cross(e2, d)
    return e1, e2


def field_spots(iso, gantry_deg, n_spots, rng, half_width_cm=4.0, e_range=(70.0, 230.0),
                sigma_cm=0.3, source_distance_cm=30.0, histories=None):
    d = gantry_direction(gantry_deg)
    e1, e2 = field_frame(d)
    a = rng.uniform(-half_width_cm, half_width_cm, n_spots)
    b = rng.uniform(-half_width_cm, half_width_cm, n_spots)
    E = rng.uniform(e_range[0], e_range[1], n_spots)
    pos = (np.asarray(iso, np.float64)[None, :] - source_distance_cm * d[None, :]
           + a[:, None] * e1[None, :] + b[:, None] * e2[None, :])
    dirs = np.broadcast_to(d, (n_spots, 3))
    n = np.zeros(n_spots, np.uint64) if histories is None else histories
    return spots(pos, dirs, E, sigma_cm, n)
