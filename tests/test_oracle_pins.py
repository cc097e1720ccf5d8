"""Pins of the CPU oracle against facts fixed outside the oracle itself:
published generator values, closed forms, exact one-dimensional integrals,
invariants and symmetries.  CPU only."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_1011_2188_amd import inputs as I
from paper_1011_2188_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
FP = 2.0 ** 24


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


# ---------------------------------------------------------------- Philox ----
def _kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    for ctr, key, out in _kat():
        assert O.philox(ctr, key).tolist() == out


def test_philox_matches_torch_engine(tmp_path):
    """PyTorch ships an independent header-only Philox4x32-10; compare 2000 counters."""
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if shutil.which("g++") is None or not os.path.exists(os.path.join(inc, "ATen/core/PhiloxRNGEngine.h")):
        pytest.skip("no g++ or torch headers")
    exe = str(tmp_path / "ph")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", inc, os.path.join(HERE, "philox_torch_ref.cpp"),
                    "-o", exe], check=True)
    rng = np.random.default_rng(5)
    cases = rng.integers(0, 2 ** 32, size=(2000, 6), dtype=np.uint64)
    cases[:10, 1:4] = 0          # small counters as used for histories
    txt = "\n".join(" ".join(str(int(x)) for x in row) for row in cases)
    out = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True).stdout.split("\n")
    for row, line in zip(cases, out):
        ref = [int(x) for x in line.split()]
        assert O.philox(row[:4], row[4:6]).tolist() == ref


def test_uniform_open_interval():
    assert O.uniform(0) == 2.0 ** -25
    assert O.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -25
    assert O.uniform(0x80000000) == 0.5 + 2.0 ** -25


# -------------------------------------------------------------- rotation ----
def test_rotation_invariants():
    rng = np.random.default_rng(1)
    for _ in range(300):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        th = rng.uniform(0, 0.5)
        ph = rng.uniform(-math.pi, math.pi)
        r = O.rotate(d, th, ph)
        assert abs(np.linalg.norm(r) - 1) < 1e-14
        assert abs(np.dot(r, d) - math.cos(th)) < 1e-12      # polar angle is theta
        # equivariance under rotations about z (azimuth reference = global frame)
        a = rng.uniform(0, 2 * math.pi)
        Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
        assert np.allclose(Rz @ r, O.rotate(Rz @ d, th, ph), atol=1e-13)


def test_rotation_conventions():
    th, ph = 0.3, 0.7
    # along +z the azimuth is measured from +x toward +y
    r = O.rotate([0, 0, 1.0], th, ph)
    assert np.allclose(r, [math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    r = O.rotate([0, 0, -1.0], th, ph)
    assert np.allclose(r, [math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), -math.cos(th)])
    # along +x with phi = 0 the deflection tilts toward -z; phi = pi/2 toward +y
    assert np.allclose(O.rotate([1.0, 0, 0], th, 0.0), [math.cos(th), 0, -math.sin(th)])
    assert np.allclose(O.rotate([1.0, 0, 0], th, math.pi / 2), [math.cos(th), math.sin(th), 0], atol=1e-15)


# --------------------------------------------------------------- material ----
def test_material_table():
    hu = np.array([-1024, -1000, -991, -990, -800, 0, 500, 1000, 3071, 4000], np.int16)
    rho, rsp, g, vac = O.material(hu)
    assert vac.tolist() == [True, True, True, False, False, False, False, False, False, False]
    assert rsp[5] == 1.0 and g[5] == 1.0 and rho[5] == 1.0          # water is (1,1,1)
    assert math.isclose(rsp[4], 0.0011 + 0.9989 * 0.2, rel_tol=1e-15)
    assert math.isclose(rsp[7], 1.5) and math.isclose(g[7], 2.16 / 1.5)
    assert rsp[9] == rsp[8] == 2.64                                 # clamped at HU 3071
    assert math.isclose(rho[6], 1.3)


# ------------------------------------------------------------ DB (inputs) ----
def test_water_db_physics():
    """The synthetic water database: Bragg-Kleeman mean range, exact energy sum,
    Bohr-Gaussian straggling and Highland angles."""
    db = I.make_water_track_db([70.0, 150.0], 2000, seed=3)
    for b, Eb in enumerate(db.bin_E):
        ts = range(int(db.bin_first[b]), int(db.bin_first[b + 1]))
        L = np.array([db.steps[db.track_off[t]:db.track_off[t + 1], 0].sum(dtype=np.float64) for t in ts])
        S = np.array([db.steps[db.track_off[t]:db.track_off[t + 1], 1].sum(dtype=np.float64) for t in ts])
        assert abs(L.mean() / (0.0022 * float(Eb) ** 1.77) - 1) < 5e-3
        assert np.max(np.abs(S - Eb)) < 1e-4 * Eb
    # first step at 150 MeV: dE ~ N(mean, bohr sigma), theta ~ Rayleigh(theta0)
    t0 = db.track_off[db.bin_first[1]:db.bin_first[2]]
    first = db.steps[t0.astype(np.int64)]
    Emid = I.energy_at_range(I.csda_range(150.0) - 0.05)
    mean = 150.0 - I.energy_at_range(I.csda_range(150.0) - 0.1)
    sig = I.bohr_sigma(Emid, 0.1)
    assert stats.kstest((first[:, 1] - mean) / sig, "norm").pvalue > 1e-3
    th0 = I.highland_theta0(Emid, 0.1)
    assert abs(th0 - 2.12e-3) < 0.01e-3 and abs(sig - 0.101) < 0.001
    assert stats.kstest(first[:, 2] / th0, "rayleigh").pvalue > 1e-3


# ------------------------------------------------------------ replay pins ----
def _straight(db):
    """Same database with all deflection angles set to zero."""
    s = db.steps.copy()
    s[:, 2] = 0.0
    return I.TrackDB(s, db.track_off, db.bin_E, db.bin_first)


def _track_profile(db, t, skip_fp):
    """Exact 1-D deposit of one straight track entering water at depth 0:
    returns (step start WEL, step WEL, step energy fp) after the energy skip."""
    rec = db.steps[db.track_off[t]:db.track_off[t + 1]].astype(np.float64)
    e = np.rint(rec[:, 1] * FP).astype(np.int64)
    cum = np.concatenate([[0], np.cumsum(e)])
    k0 = int(np.argmax(cum[1:] > skip_fp))
    e_first = cum[k0 + 1] - skip_fp
    f = e_first / e[k0]
    dx = rec[k0:, 0].copy()
    dx[0] *= f
    ee = e[k0:].copy()
    ee[0] = e_first
    z0 = np.concatenate([[0.0], np.cumsum(dx)[:-1]])
    return z0, dx, ee


def _slab_energy(z0, dx, ee, W):
    """Energy per slab whose WEL boundaries are W (len n+1), uniform in WEL per step."""
    out = np.zeros(len(W) - 1)
    for a, w, e in zip(z0, dx, ee):
        lo = np.clip(W[:-1], a, a + w)
        hi = np.clip(W[1:], a, a + w)
        out += e * (hi - lo) / w
    return out


def test_water_depth_dose_equals_database_track():
    """Homogeneous water reproduces the database depth-dose: straight single-track
    database, laterally wide phantom, all energy stops inside."""
    db = _straight(I.make_water_track_db([150.0], 1, seed=11))
    ph = I.water_phantom((16, 16, 96), 0.2, origin=(-1.6, -1.6, 0.0))
    sp = I.spots([[0, 0, -1.0]], [[0, 0, 1.0]], [150.0], 0.3, 2000)
    r = O.replay(db, ph, sp, threads=4)
    idd = r["E"].sum(axis=(1, 2)).astype(np.float64)
    z0, dx, ee = _track_profile(db, 0, 0)
    xyz, why = O.endpoints(db, ph, sp, 0, 0, 2000)
    n_stop = int((why == O.END_STOP).sum())
    assert n_stop == 2000 - int((why == O.END_ESCAPE).sum())
    W = np.arange(97) * float(ph.voxel_cm[2])     # voxel size as stored (float32)
    expect = _slab_energy(z0, dx, ee, W)
    # with sigma 3 mm and a 3.2 cm wide box no history leaves through a side face
    assert n_stop == 2000
    assert np.max(np.abs(idd - 2000 * expect)) <= 2000 * 2
    assert r["E"].sum() == 2000 * ee.sum() == r["incident"]


def test_energy_identity_and_skip():
    """Deposited + escaped == incident exactly; the incident energy of a spot
    below its bin energy is the track energy minus the skip."""
    db = I.make_water_track_db([100.0, 105.0], 1, seed=4)
    ph = I.thorax_phantom((48, 40, 24), 0.4, seed=9)
    sp = I.spots([[3, 0, -20.0], [-2, 1, 20.0], [0, 30, 0.0]],
                 [[0, 0, 1.0], [0, 0.2, -1.0], [0, 1.0, 0]], [101.5, 105.0, 100.0], 0.5, 700)
    r = O.replay(db, ph, sp, flags=O.FLAG_VARIANCE | O.FLAG_ROTATE, threads=4)
    assert r["E"].sum() + r["escaped"] == r["incident"]
    T = [int(np.rint(db.steps[db.track_off[t]:db.track_off[t + 1], 1].astype(np.float64) * FP).sum())
         for t in range(2)]
    skip = int(np.rint(np.float32(105.0) * FP)) - int(np.rint(np.float32(101.5) * FP))
    assert r["incident"] == 700 * (T[1] - skip) + 700 * T[1] + 700 * T[0]
    assert r["vacuum_visits"] > 0
    # the third spot points away from the box: every history misses
    _, why = O.endpoints(db, ph, sp, 2, 0, 50)
    assert np.all(why == O.END_MISS)


def test_slab_range_shift_exact():
    """Straight tracks through bone and lung slabs: each geometric slab receives
    the water deposit over its water-equivalent interval (per-voxel RSP scaling)."""
    db = _straight(I.make_water_track_db([120.0], 1, seed=21))
    n = 64
    ph = I.water_phantom((8, 8, 150), 0.1, origin=(-0.4, -0.4, 0.0))
    zc = (np.arange(150) + 0.5) * 0.1
    ph.hu[(zc >= 2.0) & (zc < 3.0)] = 1000
    ph.hu[(zc >= 4.0) & (zc < 6.0)] = -800
    sp = I.spots([[0, 0, -1.0]], [[0, 0, 1.0]], [118.0], 0.02, n)
    r = O.replay(db, ph, sp, threads=2)
    _, rsp, _, _ = O.material(ph.hu[:, 0, 0])
    W = np.concatenate([[0.0], np.cumsum(rsp * float(ph.voxel_cm[2]))])
    skip = int(np.rint(np.float32(120.0) * FP)) - int(np.rint(np.float32(118.0) * FP))
    z0, dx, ee = _track_profile(db, 0, skip)
    expect = _slab_energy(z0, dx, ee, W)
    idd = r["E"].sum(axis=(1, 2)).astype(np.float64)
    assert r["escaped"] == 0
    assert np.max(np.abs(idd - n * expect)) <= n * 2
    # water-equivalent range: bone adds 0.5 cm, lung removes (1-0.20088)*2 cm
    stop = np.nonzero(idd)[0].max()
    R_wel = dx.sum()
    zgeo = np.interp(R_wel, W, np.arange(151) * float(ph.voxel_cm[2]))
    assert int(zgeo / float(ph.voxel_cm[2])) == stop


def test_uniform_medium_scaling():
    """RSP = 1/2 with G = 1 everywhere is water stretched by 2: doubling the voxel
    size, the spot position and its width leaves the tally unchanged."""
    db = I.make_water_track_db([90.0], 20, seed=8)
    half = {"hu": np.array([-1000.0, 3071.0]), "rho": np.array([1.0, 1.0]),
            "rsp": np.array([0.5, 0.5]), "rscp": np.array([0.5, 0.5]), "vacuum_below_hu": -5000.0}
    ph_w = I.water_phantom((24, 24, 80), 0.1, origin=(-1.2, -1.2, 0.0))
    ph_h = I.water_phantom((24, 24, 80), 0.2, origin=(-2.4, -2.4, 0.0))
    sp_w = I.spots([[0.05, -0.1, -0.5]], [[0, 0, 1.0]], [90.0], 0.15, 3000)
    sp_h = I.spots([[0.1, -0.2, -1.0]], [[0, 0, 1.0]], [90.0], 0.3, 3000)
    rw = O.replay(db, ph_w, sp_w, threads=4)
    rh = O.replay(db, ph_h, sp_h, threads=4, table=half)
    assert rw["incident"] == rh["incident"]
    diff = np.abs(rw["E"] - rh["E"]).sum()
    assert diff <= 1e-9 * rw["E"].sum()
    xw, _ = O.endpoints(db, ph_w, sp_w, 0, 0, 200)
    xh, _ = O.endpoints(db, ph_h, sp_h, 0, 0, 200, table=half)
    assert np.allclose(2 * xw, xh, atol=1e-9)


def test_scattering_power_scales_angle():
    """G = 4 with RSP = 1 deflects like water with every database angle doubled."""
    db = I.make_water_track_db([110.0], 30, seed=12)
    db2 = I.TrackDB(db.steps.copy(), db.track_off, db.bin_E, db.bin_first)
    db2.steps[:, 2] *= 2.0
    g4 = {"hu": np.array([-1000.0, 3071.0]), "rho": np.array([1.0, 1.0]),
          "rsp": np.array([1.0, 1.0]), "rscp": np.array([4.0, 4.0]), "vacuum_below_hu": -5000.0}
    ph = I.water_phantom((30, 30, 60), 0.2, origin=(-3.0, -3.0, 0.0))
    sp = I.spots([[0, 0, -1.0]], [[0, 0, 1.0]], [110.0], 0.3, 640)
    xa, ra = O.endpoints(db, ph, sp, 0, 0, 640, table=g4)
    xb, rb = O.endpoints(db2, ph, sp, 0, 0, 640)
    assert np.array_equal(ra, rb)
    assert np.max(np.abs(xa - xb)) < 1e-9
    x1, _ = O.endpoints(db, ph, sp, 0, 0, 640)
    assert np.max(np.abs(x1 - xa)) > 1e-3      # the scaling is not a no-op


def test_source_is_gaussian_and_tracks_rotate_rigidly():
    """Straight tracks end at source + range * direction with a Gaussian lateral
    spread; with track rotation on, each history's deflected end point differs
    from its straight end point by a vector of the same length as without it."""
    db = I.make_water_track_db([100.0], 3, seed=2)
    ph = I.water_phantom((60, 60, 50), 0.2, origin=(-6.0, -6.0, 0.0))
    sp = I.spots([[0.4, -0.3, -2.0]], [[0, 0, 1.0]], [100.0], 0.5, 4096)
    x0, r0 = O.endpoints(_straight(db), ph, sp, 0, 0, 4096)
    assert np.all(r0 == O.END_STOP)
    assert stats.kstest((x0[:, 0] - 0.4) / 0.5, "norm").pvalue > 1e-3
    assert stats.kstest((x0[:, 1] + 0.3) / 0.5, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(x0[:, 0], x0[:, 1])[0, 1]) < 0.05
    xa, _ = O.endpoints(db, ph, sp, 0, 0, 4096)
    xb, _ = O.endpoints(db, ph, sp, 0, 0, 4096, flags=O.FLAG_ROTATE)
    la = np.linalg.norm((xa - x0)[:, :2], axis=1)
    lb = np.linalg.norm((xb - x0)[:, :2], axis=1)
    assert np.allclose(la, lb, atol=1e-9)
    assert np.allclose(xa[:, 2], xb[:, 2], atol=1e-9)
    # without rotation the 64 histories of a chunk share the deflection pattern
    dev = (xa - x0)[:, :2].reshape(64, 64, 2)
    assert np.allclose(dev, dev[:, :1, :], atol=1e-9)
    assert not np.allclose((xb - x0)[:64, :2], (xb - x0)[:1, :2], atol=1e-6)


def test_disk_field_is_uniform_over_its_disk():
    """A spot with sigma = -R starts its histories uniformly over the disk of
    radius R perpendicular to the beam (the circular field of Section 2.5):
    straight tracks end at the start point's lateral position, so every end
    point lies within R of the axis, (r / R)^2 and the polar angle are
    uniform, and the lateral centroid is the axis."""
    db = I.make_water_track_db([100.0], 3, seed=2)
    ph = I.water_phantom((60, 60, 50), 0.2, origin=(-6.0, -6.0, 0.0))
    R = 2.5
    sp = I.disk_field([0.4, -0.3, -2.0], [0, 0, 1.0], 100.0, R, 4096)
    assert sp["sigma_cm"][0] == -R
    x0, r0 = O.endpoints(_straight(db), ph, sp, 0, 0, 4096)
    assert np.all(r0 == O.END_STOP)
    dx, dy = x0[:, 0] - 0.4, x0[:, 1] + 0.3
    rr = np.hypot(dx, dy)
    assert rr.max() <= R * (1 + 1e-6) and rr.max() > 0.98 * R
    assert stats.kstest((rr / R) ** 2, "uniform").pvalue > 1e-3
    assert stats.kstest((np.arctan2(dy, dx) + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3
    assert abs(dx.mean()) < 4 * R / 2 / np.sqrt(4096) and abs(dy.mean()) < 4 * R / 2 / np.sqrt(4096)
    # the same draws with sigma = +R give the Gaussian spot: a different law
    g, _ = O.endpoints(_straight(db), ph, I.spots([[0.4, -0.3, -2.0]], [[0, 0, 1.0]], [100.0], R, 4096), 0, 0, 4096)
    assert np.hypot(g[:, 0] - 0.4, g[:, 1] + 0.3).max() > 1.5 * R


def test_gantry_direction_straight_tracks():
    db = _straight(I.make_water_track_db([80.0], 1, seed=5))
    ph = I.water_phantom((40, 40, 40), 0.25, origin=(-5.0, -5.0, -5.0))
    R = db.steps[:, 0].astype(np.float64).sum()
    for d in ([0, -1.0, 0], [-1.0, 0, 0], [0.6, 0.8, 0]):
        d = np.array(d)
        p = -8.0 * d
        sp = I.spots([p], [d], [80.0], 0.0, 10)
        x, why = O.endpoints(db, ph, sp, 0, 0, 10)
        assert np.all(why == O.END_STOP)
        tin = 8.0 - 5.0 / np.max(np.abs(d))
        assert np.allclose(x, p + (tin + R) * d, atol=1e-9)


def test_single_voxel_variance_closed_form():
    """One large voxel, a single-track database: every history deposits I_h in one
    visit, so E = N I_h and E2 = N ((I_h + 2^11) >> 12)^2; Eq. (2) then gives ~0."""
    db = I.make_water_track_db([60.0], 1, seed=6)
    ph = I.water_phantom((1, 1, 1), 40.0, origin=(-20.0, -20.0, 0.0))
    sp = I.spots([[0, 0, -1.0]], [[0, 0, 1.0]], [58.0], 0.3, 500)
    r = O.replay(db, ph, sp, threads=2)
    T = int(np.rint(db.steps[:, 1].astype(np.float64) * FP).sum())
    I_h = T - (int(np.rint(np.float32(60.0) * FP)) - int(np.rint(np.float32(58.0) * FP)))
    assert r["E"].ravel()[0] == 500 * I_h
    assert int(r["E2"].ravel()[0]) == 500 * ((I_h + 2048) >> 12) ** 2
    dose, var = O.dose_and_variance(r["E"], r["E2"], 500, ph)
    m = 1.0 * 40.0 ** 3 * 1e-3
    assert math.isclose(dose.ravel()[0], I_h / FP * O.MEV_J / m, rel_tol=1e-12)
    # identical histories: only the 2^-12 MeV rounding of q remains
    assert abs(var.ravel()[0]) <= dose.ravel()[0] ** 2 * 1e-5 / 499


def test_two_valued_histories_variance():
    """Half the histories miss a thin one-voxel box: D_i is 0 or D, and Eq. (2)
    gives p (1 - p) D^2 / (N - 1) with p the hit fraction."""
    db = I.make_water_track_db([60.0], 1, seed=6)
    ph = I.water_phantom((1, 1, 1), 40.0, origin=(0.0, -20.0, 0.0))
    N = 4000
    sp = I.spots([[0, 0, -1.0]], [[0, 0, 1.0]], [60.0], 0.5, N)
    r = O.replay(db, ph, sp, threads=2)
    _, why = O.endpoints(db, ph, sp, 0, 0, N)
    hits = int((why == O.END_STOP).sum())
    assert 1700 < hits < 2300
    dose, var = O.dose_and_variance(r["E"], r["E2"], N, ph)
    p = hits / N
    D = dose.ravel()[0] / p
    assert math.isclose(var.ravel()[0], p * (1 - p) * D * D / (N - 1), rel_tol=1e-6)


def test_mean_and_batch_uncertainty():
    d = np.array([1.0, 0.9, 0.6, 0.4, 0.1])
    s = np.array([0.02, 0.01, 0.03, 0.5, 0.5])
    assert math.isclose(O.mean_uncertainty(d, s), (0.02 + 0.01 / 0.9 + 0.05) / 3)
    mean, sig = O.batch_uncertainty([np.array([1.0, 2.0]), np.array([3.0, 2.0])])
    assert np.allclose(mean, [2.0, 2.0]) and np.allclose(sig, [1.0, 0.0])


def test_openmp_split_is_bitwise_identical():
    db = I.make_water_track_db([120.0, 125.0], 8, seed=1)
    ph = I.thorax_phantom((32, 32, 16), 0.5, seed=3)
    sp = I.spots([[1, 2, -20.0], [0, 0, 20.0]], [[0, 0, 1.0], [0, 0, -1.0]], [121.0, 125.0], 0.4, 333)
    a = O.replay(db, ph, sp, threads=1)
    b = O.replay(db, ph, sp, threads=7)
    assert np.array_equal(a["E"], b["E"]) and np.array_equal(a["E2"], b["E2"])
    # a run split into two ranges equals the whole run (history identity keys everything)
    h = np.array([150, 150], np.uint64)
    c1 = O.replay(db, ph, sp, h_count=h, threads=3)
    c2 = O.replay(db, ph, sp, h_begin=h, h_count=np.array([183, 183], np.uint64), threads=3)
    assert np.array_equal(c1["E"] + c2["E"], a["E"])


def test_partial_first_step_equals_truncated_track():
    """A spot below its bin energy starts inside a step: replaying the track from
    that step with the step cut to fraction f (length f dx, angle sqrt(f) theta,
    Highland's sqrt(x) dependence) equals replaying a database whose first step
    was cut that way in advance, entered at the spot energy."""
    db = I.make_water_track_db([100.0], 1, seed=14)
    e = np.rint(db.steps[:, 1].astype(np.float64) * FP).astype(np.int64)
    skip = int(np.rint(np.float32(100.0) * FP)) - int(np.rint(np.float32(99.7) * FP))
    assert 0 < skip < e[0]
    f = (e[0] - skip) / e[0]
    cut = db.steps.copy()
    cut[0, 0] = np.float32(f * cut[0, 0])
    cut[0, 2] = np.float32(math.sqrt(f) * cut[0, 2])
    # the cut step must carry exactly e0 - skip fixed-point units
    cut[0, 1] = np.float32((e[0] - skip) / FP)
    assert int(np.rint(np.float64(cut[0, 1]) * FP)) == e[0] - skip
    db_cut = I.TrackDB(cut, db.track_off, np.array([99.7], np.float32), db.bin_first)
    ph = I.water_phantom((40, 40, 50), 0.2, origin=(-4.0, -4.0, 0.0))
    sp = I.spots([[0, 0, -1.0]], [[0, 0, 1.0]], [99.7], 0.3, 256)
    xa, ra = O.endpoints(db, ph, sp, 0, 0, 256)
    xb, rb = O.endpoints(db_cut, ph, sp, 0, 0, 256)
    assert np.array_equal(ra, rb)
    assert np.max(np.abs(xa - xb)) < 1e-6


def test_sum_of_squares_rounding_several_energies():
    """E2 adds ((I_h + 2^11) >> 12)^2 per one-visit history, for several I_h."""
    db = I.make_water_track_db([60.0], 1, seed=6)
    ph = I.water_phantom((1, 1, 1), 40.0, origin=(-20.0, -20.0, 0.0))
    Es = [57.1, 57.9, 58.3, 58.8, 59.2, 59.6]
    sp = I.spots([[0, 0, -1.0]] * 6, [[0, 0, 1.0]] * 6, Es, 0.3, 100)
    r = O.replay(db, ph, sp, threads=2)
    T = int(np.rint(db.steps[:, 1].astype(np.float64) * FP).sum())
    Ih = [T - (int(np.rint(np.float32(60.0) * FP)) - int(np.rint(np.float32(x) * FP))) for x in Es]
    assert len({(i % 4096) >= 2048 for i in Ih}) == 2       # both rounding directions occur
    assert r["E"].ravel()[0] == 100 * sum(Ih)
    assert int(r["E2"].ravel()[0]) == 100 * sum(((i + 2048) >> 12) ** 2 for i in Ih)


# ------------------------------------------------- voxel-walk tie-breaks ----
# Hand-computed walks in a 4 x 4 x 4 water phantom of 1 cm voxels (origin at
# 0): straight tracks (theta = 0) of 1 MeV steps, a spot of zero width.  Each
# event is (kind, voxel, piece, exit axis); a step of WEL 1.5 cm crossing a
# face after 1 cm deposits rint(2^24 * 1 / 1.5) = 11184811 before the face and
# the remaining 5592405 after it.  Voxel index v = (k * 4 + j) * 4 + i.
E1 = 16777216
P23, P13 = 11184811, 5592405


def _tie_db(dx, n_steps, dE=1.0):
    steps = np.zeros((n_steps, 4), np.float32)
    steps[:, 0] = dx
    steps[:, 1] = dE
    E = np.float32(dE * n_steps)
    return I.TrackDB(steps, np.array([0, n_steps], np.uint64), np.array([E], np.float32),
                     np.array([0, 1], np.uint32)), float(E)


def _tie_run(pos, d, dx=1.5, n_steps=3):
    db, E = _tie_db(dx, n_steps)
    ph = I.Phantom(np.zeros((4, 4, 4), np.int16), np.ones(3, np.float32), np.zeros(3, np.float32))
    sp = I.spots([pos], [d], [E], 0.0, 1)
    ev, reason, ep = O.trace(db, ph, sp, 0, 0)
    return ev, reason, ep, (db, ph, sp)


def test_walk_ray_along_a_face_takes_the_upper_voxel():
    """A ray along +x in the plane y = 1 (a voxel boundary, no y motion) walks
    the voxels with y index 1; a step that ends exactly on a face crosses it in
    that step (the next step starts in the entered voxel)."""
    ev, reason, ep, _ = _tie_run([-1.0, 1.0, 2.5], [1.0, 0.0, 0.0])
    got = [e[:4] for e in ev]
    assert got == [(0, 36, P23, 0), (0, 37, P13, -1), (2, 0, 0, -1),
                   (0, 37, P13, 0), (0, 38, P23, 0), (2, 1, 0, -1),       # step 2 ends on the x = 3 face
                   (0, 39, P23, 0), (3, -1, 3 * E1 - (3 * P23 + 2 * P13), 0)]
    assert [e[4] for e in ev if e[0] == 0] == [1.0, 0.5, 0.5, 1.0, 1.0]
    assert reason == O.END_ESCAPE and ep.tolist() == [4.0, 1.0, 2.5]


def test_walk_entry_on_the_far_face_moving_down():
    """Entering through the x = 4 face moving -x starts in voxel i = 3 (a point
    on a face belongs to the voxel entered); y = 2 and z = 0 are boundaries
    with no motion along them: j = 2, k = 0."""
    ev, reason, ep, _ = _tie_run([5.0, 2.0, 0.0], [-1.0, 0.0, 0.0])
    got = [e[:4] for e in ev]
    assert got == [(0, 11, P23, 0), (0, 10, P13, -1), (2, 0, 0, -1),
                   (0, 10, P13, 0), (0, 9, P23, 0), (2, 1, 0, -1),
                   (0, 8, P23, 0), (3, -1, P13, 0)]
    assert reason == O.END_ESCAPE and ep.tolist() == [0.0, 2.0, 0.0]


def test_walk_rays_along_an_axis_on_box_faces():
    """On the low face of the box (x = 0, moving along y) the ray is inside;
    on the high face (x = 4) it misses: the box is [o, o + n * voxel)."""
    ev, reason, _, _ = _tie_run([0.0, -1.0, 0.5], [0.0, 1.0, 0.0])
    assert [e[1] for e in ev if e[0] == 0][:2] == [0, 4] and reason == O.END_ESCAPE
    ev, reason, _, _ = _tie_run([4.0, -1.0, 0.5], [0.0, 1.0, 0.0])
    assert ev == [] and reason == O.END_MISS


@pytest.mark.parametrize("d,seq", [
    ((1.0, 1.0, 0.0), [32, 33, 37]),          # x before y
    ((1.0, 0.0, 1.0), [32, 33, 49]),          # x before z
    ((0.0, 1.0, 1.0), [32, 36, 52]),          # y before z
    ((1.0, 1.0, 1.0), [32, 33, 37, 53]),      # x, then y, then z
])
def test_walk_simultaneous_crossings_go_x_then_y_then_z(d, seq):
    """From the centre of voxel (0, 0, 2) along a diagonal the exit distances
    tie: the faces are crossed in the order x, y, z, through intermediate voxels
    that get a zero-length piece (no WEL, no deposit)."""
    ev, _, _, _ = _tie_run([0.5, 0.5, 2.5], list(d), dx=3.0, n_steps=1)
    vox = [e for e in ev if e[0] == 0]
    assert [e[1] for e in vox[:len(seq)]] == seq
    for e in vox[1:len(seq) - 1]:
        assert e[4] <= 1e-12 and e[2] == 0                 # the intermediate voxels: zero length
    assert vox[0][4] > 0.5 and vox[len(seq) - 1][4] > 0.5


def test_walk_trace_agrees_with_the_tallies():
    """The walk record is the replay itself: its pieces per voxel sum to the
    energy tally of the same history, and zero pieces do not flush."""
    ev, _, _, (db, ph, sp) = _tie_run([0.5, 0.5, 2.5], [1.0, 1.0, 1.0], dx=3.0, n_steps=1)
    r = O.replay(db, ph, sp)
    E = np.zeros(64, np.int64)
    for k, v, piece, *_ in ev:
        if k == 0:
            E[v] += piece
    assert np.array_equal(E, r["E"].ravel())
    runs = [v for i, (k, v, piece, *_) in enumerate(ev) if k == 0 and piece]
    assert r["flushes"] == len(runs)


# -------------------------------------------- database physics, low energy ----
@pytest.mark.parametrize("E,theta0_mrad,bohr_mev,stop_mev_cm", [
    (150.0, 2.12, 0.101, 5.42),
    (70.0, 4.52, 0.097, 9.75),
    (20.0, 16.2, 0.094, 25.6),
])
def test_db_physics_closed_forms(E, theta0_mrad, bohr_mev, stop_mev_cm):
    """Highland width, Bohr straggling and Bragg-Kleeman stopping power per
    1 mm of water at 150, 70 and 20 MeV against values worked out by hand from
    the textbook formulas (beta from the kinetic energy and the proton mass;
    stopping power = 1 / (alpha p E^(p-1))).  At 20 MeV beta^2 = 0.0413, where a
    wrong beta or momentum term moves every value by more than the tolerance."""
    assert abs(I.highland_theta0(E, 0.1) * 1e3 - theta0_mrad) <= 0.006 * theta0_mrad
    assert abs(I.bohr_sigma(E, 0.1) - bohr_mev) <= 0.006 * bohr_mev
    s = 1.0 / (0.0022 * 1.77 * E ** 0.77)
    assert abs(s - stop_mev_cm) <= 0.003 * stop_mev_cm
    # the generator's mean loss over a 1 mm step (the range difference) lies
    # between the stopping powers at the step's two ends times its length
    E_end = I.energy_at_range(I.csda_range(E) - 0.1)
    s_end = 1.0 / (0.0022 * 1.77 * E_end ** 0.77)
    assert s * 0.1 < E - E_end < s_end * 0.1


@pytest.mark.parametrize("Eb", [20.0, 70.0])
def test_db_first_step_distributions_low_energy(Eb):
    """The first step of 2000 tracks at 70 and 20 MeV: energy loss normal
    around the Bragg-Kleeman mean with Bohr's width at the mid-step energy, and
    the polar angle Rayleigh with Highland's width there."""
    db = I.make_water_track_db([Eb], 2000, seed=11)
    first = db.steps[db.track_off[:-1].astype(np.int64)]
    R = I.csda_range(Eb)
    Emid = I.energy_at_range(R - 0.05)
    mean = Eb - I.energy_at_range(R - 0.1)
    sig = I.bohr_sigma(Emid, 0.1)
    z = (first[:, 1].astype(np.float64) - mean) / sig
    assert stats.kstest(z, "norm").pvalue > 1e-3
    th0 = I.highland_theta0(Emid, 0.1)
    assert stats.kstest(first[:, 2] / th0, "rayleigh").pvalue > 1e-3
    assert stats.kstest(first[:, 3] / np.pi, "uniform", args=(-1, 2)).pvalue > 1e-3
    # the whole track: range and energy sum
    L = np.add.reduceat(db.steps[:, 0].astype(np.float64), db.track_off[:-1].astype(np.int64))
    S = np.add.reduceat(db.steps[:, 1].astype(np.float64), db.track_off[:-1].astype(np.int64))
    assert abs(L.mean() / R - 1) < 5e-3
    assert np.max(np.abs(S - Eb)) < 1e-4 * Eb


def test_per_visit_squares_against_eq2_taken_literally():
    """The squared-energy tally squares each voxel visit; Eq. (2) squares a
    history's whole dose in a voxel.  The oracle computes both (the literal
    one with a per-history voxel map): on the water pencil beam and the slab
    the mean uncertainty differs by less than 0.05%, and the literal sum of
    squares is not smaller overall (squares of sums exceed sums of squares up
    to the 2^-12 MeV rounding of each term)."""
    for (ph, sp, db), per in ((W.water_pencil(), 20_000), (W.slab(n_tracks=500), 800)):
        r = O.replay(db, ph, sp, h_count=np.full(len(sp), per, np.uint64), exact_e2=True, table=O.ORACLE_HU_TABLE)
        n = r["n_histories"]
        _, _, _, vac = O.material(ph.hu)
        vac = vac.reshape(ph.hu.shape)
        d, v = O.dose_and_variance(r["E"], r["E2"], n, ph)
        _, vx = O.dose_and_variance(r["E"], r["E2x"], n, ph)
        u = O.mean_uncertainty(d, np.sqrt(np.maximum(v, 0)), vac)
        ux = O.mean_uncertainty(d, np.sqrt(np.maximum(vx, 0)), vac)
        assert 0.9999 <= ux / u <= 1.0005, (ux, u)
        ratio = float(r["E2x"].sum()) / float(r["E2"].sum())
        assert 0.99999 <= ratio <= 1.001
    # one voxel holding every track: one visit per history, the two agree bit for bit
    db = W.water_db(200)
    ph = I.Phantom(np.zeros((1, 1, 1), np.int16), np.array([40.0, 40.0, 40.0], np.float32),
                   np.array([-20.0, -20.0, 0.0], np.float32))
    sp = I.spots([[0.0, 0.0, -1.0]], [[0.0, 0.0, 1.0]], [150.0], 0.3, 3000)
    r = O.replay(db, ph, sp, exact_e2=True)
    assert np.array_equal(r["E2"], r["E2x"]) and r["escaped"] == 0


# ------------------------------------------------------------ phase space ----
def test_phase_space_of_one_point_equals_a_zero_width_spot():
    """Protons listed at one position, direction and energy replay exactly as a
    spot of zero width there (same source index, same tracks, same histories):
    the tallies are bit for bit equal; listing them over two energy bins splits
    them into two sources whose sum keeps the energy identity."""
    db = I.make_water_track_db([95.0, 100.0, 105.0], 60, seed=4)
    ph = I.thorax_phantom((40, 36, 30), 0.4, seed=2)
    sp = I.spots([[0.3, -0.2, -20.0]], [[0.1, 0.0, 1.0]], [98.5], 0.0, 500)
    a = O.replay(db, ph, sp)
    n = 500
    ps = O.phase_space_sources(np.tile([0.3, -0.2, -20.0], (n, 1)), np.tile([0.1, 0.0, 1.0], (n, 1)),
                               np.full(n, 98.5), db.bin_E, 0)
    assert ps["count"].tolist() == [n] and ps["bins"] == [1]
    b = O.replay(db, ph, sp, phase_space=ps)              # the spot row is a placeholder now
    assert np.array_equal(a["E"], b["E"]) and np.array_equal(a["E2"], b["E2"])
    assert a["incident"] == b["incident"] and a["escaped"] == b["escaped"]
    # two bins: protons at 98.5 and 103 MeV alternate in the list -> two sources
    E = np.where(np.arange(n) % 2 == 0, 98.5, 103.0)
    ps2 = O.phase_space_sources(np.tile([0.3, -0.2, -20.0], (n, 1)), np.tile([0.1, 0.0, 1.0], (n, 1)), E,
                                db.bin_E, 0)
    assert ps2["count"].tolist() == [250, 250] and ps2["bins"] == [1, 2]
    assert np.all(ps2["E"][:250] == np.float32(98.5)) and np.all(ps2["E"][250:] == np.float32(103.0))
    sp2 = np.concatenate([sp, sp])
    c = O.replay(db, ph, sp2, h_count=ps2["count"], phase_space=ps2)
    assert int(c["E"].sum()) + c["escaped"] == c["incident"]
    # the 98.5 MeV source is the first 250 histories of the single-bin run
    d = O.replay(db, ph, sp, h_count=np.array([250], np.uint64), phase_space=ps)
    e = O.replay(db, ph, sp2, h_count=np.array([250, 0], np.uint64), phase_space=ps2)
    assert np.array_equal(d["E"], e["E"])


def test_phase_space_recycles_protons_with_new_tracks():
    """History h of a listed source is proton h mod count: a second pass over
    the list re-uses each proton (same start, same energy) on another track, so
    its incident energies follow the protons while the tallies differ."""
    db = I.make_water_track_db([100.0, 105.0], 400, seed=8)
    ph = I.water_phantom((24, 24, 60), 0.25, origin=(-3.0, -3.0, 0.0))
    rng = np.random.default_rng(3)
    n = 64
    pos = np.column_stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), np.full(n, -5.0)])
    dirs = np.column_stack([rng.normal(0, 0.01, n), rng.normal(0, 0.01, n), np.ones(n)])
    E = rng.uniform(100.5, 104.5, n)
    ps = O.phase_space_sources(pos, dirs, E, db.bin_E, 0)
    sp = I.spots([[0, 0, -5.0]], [[0, 0, 1.0]], [101.0], 0.0, n)
    one = O.replay(db, ph, sp, h_count=np.array([n], np.uint64), phase_space=ps)
    two = O.replay(db, ph, sp, h_count=np.array([2 * n], np.uint64), phase_space=ps)
    second = O.replay(db, ph, sp, h_begin=np.array([n], np.uint64), h_count=np.array([n], np.uint64),
                      phase_space=ps)
    assert np.array_equal(two["E"], one["E"] + second["E"])
    assert not np.array_equal(one["E"], second["E"])
    xo, ro = O.endpoints(db, ph, sp, 0, 0, n, phase_space=ps)
    x2, r2 = O.endpoints(db, ph, sp, 0, n, n, phase_space=ps)
    assert np.all(ro == 0) and np.all(r2 == 0)                  # all stop inside (range < 15 cm of water)
    assert not np.allclose(xo, x2)
