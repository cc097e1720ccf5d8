"""The library's per-history walk compiled for the host (tests/walk_host.cpp
includes transport.hip) under AddressSanitizer and UBSan, against the oracle:
CPU only.  Every voxel-word, step-record and table access of the walk -
including the vacuum free-flight moves across whole blocks of air - stays in
bounds, energy is conserved exactly, the incident energy equals the oracle's,
the walk's counts of steps, voxel pieces and flushes match the oracle's within
0.1%,
the dose agrees within 0.5% of Dmax above 10% of Dmax and at least 99.9% of the
end points agree within 1e-4 cm with the same end reason."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_1011_2188_amd import build as B
from paper_1011_2188_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def walk_exe(tmp_path_factory):
    hipcc = B.hipcc()
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("walk") / "walk_host")
    cmd = [hipcc, "-O1", "-g", "-std=c++17", f"--offload-arch={B.ARCH}", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", B.CSRC,
           os.path.join(HERE, "walk_host.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def _write_problem(path, ph, sp, table, flags, R):
    with open(path, "wb") as f:
        f.write(np.array(ph.shape_xyz, "<i4").tobytes())
        f.write(np.asarray(ph.voxel_cm, "<f8").tobytes())
        f.write(np.asarray(ph.origin_cm, "<f8").tobytes())
        f.write(np.array([len(table["hu"])], "<i4").tobytes())
        for k in ("hu", "rho", "rsp", "rscp"):
            f.write(np.asarray(table[k], "<f8").tobytes())
        f.write(np.array([table["vacuum_below_hu"]], "<f8").tobytes())
        f.write(np.array([len(sp)], "<u4").tobytes())
        for k, dt in (("pos_cm", "<f4"), ("dir", "<f4"), ("energy_MeV", "<f4"), ("sigma_cm", "<f4"),
                      ("n_histories", "<u8")):
            f.write(np.ascontiguousarray(sp[k], dt).tobytes())
        f.write(np.ascontiguousarray(ph.hu, "<i2").tobytes())
        f.write(np.array([flags, R], "<u4").tobytes())


def _compare(tmp_path, exe, db, ph, sp, flags=O.FLAG_VARIANCE, R=64):
    I.write_track_db_file(tmp_path / "db.bin", db)
    _write_problem(tmp_path / "p.bin", ph, sp, I.HU_TABLE_DEFAULT, flags, R)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path / "db.bin"), str(tmp_path / "p.bin"), str(tmp_path / "out")],
                       capture_output=True, text=True, env=env)
    assert r.returncode == 0 and "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    inc, esc, n_steps, n_visits, n_flushes = (int(x) for x in r.stdout.split())
    shape = ph.hu.shape
    E = np.fromfile(tmp_path / "out.E", np.int64).reshape(shape)
    E2 = np.fromfile(tmp_path / "out.E2", np.uint64).reshape(shape)
    ep = np.fromfile(tmp_path / "out.ep", np.dtype([("xyz", "<f4", (3,)), ("why", "<i4")]))
    o = O.replay(db, ph, sp, seed=1, R=R, flags=flags, table=I.HU_TABLE_DEFAULT)
    assert inc == o["incident"]
    assert int(E.sum()) + esc == inc
    # the walk's own work counts against the oracle's (steps started in the
    # phantom, non-vacuum voxel pieces, flushes; FP32 against FP64 positions
    # can move a rare crossing)
    for mine, theirs in ((n_steps, o["steps"]), (n_visits, o["visits"]), (n_flushes, o["flushes"])):
        assert abs(mine - theirs) <= 1e-3 * theirs, (mine, theirs)
    n = int(sp["n_histories"].sum())
    dose_o, _ = O.dose_and_variance(o["E"], o["E2"], n, ph, table=I.HU_TABLE_DEFAULT)
    dose_h, _ = O.dose_and_variance(E, E2, n, ph, table=I.HU_TABLE_DEFAULT)
    dmax = dose_o.max()
    sel = dose_o > 0.1 * dmax
    assert np.abs(dose_h - dose_o)[sel].max() <= 0.005 * dmax
    good = total = 0
    k = 0
    for s in range(len(sp)):
        cnt = int(sp["n_histories"][s])
        xo, ro = O.endpoints(db, ph, sp, s, 0, cnt, seed=1, R=R, flags=flags, table=I.HU_TABLE_DEFAULT)
        xh, rh = ep["xyz"][k:k + cnt].astype(np.float64), ep["why"][k:k + cnt]
        good += int(((rh == ro) & (np.linalg.norm(xh - xo, axis=1) <= 1e-4)).sum())
        total += cnt
        k += cnt
    assert good >= 0.999 * total, (good, total)
    return E, o


def test_host_walk_thorax_with_air_all_directions(tmp_path, walk_exe):
    """A small thorax in a box of air, fields from six axis directions and two
    oblique ones: each proton crosses air on the way in (free-flight moves of
    up to 15 voxels) and many leave through air, some through box edges."""
    db = I.make_water_track_db([70.0, 75.0, 80.0, 85.0, 90.0], 120, seed=17)
    ph = I.thorax_phantom((56, 48, 40), 0.5, seed=7, scale=(0.6, 0.6, 0.6))
    dirs = [[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 0.3], [-0.4, 1, -1]]
    pos = [[-30.0 * d for d in np.asarray(v, float) / np.linalg.norm(v)] for v in dirs]
    E = [72.0, 75.0, 88.0, 80.0, 84.5, 70.0, 90.0, 77.7]
    sp = I.spots(pos, dirs, E, 1.5, 400)
    _compare(tmp_path, walk_exe, db, ph, sp, flags=O.FLAG_VARIANCE | O.FLAG_ROTATE)


def test_host_walk_grazing_and_corner_rays(tmp_path, walk_exe):
    """Narrow beams along box faces and through air corridors: rays that start
    on voxel boundaries and graze the box edges."""
    db = I.make_water_track_db([100.0, 105.0], 80, seed=3)
    hu = np.full((20, 24, 28), -1000, np.int16)
    hu[5:15, 6:18, 7:21] = 0                       # a water block in air
    hu[8:12, 10:14, 12:16] = -1000                 # with an air pocket inside
    hu[:, :, 0] = 0                                # and a water wall on the x = 0 face
    ph = I.Phantom(hu, np.array([0.5, 0.5, 0.5], np.float32), np.array([-7.0, -6.0, -5.0], np.float32))
    pos = [[-7.0, 0.0, -20.0], [0.0, -6.0, -20.0], [-20.0, 0.0, 0.0], [7.0, 6.0, -20.0], [-20.0, -6.0, -5.0]]
    dirs = [[0, 0, 1.0], [0, 0, 1.0], [1.0, 0, 0], [0, 0, 1.0], [1.0, 1.0, 1.0]]
    sp = I.spots(pos, dirs, [101.0, 103.0, 105.0, 100.0, 104.0], 0.2, 300)
    _compare(tmp_path, walk_exe, db, ph, sp)
