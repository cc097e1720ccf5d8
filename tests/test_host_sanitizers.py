"""Host code under the sanitizers, and the LDS tally cache's update protocol
as a CPU model.  CPU only.

  * the CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (gcc), replaying a small thorax problem: no report, and the same integer
    results as the ordinary build;
  * the library's host runtime (the C ABI in api.hip, host side instrumented;
    the kernels are only linked) driven through a context without a GPU: every
    documented status code, no report, no leak;
  * the write-back cache protocol restated with std::atomic words and host
    threads as lanes: exact per-voxel sums for every slot count, voxel set and
    field width (misdirected adds, same-voxel merges, half-field flushes,
    deposits too large for the cache).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1011_2188_amd import build as B
from paper_1011_2188_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def _need(tool):
    if shutil.which(tool) is None and not os.path.exists(tool):
        pytest.skip(f"{tool} not available")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{cmd[0]} failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def _write_problem(path, ph, sp, table):
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


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    _need("gcc")
    from oracle import oracle as O
    db = I.make_water_track_db([95.0, 100.0, 105.0], 40, seed=9)
    ph = I.thorax_phantom((40, 36, 24), 0.4, seed=4)
    sp = I.spots([[0.2, -0.3, -20.0], [0.4, 0.1, 20.0], [-20.0, 0.0, 0.5]],
                 [[0, 0, 1.0], [0, 0, -1.0], [1.0, 0, 0]], [97.5, 105.0, 100.0], 0.4, 300)
    I.write_track_db_file(tmp_path / "db.bin", db)
    _write_problem(tmp_path / "p.bin", ph, sp, O.ORACLE_HU_TABLE)
    src = [os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "fdc_oracle.c")]
    _run(["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", *src, "-lm", "-o", str(tmp_path / "san")])
    _run(["gcc", "-O2", "-std=gnu11", "-fopenmp", *src, "-lm", "-o", str(tmp_path / "plain")])
    args = [str(tmp_path / "db.bin"), str(tmp_path / "p.bin")]
    a = _run([str(tmp_path / "san"), *args], env=SAN_ENV)
    b = _run([str(tmp_path / "plain"), *args], env=SAN_ENV)
    assert "runtime error" not in a.stderr and "Sanitizer" not in a.stderr
    assert a.stdout == b.stdout and "replay rc=0" in a.stdout
    # and the same tallies as the library-loaded oracle
    r = O.replay(db, ph, sp, flags=O.FLAG_VARIANCE, threads=2)
    assert f"incident={r['incident']} escaped={r['escaped']}" in a.stdout


def test_host_runtime_under_address_and_ub_sanitizers(tmp_path):
    hipcc = B.hipcc()
    objs = [os.path.join(B.BUILD, os.path.splitext(s)[0] + ".o") for s in B.SOURCES if s != "api.hip"]
    if not all(os.path.exists(o) for o in objs):
        B.build()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    api = str(tmp_path / "api.o")
    drv = str(tmp_path / "drv.o")
    exe = str(tmp_path / "host_runtime")
    _run([hipcc, "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={B.ARCH}", "-Xclang", "-target-feature",
          "-Xclang", "-packed-fp32-ops", *san, "-I", os.path.join(ROOT, "include"), "-I", B.CSRC, "-c",
          os.path.join(B.CSRC, "api.hip"), "-o", api])
    _run([hipcc, "-O1", "-g", "-std=c++17", *san, "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(HERE, "host_runtime_driver.cpp"), "-o", drv])
    _run([hipcc, f"--offload-arch={B.ARCH}", *san, drv, api, *objs, "-o", exe])
    I.write_track_db_file(tmp_path / "db.bin", I.make_water_track_db([100.0, 105.0], 5, seed=1))
    r = _run([exe, str(tmp_path / "db.bin")], env=SAN_ENV)
    assert r.stdout.strip().endswith("ok") and "FAIL" not in r.stdout
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr


@pytest.mark.parametrize("cfg", [
    "16 3 40 24 200000 1",        # 3 slots for 40 voxels: constant eviction and misdirected adds
    "16 61 500 20 200000 2",
    "8 256 4096 33 100000 3",     # a realistic field width (a 2^31-voxel plan)
    "16 7 7 16 100000 4",         # narrow field: half-field flushes every few thousand adds
    "16 1 64 14 100000 5",        # one slot
])
def test_lds_cache_protocol_model(tmp_path, cfg):
    _need("g++")
    exe = str(tmp_path / "cm")
    _run(["g++", "-O2", "-std=c++17", "-pthread", os.path.join(HERE, "cache_model.cpp"), "-o", exe])
    r = _run([exe, *cfg.split()])
    assert r.stdout.startswith("ok") and "mismatches=0" in r.stdout


def test_lds_cache_protocol_model_under_thread_sanitizer(tmp_path):
    """The model's shared state is only touched through atomics: no data race."""
    _need("g++")
    exe = str(tmp_path / "cm_tsan")
    _run(["g++", "-O1", "-g", "-std=c++17", "-pthread", "-fsanitize=thread", os.path.join(HERE, "cache_model.cpp"),
          "-o", exe])
    r = _run([exe, "8", "5", "40", "20", "20000", "7"], env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert r.stdout.startswith("ok") and "WARNING: ThreadSanitizer" not in r.stderr
