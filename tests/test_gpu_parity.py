"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Criteria (floating point decides only continuous quantities here; integers
that depend on integers alone must match exactly):
  * dose within 0.5% of Dmax in every voxel above 10% of Dmax;
  * at least 99.9% of sampled histories end within 1e-4 cm of the oracle's
    end point, with the same end reason;
  * deposited + escaped == incident exactly, and the incident energy (which
    depends only on the Philox track choice and integer energies) equals the
    oracle's exactly;
  * tallies bitwise identical across launch configurations and batching.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from paper_1011_2188_amd import fdc as F  # noqa: E402
from paper_1011_2188_amd import inputs as I  # noqa: E402
from paper_1011_2188_amd import workloads as W  # noqa: E402

SEED = 1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    torch.cuda.init()


def ctx_for(db, R=64, seed=SEED, **cfg):
    c = F.Context(device=0, seed=seed, reuse_R=R, table=I.HU_TABLE_DEFAULT)
    c.load_track_db(db)
    if cfg:
        c.set_launch_config(**cfg)
    return c


def gpu_run(c, ph, sp, flags=F.FDC_RUN_VARIANCE):
    p = c.load_phantom(ph)
    c.add_beam_spots(p, sp)
    c.run_histories([p], flags)
    r = c.read_dose_and_variance(p, var=bool(flags & F.FDC_RUN_VARIANCE), raw=True)
    r["plan"] = p
    return r


def check_dose(g, o, ph, n):
    dose_o, var_o = O.dose_and_variance(o["E"], o["E2"], n, ph)
    dmax = dose_o.max()
    sel = dose_o > 0.1 * dmax
    err = np.abs(g["dose"] - dose_o)[sel].max() / dmax
    assert err <= 0.005, f"dose differs by {err:.4%} of Dmax"
    return dose_o, var_o


def check_e2(g, o, ph, n):
    """The squared-energy tally voxel by voxel: within 0.5% of its maximum in
    every voxel above 10% of Dmax (the same FP32-vs-FP64 boundary shifts as the
    energy tally, squared per visit)."""
    dose_o, _ = O.dose_and_variance(o["E"], o["E2"], n, ph)
    sel = dose_o > 0.1 * dose_o.max()
    e2g, e2o = g["E2"].astype(np.float64), o["E2"].astype(np.float64)
    err = np.abs(e2g - e2o)[sel].max() / e2o[sel].max()
    assert err <= 0.005, f"squared-energy tally differs by {err:.4%} of its maximum"


def check_energy(g, o):
    assert g["deposited"] + g["escaped"] == g["incident"]
    assert int(g["E"].sum()) == g["deposited"]
    assert g["incident"] == o["incident"]


def check_endpoints(c, plan, db, ph, sp, spot, h0, n, flags=0, R=64):
    xg, rg = c.debug_endpoints(plan, spot, h0, n, flags)
    xo, ro = O.endpoints(db, ph, sp, spot, h0, n, seed=SEED, R=R, flags=flags)
    same = rg == ro
    close = np.linalg.norm(xg.astype(np.float64) - xo, axis=1) <= 1e-4
    ok = same & close
    return int(ok.sum()), n


# ---------------------------------------------------------------- units -----
def test_device_philox_bitwise():
    c = F.Context(device=0, seed=0x1234_5678_9ABC_DEF0)
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2 ** 32, size=(1_000_000, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:1000, 1:] = 0
    g = c.debug_philox(ctr)
    o = O.philox_batch(ctr, [0x9ABCDEF0, 0x12345678])
    assert np.array_equal(g, o)


def test_transport_timing_events():
    """The library's events bracket the transport kernel of each timed run:
    positive durations, the last n runs, and no more than were timed."""
    db = W.multi_bin_db(2000)
    c = ctx_for(db, waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=1, tally_mode=1,
                source_order=1)
    ph = I.slab_phantom(64, 0.2)
    p = c.load_phantom(ph)
    c.add_beam_spots(p, W.slab_spots(2000))
    c.run_histories([p])                       # untimed
    c.set_timing(True)
    for _ in range(3):
        c.run_histories([p])
    ms = c.transport_times(3)
    assert ms.shape == (3,) and np.all(ms > 0) and np.all(ms < 1000)
    with pytest.raises(F.FdcError):
        c.transport_times(4)
    for _ in range(70):                        # the ring keeps the last 64
        c.run_histories([p], 0)
    assert c.transport_times(64).shape == (64,)
    with pytest.raises(F.FdcError):
        c.transport_times(65)
    c.set_timing(False)


def test_device_material_table():
    c = F.Context(device=0, table=I.HU_TABLE_DEFAULT)
    rsp, g, rho = c.debug_material()
    hu = (np.arange(4096) - 1024).astype(np.int16)
    rho_o, rsp_o, g_o, vac = O.material(hu)
    assert np.array_equal(rsp == 0, vac)
    assert np.allclose(rsp, rsp_o, rtol=1e-6, atol=0)
    assert np.allclose(g, g_o, rtol=1e-6, atol=0)
    assert np.allclose(rho, rho_o, rtol=1e-6, atol=0)


# ---------------------------------------------------------------- parity ----
def test_water_pencil_full_parity():
    """64^3 water, one 150 MeV pencil beam, 1e5 histories (all of them)."""
    ph, sp, db = W.water_pencil()
    c = ctx_for(db)
    g = gpu_run(c, ph, sp)
    o = O.replay(db, ph, sp, seed=SEED)
    check_energy(g, o)
    _, var_o = check_dose(g, o, ph, 100_000)
    check_e2(g, o, ph, 100_000)
    assert abs(g["escaped"] - o["escaped"]) <= 1e-6 * o["incident"]
    sel = g["dose"] > 0.5 * g["dose"].max()
    ug = np.mean(np.sqrt(g["var"][sel]) / g["dose"][sel])
    uo = np.mean(np.sqrt(var_o[sel]) / g["dose"][sel])
    assert abs(ug / uo - 1) < 0.01
    ok, n = check_endpoints(c, g["plan"], db, ph, sp, 0, 0, 4096)
    assert ok >= 0.999 * n


def test_slab_parity():
    """Bone/lung slab phantom, 25 spots from 70 to 230 MeV, 4e4 histories each."""
    ph = I.slab_phantom(128, 0.1)
    sp = W.slab_spots(40_000)
    db = W.multi_bin_db(2000)
    c = ctx_for(db)
    g = gpu_run(c, ph, sp)
    o = O.replay(db, ph, sp, seed=SEED)
    check_energy(g, o)
    check_dose(g, o, ph, int(sp["n_histories"].sum()))
    check_e2(g, o, ph, int(sp["n_histories"].sum()))
    tot = good = 0
    for s in range(25):
        ok, n = check_endpoints(c, g["plan"], db, ph, sp, s, 1000, 200)
        good += ok
        tot += n
    assert good >= 0.999 * tot


def test_thorax_subset_parity():
    """Synthetic thorax, 3 fields x 60 spots, 3000 histories each, rotation on."""
    ph = I.thorax_phantom((256, 256, 128), 0.2, seed=2188)
    sp_all = W.thorax_spots(total=6000 * 3000)
    sp = np.concatenate([sp_all[f * 2000:f * 2000 + 60] for f in range(3)])
    db = W.multi_bin_db(2000)
    c = ctx_for(db)
    flags = F.FDC_RUN_VARIANCE | F.FDC_RUN_ROTATE_TRACKS
    g = gpu_run(c, ph, sp, flags)
    o = O.replay(db, ph, sp, seed=SEED, flags=flags)
    check_energy(g, o)
    check_dose(g, o, ph, int(sp["n_histories"].sum()))
    tot = good = 0
    for s in range(0, 180, 6):
        ok, n = check_endpoints(c, g["plan"], db, ph, sp, s, 0, 128, flags)
        good += ok
        tot += n
    assert good >= 0.999 * tot


@pytest.mark.parametrize("R", [1, 320])
def test_reuse_factor_parity(R):
    ph = I.thorax_phantom((64, 64, 48), 0.4, seed=5)
    rng = np.random.default_rng(7)
    sp = I.field_spots((3.0, -1.0, 0.0), 90.0, 12, rng, histories=np.full(12, 777, np.uint64))
    db = W.multi_bin_db(2000)
    c = ctx_for(db, R=R)
    g = gpu_run(c, ph, sp)
    o = O.replay(db, ph, sp, seed=SEED, R=R)
    check_energy(g, o)
    check_dose(g, o, ph, 12 * 777)
    ok, n = check_endpoints(c, g["plan"], db, ph, sp, 3, 5, 300, R=R)
    assert ok >= 0.999 * n


def test_disk_field_anisotropic_voxels_parity():
    """The paper's kind of test field (Section 2.5): a mono-energetic field of
    circular cross-section on a thorax of anisotropic voxels (4 x 4 x 10 mm),
    against the oracle: energy identity, dose, and end points."""
    ph = I.thorax_phantom((80, 60, 30), (0.4, 0.4, 1.0), seed=5, scale=(0.8, 0.9, 1.0))
    db = W.water_db(600, 2188, 121.0)
    d = I.gantry_direction(0.0)
    sp = I.disk_field(np.array([5.0, -1.0, 0.0]) - 30.0 * d, d, 121.0, 2.5, 20_000)
    c = ctx_for(db)
    g = gpu_run(c, ph, sp)
    o = O.replay(db, ph, sp, seed=SEED)
    check_energy(g, o)
    check_dose(g, o, ph, 20_000)
    ok, n = check_endpoints(c, g["plan"], db, ph, sp, 0, 1000, 2000)
    assert ok >= 0.999 * n


# ------------------------------------------------------ order independence --
def _tallies(db, ph, sp, **cfg):
    c = ctx_for(db, **cfg)
    g = gpu_run(c, ph, sp)
    return g["E"], g["E2"], g["escaped"]


def test_launch_configs_bitwise():
    ph = I.thorax_phantom((96, 96, 64), 0.3, seed=11)
    rng = np.random.default_rng(1)
    sp = I.field_spots((3.0, -1.0, 0.0), 0.0, 40, rng, histories=np.full(40, 1500, np.uint64))
    db = W.multi_bin_db(2000)
    ref = _tallies(db, ph, sp)
    for cfg in [dict(waves_per_block=1), dict(waves_per_block=16), dict(waves_per_block=4, blocks_per_cu=2),
                dict(waves_per_block=8, blocks_per_cu=8),
                dict(waves_per_block=16, blocks_per_cu=1, tally_slots=4096),
                dict(waves_per_block=8, blocks_per_cu=2, tally_slots=1024, units_per_wave=3),
                dict(waves_per_block=4, blocks_per_cu=1, tally_slots=256, units_per_wave=1),
                # write-back cache: tiny tables force evictions and lanes racing on a word
                dict(waves_per_block=16, blocks_per_cu=1, tally_slots=256, units_per_wave=4, tally_mode=1),
                dict(waves_per_block=4, blocks_per_cu=2, tally_slots=320, units_per_wave=1, tally_mode=1),
                dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=2, tally_mode=1),
                # whole-launch cache (one plan), also tiny; chunks of 16, 8, 15 and 1 units
                dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=1, tally_mode=2),
                dict(waves_per_block=4, blocks_per_cu=2, tally_slots=256, units_per_wave=2, tally_mode=2),
                dict(waves_per_block=5, blocks_per_cu=1, tally_slots=512, units_per_wave=3, tally_mode=2),
                dict(waves_per_block=1, blocks_per_cu=4, tally_slots=256, units_per_wave=1, tally_mode=2),
                # histories in start-position order, every launch kind
                dict(waves_per_block=4, source_order=1), dict(waves_per_block=8, blocks_per_cu=2, source_order=1),
                dict(waves_per_block=8, blocks_per_cu=1, tally_slots=1024, units_per_wave=2, source_order=1),
                dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=1, tally_mode=1,
                     source_order=1),
                dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=1, tally_mode=2,
                     source_order=1)]:
        got = _tallies(db, ph, sp, **cfg)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]) and got[2] == ref[2], cfg


def test_autotuner_candidates_bitwise_and_tuning_leaves_no_trace(tmp_path):
    """Every configuration the autotuner may pick gives the same tallies, and a
    tuned run (candidates timed on the real plan, then rewound) equals an
    untuned one bitwise."""
    from paper_1011_2188_amd import autotune as A
    ph = I.thorax_phantom((72, 72, 48), 0.3, seed=12)
    rng = np.random.default_rng(3)
    sp = I.field_spots((2.0, -1.0, 0.0), 90.0, 30, rng, histories=np.full(30, 700, np.uint64))
    db = W.multi_bin_db(2000)
    ref = _tallies(db, ph, sp)
    for cfg in A.CANDIDATES:
        got = _tallies(db, ph, sp, **cfg)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]) and got[2] == ref[2], cfg
    c = ctx_for(db)
    p = c.load_phantom(ph)
    c.add_beam_spots(p, sp)
    best, timings = A.tune(c, [p], F.FDC_RUN_VARIANCE, reps=1, cache_path=str(tmp_path / "tune.json"))
    assert best in A.CANDIDATES and len(timings) == len(A.CANDIDATES)
    c.run_histories([p], F.FDC_RUN_VARIANCE)
    r = c.read_dose_and_variance(p, raw=True)
    assert np.array_equal(r["E"], ref[0]) and np.array_equal(r["E2"], ref[1]) and r["escaped"] == ref[2]
    assert r["n_histories"] == 30 * 700
    again, _ = A.tune(c, [p], F.FDC_RUN_VARIANCE, cache_path=str(tmp_path / "tune.json"))   # cache hit
    assert again == best


@pytest.mark.parametrize("cfg", [{}, dict(waves_per_block=8, blocks_per_cu=1, tally_slots=2048, units_per_wave=2),
                                 dict(waves_per_block=8, blocks_per_cu=1, tally_slots=512, units_per_wave=3,
                                      tally_mode=1),
                                 dict(waves_per_block=8, blocks_per_cu=1, tally_slots=512, tally_mode=2),
                                 dict(waves_per_block=8, blocks_per_cu=1, tally_slots=512, tally_mode=1,
                                      source_order=1)])
def test_split_runs_and_batching_bitwise(cfg):
    """run(n) twice == run(2n) (history counters continue, unaligned h0), and
    plans launched together == plans launched one by one (also with the LDS
    sub-tally, whose rounds then straddle the two plans)."""
    db = W.multi_bin_db(2000)
    ph1 = I.thorax_phantom((80, 80, 40), 0.3, seed=1)
    ph2 = I.slab_phantom(64, 0.2)
    rng = np.random.default_rng(2)
    sp1 = I.field_spots((2.0, 0.0, 0.0), 180.0, 9, rng, histories=np.full(9, 100, np.uint64))
    sp2 = W.slab_spots(150)[::3]
    c = ctx_for(db, **cfg)
    a1, a2 = c.load_phantom(ph1), c.load_phantom(ph2)
    c.add_beam_spots(a1, sp1)
    c.add_beam_spots(a2, sp2)
    c.run_histories([a1, a2])
    c.run_histories([a2, a1])
    ra1 = c.read_dose_and_variance(a1, raw=True)
    ra2 = c.read_dose_and_variance(a2, raw=True)
    c2 = ctx_for(db)
    b1 = c2.load_phantom(ph1)
    sp1b = sp1.copy()
    sp1b["n_histories"] = 200
    c2.add_beam_spots(b1, sp1b)
    c2.run_histories([b1])
    b2 = c2.load_phantom(ph2)
    sp2b = sp2.copy()
    sp2b["n_histories"] = 300
    c2.add_beam_spots(b2, sp2b)
    c2.run_histories([b2])
    rb1 = c2.read_dose_and_variance(b1, raw=True)
    rb2 = c2.read_dose_and_variance(b2, raw=True)
    assert np.array_equal(ra1["E"], rb1["E"]) and np.array_equal(ra1["E2"], rb1["E2"])
    assert np.array_equal(ra2["E"], rb2["E"]) and np.array_equal(ra2["E2"], rb2["E2"])
    o = O.replay(db, ph1, sp1b, seed=SEED, plan=0)
    assert ra1["incident"] == o["incident"]


# ------------------------------------------------------------ edge cases ----
def test_edge_cases():
    db = W.multi_bin_db(2000)
    ph = I.water_phantom((20, 20, 20), 0.5)
    c = ctx_for(db)
    p = c.load_phantom(ph)
    # a spot aimed away from the box: every history misses, all energy escapes
    c.add_beam_spots(p, I.spots([[0, 0, -2.0]], [[0, 0, -1.0]], [150.0], 0.3, 65))
    c.run_histories([p])
    r = c.read_dose_and_variance(p, raw=True)
    assert r["E"].sum() == 0 and r["escaped"] == r["incident"] > 0
    _, why = c.debug_endpoints(p, 0, 0, 65)
    assert np.all(why == 2)
    # a run with no histories is a no-op; reading a plan that never ran is an error
    q = c.load_phantom(ph)
    c.add_beam_spots(q, I.spots([[0, 0, -1.0]], [[0, 0, 1.0]], [100.0], 0.3, 0))
    c.run_histories([q])
    with pytest.raises(F.FdcError):
        c.read_dose_and_variance(q)
    # ragged history counts and spot energies exactly on / between bins
    for n in (1, 63, 64, 65, 129):
        sp = I.spots([[0.3, 0, -1.0], [0, 0.2, -1.0]], [[0, 0, 1.0], [0, 0, 1.0]], [70.0, 71.3], 0.4, n)
        pl = c.load_phantom(ph)
        c.add_beam_spots(pl, sp)
        c.run_histories([pl])
        g = c.read_dose_and_variance(pl, raw=True)
        o = O.replay(db, ph, sp, seed=SEED, plan=pl)
        assert g["incident"] == o["incident"] and g["deposited"] + g["escaped"] == g["incident"]
        assert np.abs(g["E"] - o["E"]).sum() <= 1e-5 * o["incident"]


# ------------------------------------------------------ full-size checks ----
# the configuration the benchmark's autotuner picks for the slab workload
BENCH_LAUNCH = dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=1, tally_mode=2,
                    source_order=1)


def test_full_size_slab_dose_vs_oracle():
    """The 1e7-history slab workload in the benchmark's launch configuration
    (whole-launch LDS cache, start-position order): dose and Eq. (2) variance against the oracle run
    on the same 1e7 histories, energy identity exactly, incident energy equal
    to the oracle's, the tallies bitwise equal to the plain global-atomic
    launch, and sampled end points."""
    ph, sp, db = W.slab()
    c = ctx_for(db, **BENCH_LAUNCH)
    g = gpu_run(c, ph, sp)
    assert g["n_histories"] == 10_000_000
    assert g["deposited"] + g["escaped"] == g["incident"]
    ref = gpu_run(ctx_for(db, waves_per_block=4), ph, sp)
    assert np.array_equal(g["E"], ref["E"]) and np.array_equal(g["E2"], ref["E2"])
    o = O.replay(db, ph, sp, seed=SEED)
    assert g["incident"] == o["incident"]
    dose_o, var_o = check_dose(g, o, ph, 10_000_000)
    check_e2(g, o, ph, 10_000_000)
    sel = dose_o > 0.5 * dose_o.max()
    rel = np.abs(np.sqrt(g["var"][sel]) - np.sqrt(var_o[sel])) / np.sqrt(var_o[sel])
    assert np.median(rel) < 0.01
    tot = good = 0
    for s in range(0, 25, 2):
        ok, n = check_endpoints(c, g["plan"], db, ph, sp, s, 400_000 - 96, 96)
        good += ok
        tot += n
    assert good >= 0.999 * tot


def test_full_size_thorax_sampled():
    """The 1e8-history thorax workload in the benchmark's launch configuration:
    tallies bitwise equal to the global-atomic launch, energy identity, and
    sampled end points (with track rotation off, as the workload runs)."""
    ph, sp, db = W.thorax()
    c = ctx_for(db, **BENCH_LAUNCH)
    g = gpu_run(c, ph, sp)
    assert g["n_histories"] == int(sp["n_histories"].sum())
    assert g["deposited"] + g["escaped"] == g["incident"]
    ref = gpu_run(ctx_for(db, waves_per_block=4, blocks_per_cu=4), ph, sp)
    assert np.array_equal(g["E"], ref["E"]) and np.array_equal(g["E2"], ref["E2"])
    tot = good = 0
    for s in range(0, len(sp), 500):
        n0 = int(sp["n_histories"][s])
        ok, n = check_endpoints(c, g["plan"], db, ph, sp, s, n0 - 64, 64)
        good += ok
        tot += n
    assert good >= 0.999 * tot


def test_full_size_paper_field_sampled():
    """The paper-field workload at full size (6.08e6 voxels of 1 x 1 x 2.5 mm,
    121 MeV disk of 4 cm radius, 1e7 histories) in the benchmark's launch
    configuration: tallies bitwise equal to the global-atomic launch, energy
    identity, and sampled end points against the oracle."""
    ph, sp, db = W.paper_field()
    c = ctx_for(db, **BENCH_LAUNCH)
    g = gpu_run(c, ph, sp)
    assert g["n_histories"] == int(sp["n_histories"].sum())
    assert g["deposited"] + g["escaped"] == g["incident"]
    ref = gpu_run(ctx_for(db, waves_per_block=4, blocks_per_cu=4), ph, sp)
    assert np.array_equal(g["E"], ref["E"]) and np.array_equal(g["E2"], ref["E2"])
    tot = good = 0
    for h0 in (0, 4_000_000, 9_999_000):
        ok, n = check_endpoints(c, g["plan"], db, ph, sp, 0, h0, 1000)
        good += ok
        tot += n
    assert good >= 0.999 * tot


def test_batched_graph_full_size():
    """The 64-plan batched workload (1.6e8 histories) as one captured graph
    launch in the benchmark's launch configuration equals separate eager runs
    of each plan with global atomics, plan by plan, bitwise; every plan keeps
    the energy identity."""
    plans = W.batched_plans(64)
    db = W.multi_bin_db()
    cg = ctx_for(db, **BENCH_LAUNCH)
    ce = ctx_for(db, waves_per_block=4)
    ig, ie = [], []
    for ph, sp in plans:
        for c, ids in ((cg, ig), (ce, ie)):
            p = c.load_phantom(ph)
            c.add_beam_spots(p, sp)
            ids.append(p)
    gr = cg.graph_create(ig, F.FDC_RUN_VARIANCE, reset=True)
    gr.launch()
    torch.cuda.synchronize()
    for p in ie:
        ce.run_histories([p], F.FDC_RUN_VARIANCE)
    for a, b, (ph, sp) in zip(ig, ie, plans):
        ra = cg.read_dose_and_variance(a, dose=False, var=False, raw=True)
        rb = ce.read_dose_and_variance(b, dose=False, var=False, raw=True)
        assert ra["n_histories"] == rb["n_histories"] == int(sp["n_histories"].sum())
        assert ra["deposited"] + ra["escaped"] == ra["incident"] == rb["incident"]
        assert np.array_equal(ra["E"], rb["E"]) and np.array_equal(ra["E2"], rb["E2"])
    gr.close()


def test_batched_graph_plans_vs_oracle():
    """Four plans of the batched workload's generator (thorax-like phantoms of
    different sizes, one field each), 1e5 histories each, run as ONE captured
    graph launch in the benchmark's launch configuration (tallies cleared, dose
    and variance computed inside the graph): every plan's dose against the
    oracle replaying that plan, its squared-energy tally, its incident energy
    exactly, and the energy identity."""
    plans = W.batched_plans(4, seed=77, hist_scale=1.0)
    db = W.multi_bin_db(2000)
    c = ctx_for(db, **BENCH_LAUNCH)
    ids, doses, vars_ = [], [], []
    for ph, sp in plans:
        sp = sp.copy()
        base, extra = divmod(100_000, len(sp))
        sp["n_histories"] = base
        sp["n_histories"][:extra] += 1
        p = c.load_phantom(ph)
        c.add_beam_spots(p, sp)
        ids.append((p, ph, sp))
        doses.append(torch.empty(ph.hu.size, dtype=torch.float64, device="cuda"))
        vars_.append(torch.empty(ph.hu.size, dtype=torch.float64, device="cuda"))
    gr = c.graph_create([p for p, _, _ in ids], F.FDC_RUN_VARIANCE, reset=True, doses=doses, variances=vars_)
    gr.launch()
    torch.cuda.synchronize()
    for (p, ph, sp), d, v in zip(ids, doses, vars_):
        g = c.read_dose_and_variance(p, dose=False, var=False, raw=True)
        g["dose"] = d.cpu().numpy().reshape(ph.hu.shape)
        o = O.replay(db, ph, sp, seed=SEED, plan=p)
        assert g["n_histories"] == 100_000
        check_energy(g, o)
        dose_o, var_o = check_dose(g, o, ph, 100_000)
        check_e2(g, o, ph, 100_000)
        sel = dose_o > 0.5 * dose_o.max()
        ug = np.mean(np.sqrt(v.cpu().numpy().reshape(ph.hu.shape)[sel]) / dose_o[sel])
        uo = np.mean(np.sqrt(var_o[sel]) / dose_o[sel])
        assert abs(ug / uo - 1) < 0.01
    gr.close()


# ---------------------------------------------------------------- graphs ----
@pytest.mark.parametrize("cfg", [{}, dict(waves_per_block=16, blocks_per_cu=1, tally_slots=4096, units_per_wave=2),
                                 dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=2,
                                      tally_mode=1),
                                 dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, tally_mode=2),
                                 dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, tally_mode=1,
                                      source_order=1)])
def test_graph_replays_match_eager(cfg):
    """A captured run (clear tallies -> transport -> advance counters -> dose)
    replayed four times, with eager work and synchronisation in between,
    equals four eager passes bitwise, replay by replay."""
    db = W.multi_bin_db(2000)
    ph = I.thorax_phantom((64, 56, 40), 0.3, seed=21)
    rng = np.random.default_rng(4)
    sp = I.field_spots((2.0, -1.0, 0.0), 180.0, 15, rng, histories=np.full(15, 1000, np.uint64))
    n = ph.hu.size
    ce = ctx_for(db, **cfg)
    pe = ce.load_phantom(ph)
    ce.add_beam_spots(pe, sp)
    de = torch.empty(n, dtype=torch.float64, device="cuda")
    ve = torch.empty(n, dtype=torch.float64, device="cuda")
    eager = []
    for _ in range(4):
        ce.reset_plan(pe)
        ce.run_histories([pe], F.FDC_RUN_VARIANCE)
        ce.compute_dose(pe, de, ve)
        r = ce.read_dose_and_variance(pe, dose=False, var=False, raw=True)
        eager.append((r["E"], r["E2"], de.cpu().numpy(), ve.cpu().numpy(), r["incident"]))
    cg = ctx_for(db, **cfg)
    pg = cg.load_phantom(ph)
    cg.add_beam_spots(pg, sp)
    dg = torch.empty(n, dtype=torch.float64, device="cuda")
    vg = torch.empty(n, dtype=torch.float64, device="cuda")
    g = cg.graph_create([pg], F.FDC_RUN_VARIANCE, reset=True, doses=[dg], variances=[vg])
    for k in range(4):
        g.launch()
        torch.cuda.synchronize()
        cg.debug_philox(np.arange(64, dtype=np.uint32).reshape(16, 4))     # eager work in between
        r = cg.read_dose_and_variance(pg, dose=False, var=False, raw=True)
        E, E2, d, v, inc = eager[k]
        assert np.array_equal(r["E"], E) and np.array_equal(r["E2"], E2), k
        assert r["incident"] == inc and r["n_histories"] == 15000
        assert np.array_equal(dg.cpu().numpy(), d) and np.array_equal(vg.cpu().numpy(), v), k
    g.close()
