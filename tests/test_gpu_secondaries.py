"""Secondary trajectories (Section 2.2: a stored history is the set of its
particles' trajectories) on the GPU against the oracle, through the C ABI.

A thorax-like phantom, a generated database with secondaries at four times
the default interaction rate (so that a good share of histories carry them),
spots at their bin energies and below (skips that end inside a secondary's
energy), one spot through a range compensator (secondaries emitted inside it
stay there).  Same criteria as the other parity tests: incident energy exact,
deposited + escaped = incident exactly, dose within 0.5% of Dmax above 10% of
Dmax, squared-energy tally likewise, 99.9% of sampled primary end points within
1e-4 cm with the same end reason, tallies bitwise equal across launch
configurations; and a hand-built straight track whose depth and lateral
profiles the oracle pins in closed form."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from paper_1011_2188_amd import fdc as F  # noqa: E402
from paper_1011_2188_amd import inputs as I  # noqa: E402

LAUNCHES = [
    dict(waves_per_block=4, blocks_per_cu=0, tally_slots=0, units_per_wave=0, tally_mode=0, source_order=0),
    dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=2, tally_mode=2, source_order=1),
    dict(waves_per_block=16, blocks_per_cu=1, tally_slots=4096, units_per_wave=1, tally_mode=1, source_order=0),
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    torch.cuda.init()


def _case():
    db = I.make_water_track_db([100.0, 105.0, 110.0, 115.0], 300, seed=23, secondaries=True,
                               nuc_per_cm=4 * I.NUC_PER_CM)
    ph = I.thorax_phantom((64, 56, 40), 0.3, seed=19, scale=(64 * 0.3 / 51.2, 56 * 0.3 / 51.2, 40 * 0.3 / 25.6))
    d1 = np.array([0.0, 1.0, 0.0])
    d2 = np.array([1.0, 0.0, 0.0])
    sp = I.spots([[0.5, -20.0, 0.3], [-0.8, -20.0, -0.4], [-20.0, 0.2, 0.0], [-20.0, -1.0, 0.5]],
                 [d1, d1, d2, d2], [105.0, 107.5, 110.0, 111.3], [0.5, 0.4, 0.4, 0.6], 4000)
    dev = I.aperture_compensator([0.0, -12.0, 0.0], d1, 3.0, ramp_cm=(1.5, 3.5), pitch_cm=0.05)
    return db, ph, sp, ([dev], [0, -1, -1, -1])


def _gpu_run(db, ph, sp, devices, launch, flags=F.FDC_RUN_VARIANCE):
    c = F.Context(0, 1, table=I.HU_TABLE_DEFAULT)
    c.load_track_db(db)
    c.set_launch_config(**launch)
    p = c.load_phantom(ph)
    c.add_beam_spots(p, sp)
    for dev in devices[0]:
        c.add_beam_device(dev)
    for s, dv in enumerate(devices[1]):
        if dv >= 0:
            c.set_spot_device(p, s, 1, dv)
    c.run_histories([p], flags)
    return c, p, c.read_dose_and_variance(p, raw=True)


def test_secondaries_match_the_oracle():
    db, ph, sp, devices = _case()
    assert db.sec.n > 0.3 * db.n_tracks
    o = O.replay(db, ph, sp, devices=devices)
    c, p, g = _gpu_run(db, ph, sp, devices, LAUNCHES[1])
    try:
        assert g["incident"] == o["incident"]
        assert g["deposited"] + g["escaped"] == g["incident"]
        assert int(g["E"].sum()) == g["deposited"]
        n = int(sp["n_histories"].sum())
        dose_o, _ = O.dose_and_variance(o["E"], o["E2"], n, ph)
        dmax = dose_o.max()
        sel = dose_o > 0.1 * dmax
        assert np.abs(g["dose"] - dose_o)[sel].max() <= 0.005 * dmax
        e2g, e2o = g["E2"].astype(np.float64), o["E2"].astype(np.float64)
        assert np.abs(e2g - e2o)[sel].max() <= 0.005 * e2o[sel].max()
        assert abs(g["escaped"] - o["escaped"]) <= 1e-3 * o["incident"]
        ok = total = 0
        for spot in range(len(sp)):
            xg, rg = c.debug_endpoints(p, spot, 0, 2000)
            xo, ro = O.endpoints(db, ph, sp, spot, 0, 2000, devices=devices)
            close = np.linalg.norm(xg.astype(np.float64) - xo, axis=1) <= 1e-4
            ok += int(((rg == ro) & close).sum())
            total += 2000
        assert ok >= 0.999 * total, f"{total - ok} of {total} end points differ"
    finally:
        c.close()


def test_secondaries_bitwise_across_launch_configurations():
    db, ph, sp, devices = _case()
    runs = []
    for launch in LAUNCHES:
        c, p, g = _gpu_run(db, ph, sp, devices, launch)
        runs.append(g)
        c.close()
    for g in runs[1:]:
        assert np.array_equal(g["E"], runs[0]["E"]) and np.array_equal(g["E2"], runs[0]["E2"])
        assert g["escaped"] == runs[0]["escaped"] and g["incident"] == runs[0]["incident"]


def test_secondaries_add_to_unchanged_primaries():
    """The same primaries with and without their secondaries, spots at the bin
    energies: the secondaries add energy to the tallies and the incident
    energy, and the primaries' end points do not move."""
    db, ph, sp, _ = _case()
    sp = sp.copy()
    sp["energy_MeV"] = [105.0, 105.0, 110.0, 115.0]
    prim = I.TrackDB(db.steps, db.track_off, db.bin_E, db.bin_first, None)
    c1, p1, a = _gpu_run(db, ph, sp, ([], []), LAUNCHES[1])
    c2, p2, b = _gpu_run(prim, ph, sp, ([], []), LAUNCHES[1])
    try:
        assert a["incident"] > b["incident"] and a["deposited"] > b["deposited"]
        for spot in range(len(sp)):
            xa, ra = c1.debug_endpoints(p1, spot, 0, 1000)
            xb, rb = c2.debug_endpoints(p2, spot, 0, 1000)
            assert (ra == rb).mean() >= 0.999
            assert np.mean(np.linalg.norm(xa - xb, axis=1) <= 1e-5) >= 0.999
    finally:
        c1.close()
        c2.close()


def test_straight_track_profiles():
    """A hand-built track (straight steps, one deflection) with two secondaries
    in water: the GPU's depth and lateral profiles equal the oracle's (pinned
    in closed form) up to FP32 rounding of the crossing points, at the bin
    energy and with a skip that ends inside the first secondary."""
    prim = [(0.23, 2.0 + 0.1 * k) for k in range(30)]
    secs = [(4, 0.0, 0.0, [(0.21, 1.5 + 0.05 * k) for k in range(12)]),
            (11, 0.35, 0.0, [(0.19, 1.2 + 0.03 * k) for k in range(10)])]
    st = np.array([[dx, de, 0.0, 0.0] for dx, de in prim], np.float32)
    st[4, 2] = 0.3
    steps = np.array([[dx, de, 0.0, 0.0] for s in secs for dx, de in s[3]], np.float32)
    e_bin = np.float32(sum(de for _, de in prim) + sum(de for s in secs for _, de in s[3]))
    # the track twice in the top bin (the chunk's draw picks either), and a
    # low bin of one short track so that the lower spot energy lies inside the
    # database's range (it still uses the top bin: the smallest one >= it)
    low = np.array([[0.2, 2.0, 0.0, 0.0]] * 5, np.float32)
    st3 = np.concatenate([low, st, st])
    sec = I.Secondaries(np.array([0, 0, 2, 4], np.uint32), np.array([0, 12, 22, 34, 44], np.uint64),
                        np.concatenate([steps, steps]), np.array([4, 11, 4, 11], np.uint32),
                        np.array([[0.0, 0.0], [0.35, 0.0]] * 2, np.float32))
    db = I.TrackDB(st3, np.array([0, 5, 35, 65], np.uint64), np.array([10.0, e_bin], np.float32),
                   np.array([0, 1, 3], np.uint32), sec)
    ph = I.water_phantom((64, 64, 64), 0.25, origin=(-8.0, -8.0, 0.0))
    p4 = sum(int(np.rint(np.float32(de) * 2.0 ** 24)) for _, de in prim[:5])
    s1 = sum(int(np.rint(np.float32(de) * 2.0 ** 24)) for _, de in secs[0][3])
    e_low = np.float32(float(e_bin) - (p4 + 0.5 * s1) / 2.0 ** 24)
    sp = I.spots([[0.125, 0.125, -2.0]] * 2, [[0.0, 0.0, 1.0]] * 2, [e_bin, e_low], 0.0, 256)
    o = O.replay(db, ph, sp)
    c, p, g = _gpu_run(db, ph, sp, ([], []), LAUNCHES[1])
    c.close()
    assert g["incident"] == o["incident"] and g["deposited"] + g["escaped"] == g["incident"]
    for ax in ((1, 2), (0, 1), (0, 2)):
        a, b = g["E"].sum(axis=ax).astype(np.float64), o["E"].sum(axis=ax).astype(np.float64)
        assert np.abs(a - b).max() <= 1e-5 * b.max(), ax


def test_secondaries_from_a_database_file(tmp_path):
    """The same database through the version-2 file: bit-identical tallies,
    and the allocation-free run gives them too."""
    db, ph, sp, devices = _case()
    path = tmp_path / "db2.bin"
    I.write_track_db_file(path, db)
    c1, p1, a = _gpu_run(db, ph, sp, devices, LAUNCHES[1])
    c1.close()
    c = F.Context(0, 1, table=I.HU_TABLE_DEFAULT)
    try:
        c.load_track_db_file(path)
        c.set_launch_config(**LAUNCHES[1])
        p = c.load_phantom(ph)
        c.add_beam_spots(p, sp)
        c.add_beam_device(devices[0][0])
        c.set_spot_device(p, 0, 1, 0)
        c.prepare_run()                       # device tables in place, so the run allocates nothing
        c.run_histories_noalloc([p], F.FDC_RUN_VARIANCE)
        b = c.read_dose_and_variance(p, raw=True)
        assert np.array_equal(a["E"], b["E"]) and np.array_equal(a["E2"], b["E2"])
        assert a["incident"] == b["incident"] and a["escaped"] == b["escaped"]
    finally:
        c.close()


def test_secondaries_with_a_phase_space():
    """Listed protons (a phase space, each with its own start, direction,
    energy and frame) on a database with secondaries, against the oracle."""
    db, ph, _, _ = _case()
    q = I.synthetic_phase_space(6000, 5, e_mean=107.5, e_sigma=2.0, tail_fraction=0.1, tail_min=101.0,
                                radius_cm=1.5, source_cm=(0.0, -20.0, 0.0), direction=(0.0, 1.0, 0.0))
    c = F.Context(0, 1, table=I.HU_TABLE_DEFAULT)
    try:
        c.load_track_db(db)
        c.set_launch_config(**LAUNCHES[1])
        p = c.load_phantom(ph)
        n_src = c.add_phase_space(p, q)
        c.run_histories([p], F.FDC_RUN_VARIANCE)
        g = c.read_dose_and_variance(p, raw=True)
        ps = O.phase_space_sources(q["pos_cm"], q["dir"], q["energy_MeV"], db.bin_E, 0)
        rows = np.zeros(len(ps["count"]), I.SPOT_DTYPE)
        rows["dir"] = (0.0, 0.0, 1.0)
        rows["energy_MeV"] = db.bin_E[-1]
        assert n_src == len(ps["count"]) >= 2
        o = O.replay(db, ph, rows, h_count=ps["count"], phase_space=ps)
        assert g["incident"] == o["incident"] and g["deposited"] + g["escaped"] == g["incident"]
        dose_o, _ = O.dose_and_variance(o["E"], o["E2"], q.size, ph)
        dmax = dose_o.max()
        sel = dose_o > 0.1 * dmax
        assert np.abs(g["dose"] - dose_o)[sel].max() <= 0.005 * dmax
    finally:
        c.close()


def test_secondaries_in_a_captured_graph():
    """A captured run (tallies cleared, transport, counters advanced) replayed
    three times with eager work between the replays: each replay equals the
    eager run of the same histories bit for bit."""
    db, ph, sp, devices = _case()
    c = F.Context(0, 1, table=I.HU_TABLE_DEFAULT)
    e = F.Context(0, 1, table=I.HU_TABLE_DEFAULT)
    try:
        for x in (c, e):
            x.load_track_db(db)
            x.set_launch_config(**LAUNCHES[1])
        p = c.load_phantom(ph)
        c.add_beam_spots(p, sp)
        q = e.load_phantom(ph)
        e.add_beam_spots(q, sp)
        gr = c.graph_create([p], F.FDC_RUN_VARIANCE)
        for rep in range(3):
            gr.launch()
            torch.cuda.synchronize()
            a = c.read_dose_and_variance(p, raw=True)
            e.reset_plan(q)
            e.run_histories([q], F.FDC_RUN_VARIANCE)
            b = e.read_dose_and_variance(q, raw=True)
            assert np.array_equal(a["E"], b["E"]) and np.array_equal(a["E2"], b["E2"]), rep
            assert a["incident"] == b["incident"] and a["escaped"] == b["escaped"]
        gr.close()
    finally:
        c.close()
        e.close()
