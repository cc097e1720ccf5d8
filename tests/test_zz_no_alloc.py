"""The allocation-free run, fdc_run_histories_noalloc, against fdc_run_histories
through the C ABI: two calls in a row (two plans in one launch, then a smaller
plan), in three launch configurations, give bit-identical integer tallies and
summaries; the noalloc calls make no allocation through the context's
allocator hook; the second call also matches the oracle voxel by voxel; sizes
beyond the static scratch and stale device tables are refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from paper_1011_2188_amd import fdc as F  # noqa: E402
from paper_1011_2188_amd import inputs as I  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    torch.cuda.init()


class _CountingAllocator:
    """torch-backed device memory that counts the calls."""

    def __init__(self):
        self.calls = 0
        self.live = {}
        self.fa = F.ALLOC_FN(self._alloc)
        self.ff = F.FREE_FN(self._free)

    def _alloc(self, n, user):
        self.calls += 1
        t = torch.empty(int(n), dtype=torch.uint8, device="cuda")
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, p, user):
        self.live.pop(p, None)


DB = dict(bins=[95.0, 100.0, 105.0, 110.0], tracks=300, seed=5)

# (waves_per_block, blocks_per_cu, tally_slots, units_per_wave, tally_mode, source_order)
LAUNCHES = [
    (4, 0, 0, 0, 0, 0),          # one workgroup per unit, global atomics, history order
    (16, 1, 4096, 2, 1, 0),      # persistent rounds with the LDS cache, history order
    (16, 1, 8064, 1, 2, 1),      # whole-launch LDS cache, start-position order
]


def _first_call_inputs():
    ph_a = I.thorax_phantom((64, 48, 40), 0.3, seed=11)
    ph_b = I.thorax_phantom((40, 56, 32), 0.35, seed=12)
    sp_a = I.spots([[0.3, -0.2, -20.0], [-0.5, 0.4, 20.0], [1.0, 0.0, -20.0]], [[0, 0, 1.0], [0, 0, -1.0], [0, 0, 1.0]],
                   [97.5, 110.0, 102.0], 0.4, 7000)
    sp_a["n_histories"][2] = 70_000       # more than four ordering chunks: the whole-spot histogram order
    sp_b = I.spots([[0.0, -20.0, 0.5], [20.0, 0.0, -0.5]], [[0, 1.0, 0], [-1.0, 0, 0]], [100.0, 108.5], 0.3, 5001)
    return (ph_a, sp_a), (ph_b, sp_b)


def _second_call_inputs():
    ph = I.thorax_phantom((24, 20, 16), 0.5, seed=13)
    sp = I.spots([[0.2, 0.1, -20.0]], [[0, 0, 1.0]], [96.0], 0.3, 1500)
    return ph, sp


def _setup(ctx, launch, db, inputs):
    ctx.set_launch_config(**dict(zip(("waves_per_block", "blocks_per_cu", "tally_slots", "units_per_wave",
                                      "tally_mode", "source_order"), launch)))
    plans = []
    for ph, sp in inputs:
        p = ctx.load_phantom(ph)
        ctx.add_beam_spots(p, sp)
        plans.append(p)
    return plans


def _same(ga, gb):
    assert np.array_equal(ga["E"], gb["E"]) and np.array_equal(ga["E2"], gb["E2"])
    for k in ("n_histories", "incident", "deposited", "escaped"):
        assert ga[k] == gb[k], k
    assert ga["deposited"] + ga["escaped"] == ga["incident"]


@pytest.mark.parametrize("launch", LAUNCHES)
def test_noalloc_matches_run_two_calls(launch):
    db = I.make_water_track_db(DB["bins"], DB["tracks"], seed=DB["seed"])
    al = _CountingAllocator()
    ref = F.Context(0, 1, table=I.HU_TABLE_DEFAULT)
    nal = F.Context(0, 1)
    try:
        F._check(nal.h, F.lib().fdc_set_allocator(nal.h, al.fa, al.ff, None))
        nal.set_hu_table(I.HU_TABLE_DEFAULT)
        for c in (ref, nal):
            c.load_track_db(db)
        first = _first_call_inputs()
        pr = _setup(ref, launch, db, first)
        pn = _setup(nal, launch, db, first)
        with pytest.raises(F.FdcError) as e:          # tables not yet on the device
            nal.run_histories_noalloc(pn, F.FDC_RUN_VARIANCE)
        assert e.value.code == F.FDC_E_STATE
        nal.prepare_run()
        calls = al.calls
        print(f"noalloc first call, launch {launch}", flush=True)
        ref.run_histories(pr, F.FDC_RUN_VARIANCE)
        nal.run_histories_noalloc(pn, F.FDC_RUN_VARIANCE)
        torch.cuda.synchronize()
        assert al.calls == calls                      # nothing allocated
        for a, b in zip(pr, pn):
            _same(ref.read_dose_and_variance(a, raw=True), nal.read_dose_and_variance(b, raw=True))

        # second call: a smaller plan (the scratch still holds the first call's table)
        ph, sp = _second_call_inputs()
        (qr,) = _setup(ref, launch, db, [(ph, sp)])
        (qn,) = _setup(nal, launch, db, [(ph, sp)])
        nal.prepare_run()
        calls = al.calls
        print(f"noalloc second call, launch {launch}", flush=True)
        ref.run_histories([qr], F.FDC_RUN_VARIANCE)
        nal.run_histories_noalloc([qn], F.FDC_RUN_VARIANCE)
        torch.cuda.synchronize()
        assert al.calls == calls
        gr = ref.read_dose_and_variance(qr, raw=True)
        gn = nal.read_dose_and_variance(qn, raw=True)
        _same(gr, gn)
        # and the oracle on the same histories (plan id as in the contexts)
        o = O.replay(db, ph, sp, seed=1, plan=qn)
        assert gn["incident"] == o["incident"]
        dose_o, _ = O.dose_and_variance(o["E"], o["E2"], int(sp["n_histories"].sum()), ph)
        dmax = dose_o.max()
        sel = dose_o > 0.1 * dmax
        assert np.abs(gn["dose"] - dose_o)[sel].max() <= 0.005 * dmax
    finally:
        ref.close()
        nal.close()


def test_noalloc_refuses_what_the_scratch_cannot_hold():
    db = I.make_water_track_db(DB["bins"], DB["tracks"], seed=DB["seed"])
    with F.Context(0, 1, table=I.HU_TABLE_DEFAULT) as c:
        c.load_track_db(db)
        ph = I.thorax_phantom((24, 20, 16), 0.5, seed=13)
        # start-position order of 9e6 histories: more wave units than the lane table holds
        c.set_launch_config(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=1, tally_mode=2,
                            source_order=1)
        p = c.load_phantom(ph)
        c.add_beam_spots(p, I.spots([[0.0, 0.0, -20.0]], [[0, 0, 1.0]], [100.0], 0.3, 9_000_000))
        c.prepare_run()
        with pytest.raises(F.FdcError) as e:
            c.run_histories_noalloc([p], F.FDC_RUN_VARIANCE)
        assert e.value.code == F.FDC_E_RANGE
        # more spots with histories than the work table holds
        q = c.load_phantom(ph)
        c.add_beam_spots(q, I.spots(np.tile([[0.0, 0.0, -20.0]], (16385, 1)), np.tile([[0, 0, 1.0]], (16385, 1)),
                                    np.full(16385, 100.0), 0.3, 1))
        c.prepare_run()
        with pytest.raises(F.FdcError) as e:
            c.run_histories_noalloc([q], F.FDC_RUN_VARIANCE)
        assert e.value.code == F.FDC_E_RANGE
        assert c.read_dose_and_variance(p, dose=False, var=False)["n_histories"] == 0   # nothing ran
