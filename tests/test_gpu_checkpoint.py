"""Checkpoint and resume through the C ABI: a plan run for N histories per
source, saved, restored into a fresh context (same database, seed, phantom and
sources) and run again for N equals the plan run for 2N in one context, bit for
bit (tallies, summary, next histories), with and without the squared-energy
tally; restoring into the same context rewinds it to the checkpoint."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1011_2188_amd import fdc as F  # noqa: E402
from paper_1011_2188_amd import inputs as I  # noqa: E402

LAUNCH = dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=2, tally_mode=2, source_order=1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


def _ctx(db, ph, sp):
    c = F.Context(0, 7, table=I.HU_TABLE_DEFAULT)
    c.load_track_db(db)
    c.set_launch_config(**LAUNCH)
    p = c.load_phantom(ph)
    c.add_beam_spots(p, sp)
    return c, p


def test_resume_equals_an_uninterrupted_run():
    db = I.make_water_track_db([100.0, 110.0, 120.0], 200, seed=3)
    ph = I.thorax_phantom((64, 56, 40), 0.3, seed=11, scale=(64 * 0.3 / 51.2, 56 * 0.3 / 51.2, 40 * 0.3 / 25.6))
    sp = I.spots([[0.5, -20.0, 0.3], [-20.0, 0.2, 0.0]], [[0.0, 1.0, 0.0], [1.0, 0.0, 0.0]], [105.0, 117.0],
                 [0.5, 0.4], [3000, 1777])
    a, pa = _ctx(db, ph, sp)
    b, pb = _ctx(db, ph, sp)
    try:
        a.run_histories([pa], F.FDC_RUN_VARIANCE)
        a.run_histories([pa], F.FDC_RUN_VARIANCE)
        full = a.read_dose_and_variance(pa, raw=True)
        b.run_histories([pb], F.FDC_RUN_VARIANCE)
        state = b.save_plan_state(pb)
        b.close()
        c, pc = _ctx(db, ph, sp)
        c.restore_plan_state(pc, state)
        c.run_histories([pc], F.FDC_RUN_VARIANCE)
        res = c.read_dose_and_variance(pc, raw=True)
        assert np.array_equal(res["E"], full["E"]) and np.array_equal(res["E2"], full["E2"])
        for k in ("incident", "escaped", "deposited", "n_histories"):
            assert res[k] == full[k], k
        assert c.save_plan_state(pc) == a.save_plan_state(pa)
        # the same context, back to the checkpoint: the second half again
        c.restore_plan_state(pc, state)
        c.run_histories([pc], F.FDC_RUN_VARIANCE)
        again = c.read_dose_and_variance(pc, raw=True)
        assert np.array_equal(again["E"], full["E"]) and again["incident"] == full["incident"]
        c.close()
    finally:
        a.close()
