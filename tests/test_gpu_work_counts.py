"""The device's work counters (FDC_RUN_COUNT_WORK: steps started in the
phantom, non-vacuum voxel pieces, deposits flushed) against the oracle's counts
of the same histories, through the C ABI, on a thorax-like phantom with track
rotation and on a database with secondary trajectories: within 0.1% (FP32
against FP64 positions can move a rare crossing).  The counting run's tallies
are bitwise those of the benchmark's launch configuration, and a reset clears
the counters."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from paper_1011_2188_amd import fdc as F  # noqa: E402
from paper_1011_2188_amd import inputs as I  # noqa: E402

CACHE = dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=2, tally_mode=2, source_order=1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    torch.cuda.init()


def _case(secondaries):
    db = I.make_water_track_db([100.0, 110.0, 120.0, 130.0], 250, seed=41, secondaries=secondaries,
                               nuc_per_cm=4 * I.NUC_PER_CM)
    ph = I.thorax_phantom((64, 56, 40), 0.3, seed=5, scale=(64 * 0.3 / 51.2, 56 * 0.3 / 51.2, 40 * 0.3 / 25.6))
    sp = I.spots([[0.5, -20.0, 0.3], [-20.0, 0.2, 0.0], [0.0, 20.0, -1.0]],
                 [[0.0, 1.0, 0.0], [1.0, 0.0, 0.0], [0.0, -1.0, 0.0]], [105.0, 118.0, 127.5], [0.5, 0.4, 0.6], 3000)
    return db, ph, sp


@pytest.mark.parametrize("secondaries", [False, True])
def test_work_counts_match_the_oracle(secondaries):
    db, ph, sp = _case(secondaries)
    flags = F.FDC_RUN_VARIANCE | F.FDC_RUN_ROTATE_TRACKS
    o = O.replay(db, ph, sp, flags=O.FLAG_VARIANCE | O.FLAG_ROTATE)
    c = F.Context(0, 1, table=I.HU_TABLE_DEFAULT)
    try:
        c.load_track_db(db)
        c.set_launch_config(**CACHE)
        p = c.load_phantom(ph)
        c.add_beam_spots(p, sp)
        c.run_histories([p], flags)
        ref = c.read_dose_and_variance(p, raw=True)
        c.reset_plan(p, rewind=True)
        c.run_histories([p], flags | F.FDC_RUN_COUNT_WORK)
        got = c.read_dose_and_variance(p, raw=True)
        wk = c.read_work_counts(p)
        assert np.array_equal(got["E"], ref["E"]) and np.array_equal(got["E2"], ref["E2"])
        assert got["incident"] == o["incident"] and got["escaped"] == ref["escaped"]
        for k, ok in (("steps", "steps"), ("visits", "visits"), ("flushes", "flushes")):
            assert abs(wk[k] - o[ok]) <= 1e-3 * o[ok], (k, wk[k], o[ok])
        c.reset_plan(p)
        assert c.read_work_counts(p) == dict(steps=0, visits=0, flushes=0)
    finally:
        c.close()
