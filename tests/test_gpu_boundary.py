"""The C ABI's loaders and allocator hook on the GPU: the track database read
from its file gives the same tallies as the arrays; contexts whose device
memory comes from torch's caching allocator agree with the oracle; an
allocator that returns NULL makes the loaders fail with FDC_E_NOMEM and leave
the context as it was, and a retry then succeeds."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from paper_1011_2188_amd import fdc as F  # noqa: E402
from paper_1011_2188_amd import inputs as I  # noqa: E402
from paper_1011_2188_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    torch.cuda.init()


def _small():
    ph = I.thorax_phantom((64, 48, 40), 0.3, seed=11)
    sp = I.spots([[0.3, -0.2, -20.0], [-0.5, 0.4, 20.0]], [[0, 0, 1.0], [0, 0, -1.0]], [97.5, 110.0], 0.4, 5000)
    db = I.make_water_track_db([95.0, 100.0, 105.0, 110.0], 300, seed=5)
    return ph, sp, db


def _run(c, ph, sp):
    p = c.load_phantom(ph)
    c.add_beam_spots(p, sp)
    c.run_histories([p], F.FDC_RUN_VARIANCE)
    return c.read_dose_and_variance(p, raw=True)


def _check_oracle(g, o, ph, n):
    assert g["deposited"] + g["escaped"] == g["incident"] == o["incident"]
    dose_o, _ = O.dose_and_variance(o["E"], o["E2"], n, ph)
    dmax = dose_o.max()
    sel = dose_o > 0.1 * dmax
    assert np.abs(g["dose"] - dose_o)[sel].max() <= 0.005 * dmax


def test_track_db_file_same_tallies(tmp_path):
    ph, sp, db = _small()
    path = tmp_path / "db.bin"
    I.write_track_db_file(path, db, db_seed=5)
    with F.Context(0, 1, table=I.HU_TABLE_DEFAULT) as a, F.Context(0, 1, table=I.HU_TABLE_DEFAULT) as b:
        a.load_track_db(db)
        b.load_track_db_file(path)
        ga, gb = _run(a, ph, sp), _run(b, ph, sp)
    assert np.array_equal(ga["E"], gb["E"]) and np.array_equal(ga["E2"], gb["E2"])
    assert ga["incident"] == gb["incident"] and ga["escaped"] == gb["escaped"]


def test_torch_allocator_matches_oracle_and_default():
    ph, sp, db = _small()
    with F.Context(0, 1, torch_allocator=True, table=I.HU_TABLE_DEFAULT) as t, \
            F.Context(0, 1, table=I.HU_TABLE_DEFAULT) as d:
        before = torch.cuda.memory_allocated()
        t.load_track_db(db)
        assert torch.cuda.memory_allocated() > before          # the database went through torch
        d.load_track_db(db)
        gt, gd = _run(t, ph, sp), _run(d, ph, sp)
    assert np.array_equal(gt["E"], gd["E"]) and np.array_equal(gt["E2"], gd["E2"])
    o = O.replay(db, ph, sp, seed=1)
    _check_oracle(gt, o, ph, int(sp["n_histories"].sum()))


class _FlakyAllocator:
    """torch-backed device memory; returns NULL once `budget` is used up."""

    def __init__(self):
        self.budget = None          # allocations that still succeed (None: all)
        self.live = {}
        self.calls = 0
        self.fa = F.ALLOC_FN(self._alloc)
        self.ff = F.FREE_FN(self._free)

    def _alloc(self, n, user):
        self.calls += 1
        if self.budget is not None:
            if self.budget <= 0:
                return None
            self.budget -= 1
        t = torch.empty(int(n), dtype=torch.uint8, device="cuda")
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, p, user):
        self.live.pop(p, None)


def test_allocator_null_gives_nomem_and_keeps_state():
    ph, sp, db = _small()
    al = _FlakyAllocator()
    c = F.Context(0, 1)
    try:
        F._check(c.h, F.lib().fdc_set_allocator(c.h, al.fa, al.ff, None))
        c.set_hu_table(I.HU_TABLE_DEFAULT)
        c.load_track_db(db)
        p0 = c.load_phantom(ph)
        c.add_beam_spots(p0, sp)
        live = len(al.live)
        for budget in (0, 2, 4):                               # the 1st, 3rd and 5th of its 5 buffers fail
            al.budget = budget
            calls = al.calls
            with pytest.raises(F.FdcError) as e:
                c.load_phantom(ph)
            assert e.value.code == F.FDC_E_NOMEM and al.calls > calls
            assert len(al.live) == live                        # partial allocations returned
        for budget in (0, 1, 3):
            al.budget = budget
            with pytest.raises(F.FdcError) as e:
                c.load_track_db(I.make_water_track_db([95.0, 100.0, 105.0, 110.0], 200, seed=6))
            assert e.value.code == F.FDC_E_NOMEM
            assert len(al.live) == live
        al.budget = None
        p1 = c.load_phantom(ph)                                # the failed load took no plan id
        assert p1 == p0 + 1
        c.add_beam_spots(p1, sp)
        c.run_histories([p1], F.FDC_RUN_VARIANCE)              # the old database is still loaded
        g = c.read_dose_and_variance(p1, raw=True)
    finally:
        c.close()
    assert not al.live                                         # everything went back through the hook
    o = O.replay(db, ph, sp, seed=1, plan=p1)
    _check_oracle(g, o, ph, int(sp["n_histories"].sum()))


def test_allocator_hook_used_for_every_device_buffer():
    """With the hook set first, the context never calls hipMalloc: every
    buffer (database, phantom, tallies, work table, queue) comes from it and
    returns to it."""
    ph, sp, db = _small()
    al = _FlakyAllocator()
    c = F.Context(0, 1)
    F._check(c.h, F.lib().fdc_set_allocator(c.h, al.fa, al.ff, None))
    c.set_hu_table(I.HU_TABLE_DEFAULT)
    c.set_launch_config(waves_per_block=16, blocks_per_cu=1, tally_slots=4096, units_per_wave=1, tally_mode=2,
                        source_order=1)
    c.load_track_db(db)
    p = c.load_phantom(ph)
    c.add_beam_spots(p, sp)
    c.run_histories([p], F.FDC_RUN_VARIANCE)
    c.read_dose_and_variance(p)
    assert al.calls >= 8 and al.live
    c.close()
    assert not al.live
