"""Pins of the oracle's beam-line devices (an aperture and a range compensator
upstream of the phantom; Section 4 names them as the geometry the CPU code
handled and the GPU code did not) against facts fixed outside the device code:
an open device changes nothing, a closed one stops every history on its face,
an aperture stops exactly the histories whose ray meets its closed pixels, a
water compensator equals the same thickness of water voxels in front of the
phantom, and a compensator of relative stopping power r shifts the depth-dose
like r times its thickness of water.  CPU only."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1011_2188_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


DB = dict(bins=[95.0, 100.0], tracks=200, seed=31)


def _db():
    return I.make_water_track_db(DB["bins"], DB["tracks"], seed=DB["seed"])


def _water(nz=40, z0=0.0, nxy=40, vox=0.25):
    return I.water_phantom((nxy, nxy, nz), vox, origin=(-nxy * vox / 2, -nxy * vox / 2, z0))


def _spot(n=600, sigma=0.4, energy=98.0):
    return I.spots([[0.1, -0.05, -20.0]], [[0.0, 0.0, 1.0]], [energy], sigma, n)


def _device(z_face, pixels, pitch=0.1, rsp=1.0, rscp=1.0):
    return I.beam_device([0.0, 0.0, z_face], [0.0, 0.0, 1.0], [pitch, pitch], pixels, rsp, rscp)


def test_open_device_changes_nothing():
    db, ph, sp = _db(), _water(), _spot()
    dev = _device(-2.0, np.zeros((100, 100)))
    a = O.replay(db, ph, sp)
    b = O.replay(db, ph, sp, devices=([dev], [0]))
    assert np.array_equal(a["E"], b["E"]) and np.array_equal(a["E2"], b["E2"])
    assert a["incident"] == b["incident"] and a["escaped"] == b["escaped"]
    ea, ra = O.endpoints(db, ph, sp, 0, 0, 200)
    eb, rb = O.endpoints(db, ph, sp, 0, 0, 200, devices=([dev], [0]))
    assert np.array_equal(ea, eb) and np.array_equal(ra, rb)


def test_closed_device_stops_everything_on_its_face():
    db, ph, sp = _db(), _water(), _spot()
    dev = _device(-2.0, -np.ones((100, 100)))
    r = O.replay(db, ph, sp, devices=([dev], [0]))
    assert not r["E"].any() and not r["E2"].any()
    assert r["escaped"] == r["incident"] > 0
    ep, reason = O.endpoints(db, ph, sp, 0, 0, 100, devices=([dev], [0]))
    assert np.all(reason == 3)
    assert np.allclose(ep[:, 2], -2.0, atol=1e-12)            # on the device's upstream face


def test_aperture_stops_exactly_the_rays_through_closed_pixels():
    """Pixels with e1 (= +x for a beam along +z) below 0 closed: a history
    stops on the face iff its straight ray from the source (vacuum before the
    phantom) meets the plane at x < 0; every other history is untouched."""
    db, ph, sp = _db(), _water(), _spot(n=300, sigma=0.6)
    pix = np.zeros((100, 100))
    pix[:, :50] = -1.0                                         # columns = e1 = x from -5 cm to 0
    dev = _device(-2.0, pix)
    e0, r0 = O.endpoints(db, ph, sp, 0, 0, 300)
    e1, r1 = O.endpoints(db, ph, sp, 0, 0, 300, devices=([dev], [0]))
    for h in range(300):
        ev, _, _ = O.trace(db, ph, sp, 0, h)
        v = next(e[1] for e in ev if e[0] == O.EV_VOXEL)     # entry voxel: x of the straight ray at z = 0
        ix = v % 40
        if ix < 20:
            assert r1[h] == 3 and abs(e1[h, 2] + 2.0) < 1e-12
        else:
            assert r1[h] == r0[h] and np.array_equal(e1[h], e0[h])


def test_water_compensator_equals_water_voxels():
    """A water compensator (RSP = RScP = 1) of thickness T right in front of a
    water phantom replays every history exactly as T of water voxels added to
    the phantom's upstream side: same deposits in the common voxels, same end
    points, and the compensator's absorbed energy is the added voxels' dose."""
    db, sp = _db(), _spot(n=400)
    vox, T = 0.25, 1.5
    a_ph = _water(nz=40, z0=0.0)
    b_ph = _water(nz=40 + int(round(T / vox)), z0=-T)
    dev = _device(-T, np.full((100, 100), T))
    a = O.replay(db, a_ph, sp, devices=([dev], [0]))
    b = O.replay(db, b_ph, sp)
    nl = int(round(T / vox))
    Eb = b["E"][nl:]
    diff = np.abs(a["E"] - Eb)
    assert a["incident"] == b["incident"]
    # the same walk in exact arithmetic: rounding of the positions can move a
    # piece across a voxel face only in rare cases
    assert diff.sum() <= 1e-6 * Eb.sum()
    assert np.mean(diff == 0) > 0.999
    absorbed = a["escaped"] - (b["escaped"])
    assert abs(absorbed - int(b["E"][:nl].sum())) <= 1e-6 * b["incident"]
    ea, ra = O.endpoints(db, a_ph, sp, 0, 0, 150, devices=([dev], [0]))
    eb, rb = O.endpoints(db, b_ph, sp, 0, 0, 150)
    assert np.array_equal(ra, rb)
    assert np.max(np.abs(ea - eb)) < 1e-9


def test_compensator_stopping_power_shifts_the_depth_dose():
    """A compensator of RSP = RScP = 2 (G = 1) and thickness T consumes the
    same water-equivalent length, with the same deflections, as a water
    compensator of thickness 2 T: every history enters the phantom in the same
    step state and direction, only laterally displaced, so the laterally
    integrated depth-dose in a wide water phantom is the same."""
    db, sp = _db(), _spot(n=400, sigma=0.3)
    ph = _water(nz=48, z0=0.0, nxy=80, vox=0.25)
    T = 0.75
    d2 = _device(-T, np.full((100, 100), T), rsp=2.0, rscp=2.0)
    dw = _device(-2 * T, np.full((100, 100), 2 * T))
    a = O.replay(db, ph, sp, devices=([d2], [0]))
    b = O.replay(db, ph, sp, devices=([dw], [0]))
    ia, ib = a["E"].sum(axis=(1, 2)), b["E"].sum(axis=(1, 2))
    assert a["incident"] == b["incident"]
    assert np.abs(ia - ib).sum() <= 1e-6 * ib.sum()
    assert abs(a["escaped"] - b["escaped"]) <= 1e-6 * a["incident"]
    # and it is a real shift: the Bragg peak lies 2 T = 1.5 cm (6 slabs) upstream of the no-compensator one
    c = O.replay(db, ph, sp)
    ic = c["E"].sum(axis=(1, 2))
    assert int(np.argmax(ic)) - int(np.argmax(ia)) in (5, 6, 7)


def test_device_behind_the_source_stops_every_history():
    """A device face upstream of the start points (or a beam turned away from
    it) is never crossed: the history cannot reach the phantom through it."""
    db, ph, sp = _db(), _water(), _spot(n=50)
    ahead = _device(-2.0, np.zeros((100, 100)))
    behind = _device(-30.0, np.zeros((100, 100)))
    _, r_ahead = O.endpoints(db, ph, sp, 0, 0, 50, devices=([ahead], [0]))
    _, r_behind = O.endpoints(db, ph, sp, 0, 0, 50, devices=([behind], [0]))
    assert np.all(r_ahead != 3) and np.all(r_behind == 3)
