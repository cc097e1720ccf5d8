"""Pins of the oracle's secondary trajectories (Section 2.2: a stored history
is the set of its particles' trajectories, each broken into steps; here a
track's secondary protons, each starting at the end of one of the primary's
steps) against facts fixed outside the walk code.

Hand-built tracks with straight steps (no deflection) in water give closed
forms: a straight trajectory's energy between two depths (or two lateral
positions) is the telescoping difference of the uniform-in-WEL split at the
two path lengths where it crosses them, so the oracle's depth and lateral
profiles must equal the sums written out here, whatever voxel faces it
crosses on the way.  The generated database must conserve each track's
energy across its trajectories, and adding secondaries must leave every
primary's walk unchanged.  CPU only."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1011_2188_amd import inputs as I

FP = float(1 << 24)
VOX = 0.25
NXY, NZ = 64, 64


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _fp(e):
    return int(np.rint(float(np.float32(e)) * FP))


# primary: 30 straight steps; secondary 1 along the primary after step 4,
# secondary 2 at 0.35 rad in the +x direction after step 11
PRIMARY = [(0.23, 2.0 + 0.1 * k) for k in range(30)]
SECS = [(4, 0.0, 0.0, [(0.21, 1.5 + 0.05 * k) for k in range(12)]),
        (11, 0.35, 0.0, [(0.19, 1.2 + 0.03 * k) for k in range(10)])]


def _db(primary=PRIMARY, secs=SECS, e_bin=None):
    st = np.array([[dx, de, 0.0, 0.0] for dx, de in primary], np.float32)
    if e_bin is None:
        e_bin = np.float32(sum(de for _, de in primary) + sum(de for s in secs or [] for _, de in s[3]))
    sec = None
    if secs is not None:
        steps = np.array([[dx, de, 0.0, 0.0] for s in secs for dx, de in s[3]], np.float32).reshape(-1, 4)
        off = np.zeros(len(secs) + 1, np.uint64)
        off[1:] = np.cumsum([len(s[3]) for s in secs])
        sec = I.Secondaries(np.array([0, len(secs)], np.uint32), off, steps,
                            np.array([s[0] for s in secs], np.uint32),
                            np.array([[s[1], s[2]] for s in secs], np.float32).reshape(-1, 2))
    return I.TrackDB(st, np.array([0, len(primary)], np.uint64), np.array([e_bin], np.float32),
                     np.array([0, 1], np.uint32), sec), e_bin


def _phantom():
    return I.water_phantom((NXY, NXY, NZ), VOX, origin=(-NXY * VOX / 2, -NXY * VOX / 2, 0.0))


X0 = 0.125        # the beam runs along the middle of voxel column 32 (x in [0, 0.25))


def _spot(energy, n=8):
    return I.spots([[X0, X0, -2.0]], [[0.0, 0.0, 1.0]], [energy], 0.0, n)


def _profile(steps, s_of_bound, nb, first=None):
    """Energy (fixed point) of a straight trajectory in each of nb bins, the
    bin edges crossed at path lengths s_of_bound(0..nb): the step's energy
    split uniformly in path length, rounded to nearest at each crossing.
    first = (fraction, energy) replaces the first step's length and energy."""
    out = np.zeros(nb, np.int64)
    S0 = 0.0
    for k, (dx, de) in enumerate(steps):
        w, e = float(np.float32(dx)), _fp(de)
        if k == 0 and first is not None:
            w, e = first[0] * w, first[1]
        for b in range(nb):
            def cum(s):
                t = min(max(s - S0, 0.0), w)
                return e if t >= w else int(np.rint(e * (t / w)))
            out[b] += cum(s_of_bound(b + 1)) - cum(s_of_bound(b))
        S0 += w
    return out


def _depth(steps, z0, c, first=None):
    return _profile(steps, lambda j: (j * VOX - z0) / c if j * VOX > z0 else -1.0 if j * VOX < z0 else 0.0, NZ,
                    first)


def _lateral(steps, x0, sn):
    """x-column profile of a trajectory moving up in x at sin(theta) = sn."""
    lo = -NXY * VOX / 2
    return _profile(steps, lambda i: (lo + i * VOX - x0) / sn if lo + i * VOX > x0 else -1.0, NXY)


def _branch_depth(primary, b, start=0):
    return sum(float(np.float32(dx)) for dx, _ in primary[start:b + 1])


def _expected(primary=PRIMARY, secs=SECS, start=0, dropped=(), first=None):
    """Per-history depth (z) and x profiles in closed form, the primary from
    stored step `start` (its first step possibly partial), the secondaries not
    in `dropped`."""
    col = int((X0 + NXY * VOX / 2) // VOX)
    steps = primary[start:]
    z = _depth(steps, 0.0, 1.0, first)
    x = np.zeros(NXY, np.int64)
    x[col] += z.sum()
    # where a branch lies when the first step is partial: shorter by (1 - f) dx
    short = 0.0 if first is None else (1.0 - first[0]) * float(np.float32(primary[start][0]))
    for q, (b, th, ph, st) in enumerate(secs):
        if q in dropped:
            continue
        zb = _branch_depth(primary, b, start) - short
        th = float(np.float32(th))                      # as stored
        zs = _depth(st, zb, math.cos(th))
        z += zs
        if th == 0.0:
            x[col] += zs.sum()
        else:
            assert ph == 0.0
            x += _lateral(st, X0, math.sin(th))
    return z, x


def _oracle_profiles(db, energy, n=8):
    r = O.replay(db, _phantom(), _spot(energy, n))
    E = r["E"]
    return r, E.sum(axis=(1, 2)), E.sum(axis=(0, 1)), E.sum(axis=(0, 2))


def test_straight_secondaries_match_the_closed_form_profiles():
    db, e_bin = _db()
    n = 8
    r, z, x, y = _oracle_profiles(db, e_bin, n)
    ez, ex = _expected()
    T = sum(_fp(de) for _, de in PRIMARY) + sum(_fp(de) for s in SECS for _, de in s[3])
    assert r["incident"] == n * T and r["escaped"] == 0 and int(r["E"].sum()) == n * T
    # each crossing's rounding is the closed form's up to a tie: at most one unit per bin edge
    assert np.abs(z - n * ez).max() <= 2 * n
    assert np.abs(x - n * ex).max() <= 2 * n
    col = int((X0 + NXY * VOX / 2) // VOX)
    assert y[col] == n * T                                  # nothing moves in y (azimuth 0 is +x)
    # the profiles are really those of the branches: a secondary started one
    # step early or late, or along the wrong axis, moves them by far more
    ez_early, _ = _expected(secs=[(3, *SECS[0][1:]), SECS[1]])
    assert np.abs(n * ez_early - z).max() > 1000 * n


def test_azimuth_turns_the_secondary_about_the_primary():
    """phi = pi/2 sends the second secondary along +y: its x profile moves to y."""
    secs = [SECS[0], (SECS[1][0], SECS[1][1], math.pi / 2, SECS[1][3])]
    db, e_bin = _db(secs=secs)
    _, _, x, y = _oracle_profiles(db, e_bin, 4)
    _, ex = _expected()
    assert np.abs(y - 4 * ex).max() <= 8                  # the same profile, along y
    col = int((X0 + NXY * VOX / 2) // VOX)
    assert x[col] == x.sum()


def test_skip_inside_a_secondary_drops_it_and_starts_at_the_next_step():
    """A spot below the bin energy by more than the primary's first five
    steps but less than those and the first secondary: the energy below the
    spot's is the primary's steps 0..4 and all of secondary 1 (its energy
    comes after step 4 in the track's order); the history starts at step 5
    whole, with secondary 2."""
    db, e_bin = _db()
    p4 = sum(_fp(de) for _, de in PRIMARY[:5])
    s1 = sum(_fp(de) for _, de in SECS[0][3])
    e_spot = np.float32(float(e_bin) - (p4 + 0.5 * s1) / FP)
    skip = _fp(e_bin) - _fp(e_spot)
    assert p4 < skip < p4 + s1
    n = 4
    r, z, x, _ = _oracle_profiles(db, e_spot, n)
    T = sum(_fp(de) for _, de in PRIMARY) + s1 + sum(_fp(de) for _, de in SECS[1][3])
    assert r["incident"] == n * (T - p4 - s1)
    assert r["escaped"] == 0
    ez, ex = _expected(start=5, dropped=(0,))
    assert np.abs(z - n * ez).max() <= 2 * n and np.abs(x - n * ex).max() <= 2 * n


def test_skip_past_a_secondary_cuts_the_next_primary_step():
    """A skip that covers secondary 1 and part of step 5: step 5 is replayed
    partially (its remaining energy over the same fraction of its length)."""
    db, e_bin = _db()
    p4 = sum(_fp(de) for _, de in PRIMARY[:5])
    s1 = sum(_fp(de) for _, de in SECS[0][3])
    e5 = _fp(PRIMARY[5][1])
    e_spot = np.float32(float(e_bin) - (p4 + s1 + 0.4 * e5) / FP)
    skip = _fp(e_bin) - _fp(e_spot)
    assert p4 + s1 < skip < p4 + s1 + e5
    e_first = p4 + s1 + e5 - skip
    n = 4
    r, z, x, _ = _oracle_profiles(db, e_spot, n)
    ez, ex = _expected(start=5, dropped=(0,), first=(e_first / e5, e_first))
    assert np.abs(z - n * ez).max() <= 2 * n and np.abs(x - n * ex).max() <= 2 * n
    assert int(r["E"].sum()) == r["incident"]


def test_secondary_leaving_the_phantom_escapes():
    """A secondary turned back upstream (theta > pi/2) from the first step's
    end leaves the box through its front face after zb / |cos theta| of path:
    what it deposited up to there is the closed form's, the rest escapes."""
    secs = [(0, 2.8, 0.0, [(0.21, 1.5)] * 12)]
    db, e_bin = _db(secs=secs)
    n = 2
    r, z, _, _ = _oracle_profiles(db, e_bin, n)
    zb = _branch_depth(PRIMARY, 0)
    s_exit = zb / abs(math.cos(float(np.float32(2.8))))
    inside = _profile(secs[0][3], lambda i: (0.0, s_exit)[i], 1)[0]
    assert 0 < inside < _fp(1.5) * 2
    assert r["escaped"] == n * (12 * _fp(1.5) - inside)
    assert r["escaped"] + int(r["E"].sum()) == r["incident"]


def test_secondary_leaves_along_the_deflected_direction():
    """The primary turns by 0.3 rad towards +x at the end of step 4 (water:
    the stored angle unscaled).  Secondary 1, emitted at step 4's end with
    theta 0, follows the new direction; secondary 2, emitted at step 11's end
    at 0.35 rad with azimuth 0, leaves at 0.3 + 0.35 rad in the x-z plane from
    the point the primary reached.  Every part is a straight segment with a
    closed-form depth and x profile."""
    t4 = float(np.float32(0.3))
    st = np.array([[dx, de, 0.0, 0.0] for dx, de in PRIMARY], np.float32)
    st[4, 2] = t4
    db, e_bin = _db()
    db = I.TrackDB(st, db.track_off, db.bin_E, db.bin_first, db.sec)
    n = 4
    r, z, x, y = _oracle_profiles(db, e_bin, n)
    S = np.cumsum([float(np.float32(dx)) for dx, _ in PRIMARY])
    t2 = t4 + float(np.float32(SECS[1][1]))
    xb2 = X0 + math.sin(t4) * (S[11] - S[4])
    zb2 = S[4] + math.cos(t4) * (S[11] - S[4])
    col = int((X0 + NXY * VOX / 2) // VOX)
    ez = _depth(PRIMARY[:5], 0.0, 1.0)
    ex = np.zeros(NXY, np.int64)
    ex[col] = ez.sum()
    for steps, x0, z0, ang in ((PRIMARY[5:], X0, S[4], t4), (SECS[0][3], X0, S[4], t4), (SECS[1][3], xb2, zb2, t2)):
        ez = ez + _depth(steps, z0, math.cos(ang))
        ex = ex + _lateral(steps, x0, math.sin(ang))
    assert int(r["E"].sum()) == r["incident"]
    assert np.abs(z - n * ez).max() <= 2 * n
    assert np.abs(x - n * ex).max() <= 2 * n
    assert y[col] == y.sum()


def test_secondary_emitted_in_a_compensator_stays_there():
    """A water range compensator thicker than the primary's first five steps:
    secondary 1 (emitted at step 4's end, inside it) is absorbed there with
    its whole energy; secondary 2 (step 11, in the phantom) is replayed.  The
    phantom then holds what the track without secondary 1 leaves, and the
    escaped energy grows by exactly secondary 1's."""
    T = 1.5
    S4 = _branch_depth(PRIMARY, 4)
    assert S4 < T
    dev = I.beam_device([0.0, 0.0, -T], [0.0, 0.0, 1.0], [0.1, 0.1], np.full((100, 100), T))
    ph = I.water_phantom((NXY, NXY, NZ), VOX, origin=(-NXY * VOX / 2, -NXY * VOX / 2, 0.0))
    db, e_bin = _db()
    no1, _ = _db(secs=[SECS[1]], e_bin=e_bin)
    n = 4
    a = O.replay(db, ph, _spot(e_bin, n), devices=([dev], [0]))
    b = O.replay(no1, ph, _spot(e_bin, n), devices=([dev], [0]))
    s1 = sum(_fp(de) for _, de in SECS[0][3])
    assert np.array_equal(a["E"], b["E"])
    assert a["incident"] == b["incident"] + n * s1
    assert a["escaped"] == b["escaped"] + n * s1


def test_generated_database_conserves_each_tracks_energy():
    bins = [100.0, 150.0]
    db = I.make_water_track_db(bins, 400, seed=5, secondaries=True)
    plain = I.make_water_track_db(bins, 400, seed=5)
    s = db.sec
    assert s.n > 0 and s.sec_first[-1] == s.n
    n_sec = np.diff(s.sec_first.astype(np.int64))
    assert n_sec.max() <= I.NUC_MAX_PER_TRACK
    steps_sec = np.add.reduceat(s.steps[:, 1].astype(np.float64), s.off[:-1].astype(np.int64)) \
        if s.n else np.zeros(0)
    for t in range(db.n_tracks):
        a, b = int(db.track_off[t]), int(db.track_off[t + 1])
        e = db.steps[a:b, 1].astype(np.float64).sum()
        j0, j1 = int(s.sec_first[t]), int(s.sec_first[t + 1])
        e += steps_sec[j0:j1].sum()
        Eb = bins[int(np.searchsorted(db.bin_first[1:], t, side="right"))]
        assert abs(e - Eb) < 2e-3, (t, e, Eb)
        if j1 > j0:
            br = s.branch[j0:j1]
            assert np.all(np.diff(br.astype(np.int64)) >= 0) and br[-1] < b - a - 1
        else:
            pa, pb = int(plain.track_off[t]), int(plain.track_off[t + 1])
            assert np.array_equal(db.steps[a:b], plain.steps[pa:pb])
    # interactions per cm of primary path close to the rate (binomial spread)
    path = float(db.steps[:, 0].sum())
    assert abs(s.n / path - I.NUC_PER_CM) < 5 * math.sqrt(I.NUC_PER_CM / path)


def test_secondaries_leave_the_primary_walk_unchanged():
    """With the spot at its bin energy every secondary is replayed, after the
    primary: end points and reasons equal those of the same primaries without
    secondaries, and every voxel holds at least the primaries' deposit."""
    db = I.make_water_track_db([110.0, 120.0], 150, seed=9, secondaries=True)
    prim = I.TrackDB(db.steps, db.track_off, db.bin_E, db.bin_first, None)
    ph = I.thorax_phantom((48, 48, 40), 0.4, seed=3, scale=(48 * 0.4 / 51.2, 48 * 0.4 / 51.2, 40 * 0.4 / 25.6))
    sp = I.spots([[0.3, -12.0, 0.2], [-12.0, 0.4, -0.3]], [[0.0, 1.0, 0.0], [1.0, 0.0, 0.0]], [110.0, 120.0],
                 0.5, 3000)
    a = O.replay(db, ph, sp)
    b = O.replay(prim, ph, sp)
    assert np.all(a["E"] >= b["E"])
    T_sec = np.zeros(db.n_tracks, np.int64)
    for t in range(db.n_tracks):
        for j in range(int(db.sec.sec_first[t]), int(db.sec.sec_first[t + 1])):
            T_sec[t] += sum(_fp(v) for v in db.sec.steps[int(db.sec.off[j]):int(db.sec.off[j + 1]), 1])
    assert a["incident"] > b["incident"]
    assert a["incident"] - int(a["E"].sum()) == a["escaped"]
    for spot in (0, 1):
        ea, ra = O.endpoints(db, ph, sp, spot, 0, 1500)
        eb, rb = O.endpoints(prim, ph, sp, spot, 0, 1500)
        assert np.array_equal(ra, rb) and np.array_equal(ea, eb)
