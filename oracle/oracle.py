"""Python side of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It wraps the plain-C replay in `fdc_oracle.c` and adds the
FP64 numpy definitions of the quantities computed from the tallies:

  * dose = deposited energy / voxel mass (Section 2.3), in Gy per primary;
  * the history-by-history uncertainty of Eq. (2), summed over all N histories
    of the plan (the upper index of the sum in Eq. (2) is read as N);
  * the batch uncertainty of Eq. (1);
  * the mean dose uncertainty: mean of sigma_D / D over voxels with
    D > Dmax / 2 (Section 2.4);
  * the gamma index (Low et al. 1998) with a global dose criterion.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "fdc_oracle.c")

MEV_J = 1.602176634e-13          # J per MeV
FP_LSB_MEV = 2.0 ** -24          # fixed-point energy unit
FLAG_VARIANCE = 1
FLAG_ROTATE = 2
END_STOP, END_ESCAPE, END_MISS = 0, 1, 2


def build(force=True):
    """Compile the oracle with gcc (plain C, -O2, OpenMP)."""
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= os.path.getmtime(SRC_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                    "-o", tmp, SRC_PATH, "-lm"], check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = C.CDLL(LIB_PATH)
    return _lib


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


# The material table the oracle uses unless a test passes its own: synthetic
# piecewise-linear constants (Section 2.5 leaves the HU conversion to other
# work).  Breakpoints at HU -1000 / 0 / 1000 / 3071; water (HU 0) is exactly
# (1, 1, 1); RScP = rho * k with k = 1 up to HU 0, rising linearly to 1.35 at
# HU 1000 and flat above; HU below -990 is vacuum.
ORACLE_HU_TABLE = {
    "hu": np.array([-1000.0, 0.0, 1000.0, 3071.0]),
    "rho": np.array([0.0012, 1.0, 1.6, 2.84]),
    "rsp": np.array([0.0011, 1.0, 1.5, 2.64]),
    "rscp": np.array([0.0012 * 1.0, 1.0 * 1.0, 1.6 * 1.35, 2.84 * 1.35]),
    "vacuum_below_hu": -990.0,
}


def default_table():
    return ORACLE_HU_TABLE


# --------------------------------------------------------------------------
def philox(ctr, key):
    """Philox4x32-10 of counter ctr[4] (uint32) under key[2]."""
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def philox_batch(ctr, key):
    """Philox4x32-10 of counters ctr[n,4] under one key."""
    c = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros_like(c)
    lib().oracle_philox_batch(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32),
                              C.c_uint64(c.shape[0]))
    return out


def rotate(d, theta, phi):
    """The polar/azimuth direction rotation used at the end of every step."""
    v = np.ascontiguousarray(d, np.float64).copy()
    lib().oracle_rotate(_p(v, C.c_double), C.c_double(theta), C.c_double(phi))
    return v


def uniform(x):
    f = lib().oracle_uniform
    f.restype = C.c_double
    return f(C.c_uint32(int(x)))


def material(hu, table=None):
    """(rho, rsp, G, vacuum) for an int16 HU array, by the piecewise-linear table."""
    t = table or default_table()
    hu = np.ascontiguousarray(hu, np.int16).ravel()
    n = hu.size
    rho, rsp, g = (np.zeros(n) for _ in range(3))
    vac = np.zeros(n, np.uint8)
    pts = [np.ascontiguousarray(t[k], np.float64) for k in ("hu", "rho", "rsp", "rscp")]
    lib().oracle_material(*[_p(a, C.c_double) for a in pts], C.c_int(pts[0].size),
                          C.c_double(t["vacuum_below_hu"]), _p(hu, C.c_int16), C.c_int(n),
                          _p(rho, C.c_double), _p(rsp, C.c_double), _p(g, C.c_double),
                          _p(vac, C.c_uint8))
    return rho, rsp, g, vac.astype(bool)


def _common(db, ph, sp, table):
    t = table or default_table()
    spots = np.ascontiguousarray(sp)
    arrs = dict(
        steps=np.ascontiguousarray(db.steps, np.float32),
        track_off=np.ascontiguousarray(db.track_off, np.uint64),
        bin_E=np.ascontiguousarray(db.bin_E, np.float32),
        bin_first=np.ascontiguousarray(db.bin_first, np.uint32),
        hu=np.ascontiguousarray(ph.hu, np.int16),
        dims=np.array(ph.shape_xyz, np.int32),
        vox=np.asarray(ph.voxel_cm, np.float64),
        org=np.asarray(ph.origin_cm, np.float64),
        tab=[np.ascontiguousarray(t[k], np.float64) for k in ("hu", "rho", "rsp", "rscp")],
        pos=np.ascontiguousarray(spots["pos_cm"], np.float32),
        dir=np.ascontiguousarray(spots["dir"], np.float32),
        E=np.ascontiguousarray(spots["energy_MeV"], np.float32),
        sig=np.ascontiguousarray(spots["sigma_cm"], np.float32),
    )
    args = [_p(arrs["steps"], C.c_float), _p(arrs["track_off"], C.c_uint64), C.c_uint32(db.n_tracks),
            _p(arrs["bin_E"], C.c_float), _p(arrs["bin_first"], C.c_uint32), C.c_uint32(db.n_bins),
            _p(arrs["hu"], C.c_int16), _p(arrs["dims"], C.c_int), _p(arrs["vox"], C.c_double),
            _p(arrs["org"], C.c_double)]
    args += [_p(a, C.c_double) for a in arrs["tab"]]
    args += [C.c_int(arrs["tab"][0].size), C.c_double(t["vacuum_below_hu"]),
             _p(arrs["pos"], C.c_float), _p(arrs["dir"], C.c_float), _p(arrs["E"], C.c_float),
             _p(arrs["sig"], C.c_float)]
    return arrs, args


def phase_space_sources(pos, dirs, energies, bin_E, first_source):
    """The sources a list of incident protons (Section 2.3: the phase space
    read from a file) becomes: the protons grouped by energy bin (the smallest
    bin energy >= the proton's), bins in increasing order, protons in list order
    within a bin.  Returns a dict for replay(..., phase_space=...): per source
    index (first_source onward, after the plan's spots) the first proton and
    count in the regrouped arrays pos, dir, E."""
    pos = np.asarray(pos, np.float32).reshape(-1, 3)
    dirs = np.asarray(dirs, np.float32).reshape(-1, 3)
    E = np.asarray(energies, np.float32).ravel()
    bins = np.asarray(bin_E, np.float32)
    b = np.array([int(np.searchsorted(bins, e, side="left")) for e in E], np.int64)   # first bin >= E
    order = np.argsort(b, kind="stable")
    groups = [(int(v), int(np.count_nonzero(b == v))) for v in np.unique(b)]
    first = np.zeros(first_source + len(groups), np.uint64)
    count = np.zeros(first_source + len(groups), np.uint64)
    o = 0
    for k, (_, n) in enumerate(groups):
        first[first_source + k] = o
        count[first_source + k] = n
        o += n
    return dict(first=first, count=count, pos=np.ascontiguousarray(pos[order]),
                dir=np.ascontiguousarray(dirs[order]), E=np.ascontiguousarray(E[order]),
                bins=[g for g, _ in groups])


class _PhaseSpace:
    """Installs phase-space sources for the oracle calls inside the block."""

    def __init__(self, ps):
        self.ps = ps

    def __enter__(self):
        if self.ps is not None:
            ps = self.ps
            self.keep = [np.ascontiguousarray(ps["first"], np.uint64), np.ascontiguousarray(ps["count"], np.uint64),
                         np.ascontiguousarray(ps["pos"], np.float32), np.ascontiguousarray(ps["dir"], np.float32),
                         np.ascontiguousarray(ps["E"], np.float32)]
            f, c, p, d, e = self.keep
            lib().oracle_set_phase_space(_p(f, C.c_uint64), _p(c, C.c_uint64), _p(p, C.c_float),
                                         _p(d, C.c_float), _p(e, C.c_float))

    def __exit__(self, *a):
        if self.ps is not None:
            lib().oracle_set_phase_space(None, None, None, None, None)


class _Devices:
    """Installs beam-line devices for the oracle calls inside the block.
    devices: (list of device dicts from inputs.beam_device, spot -> device
    index array with -1 for none), or None."""

    def __init__(self, devices, n_spots):
        self.devices = devices
        self.n_spots = n_spots

    def __enter__(self):
        if self.devices is not None:
            devs, spot_dev = self.devices
            par = np.zeros((max(len(devs), 1), 16), np.float64)
            offs = np.zeros(max(len(devs), 1), np.uint64)
            pix = []
            o = 0
            for i, dv in enumerate(devs):
                par[i, 0:3] = dv["origin_cm"]
                par[i, 3:6] = dv["dir"]
                par[i, 6:8] = dv["pitch_cm"]
                par[i, 8:10] = dv["n"]
                par[i, 10] = dv["rsp"]
                par[i, 11] = dv["rscp"]
                offs[i] = o
                p = np.ascontiguousarray(dv["pixels"], np.float32).ravel()
                pix.append(p)
                o += p.size
            sd = np.full(self.n_spots, -1, np.int32)
            sd[:len(spot_dev)] = np.asarray(spot_dev, np.int32)
            self.keep = [sd, np.ascontiguousarray(par.ravel()),
                         np.ascontiguousarray(np.concatenate(pix) if pix else np.zeros(1, np.float32)), offs]
            a, b, c, d = self.keep
            lib().oracle_set_devices(_p(a, C.c_int32), _p(b, C.c_double), _p(c, C.c_float), _p(d, C.c_uint64))

    def __exit__(self, *a):
        if self.devices is not None:
            lib().oracle_set_devices(None, None, None, None)


class _Secondaries:
    """Installs a database's secondary trajectories (db.sec) for the oracle
    calls inside the block; a database without them installs nothing."""

    def __init__(self, db):
        self.sec = getattr(db, "sec", None)

    def __enter__(self):
        if self.sec is not None:
            s = self.sec
            self.keep = [np.ascontiguousarray(s.sec_first, np.uint32), np.ascontiguousarray(s.off, np.uint64),
                         np.ascontiguousarray(s.steps, np.float32).reshape(-1),
                         np.ascontiguousarray(s.branch, np.uint32), np.ascontiguousarray(s.emit, np.float32)]
            if self.keep[2].size == 0:
                self.keep[2] = np.zeros(4, np.float32)
            f, o, st, b, e = self.keep
            lib().oracle_set_secondaries(_p(f, C.c_uint32), _p(o, C.c_uint64), _p(st, C.c_float),
                                         _p(b, C.c_uint32), _p(e, C.c_float))

    def __exit__(self, *a):
        if self.sec is not None:
            lib().oracle_set_secondaries(None, None, None, None, None)


def replay(db, ph, sp, h_begin=None, h_count=None, plan=0, seed=1, R=64, flags=FLAG_VARIANCE,
           threads=None, table=None, exact_e2=False, phase_space=None, devices=None):
    """Replay histories h_begin[i] .. h_begin[i]+h_count[i]-1 of every spot i.

    Returns a dict with the int64 energy tally E, the uint64 sum-of-squares tally
    E2 (x-fastest, shape [nz,ny,nx]), incident/escaped energy (fixed point) and
    the work counters (steps, visits, vacuum_visits, flushes).  With exact_e2
    also E2x: each history's whole deposit in a voxel squared once (Eq. (2)
    taken literally; E2 squares every visit on its own).  phase_space (from
    phase_space_sources): sources past the spots are listed protons; sp must
    then hold one (placeholder) row per source and h_count give each source's
    histories.  devices: (device dicts from inputs.beam_device, per spot the
    index of the device it passes or -1): an aperture and range compensator
    upstream of the phantom, whose absorbed energy counts as escaped.  A
    database with secondary trajectories (db.sec) replays them too."""
    arrs, args = _common(db, ph, sp, table)
    ns = len(sp)
    hb = np.zeros(ns, np.uint64) if h_begin is None else np.ascontiguousarray(h_begin, np.uint64)
    hc = (np.ascontiguousarray(sp["n_histories"], np.uint64) if h_count is None
          else np.ascontiguousarray(h_count, np.uint64))
    nx, ny, nz = ph.shape_xyz
    E = np.zeros(nx * ny * nz, np.int64)
    E2 = np.zeros(nx * ny * nz, np.uint64)
    stats = np.zeros(6, np.int64)
    E2x = np.zeros(nx * ny * nz, np.uint64) if exact_e2 else None
    nthreads = threads or int(os.environ.get("ORACLE_THREADS", min(os.cpu_count() or 1, 16)))
    with _PhaseSpace(phase_space), _Devices(devices, ns), _Secondaries(db):
        rc = lib().oracle_replay_e2x(*args, C.c_uint32(ns), _p(hb, C.c_uint64), _p(hc, C.c_uint64),
                                     C.c_uint32(plan), C.c_uint64(seed), C.c_uint32(R), C.c_uint32(flags),
                                     C.c_int(nthreads), _p(E, C.c_int64), _p(E2, C.c_uint64),
                                     _p(stats, C.c_int64), _p(E2x, C.c_uint64) if exact_e2 else None)
    if rc != 0:
        raise RuntimeError("oracle replay failed: energy not conserved, or a source above the top energy bin")
    extra = dict(E2x=E2x.reshape(nz, ny, nx)) if exact_e2 else {}
    return dict(**extra, E=E.reshape(nz, ny, nx), E2=E2.reshape(nz, ny, nx), incident=int(stats[0]),
                escaped=int(stats[1]), steps=int(stats[2]), visits=int(stats[3]),
                vacuum_visits=int(stats[4]), flushes=int(stats[5]),
                n_histories=int(hc.sum()), threads=nthreads)


def endpoints(db, ph, sp, spot, h0, n, plan=0, seed=1, R=64, flags=0, table=None, phase_space=None,
              devices=None):
    """End point (cm, float64 [n,3]) and end reason of histories h0..h0+n-1 of a
    spot (0 stopped, 1 escaped, 2 missed the phantom, 3 stopped upstream by a
    beam-line device)."""
    arrs, args = _common(db, ph, sp, table)
    xyz = np.zeros((n, 3), np.float64)
    reason = np.zeros(n, np.int32)
    with _PhaseSpace(phase_space), _Devices(devices, len(sp)), _Secondaries(db):
        lib().oracle_endpoints(*args, C.c_uint32(spot), C.c_uint64(h0), C.c_uint32(n), C.c_uint32(plan),
                               C.c_uint64(seed), C.c_uint32(R), C.c_uint32(flags),
                               _p(xyz, C.c_double), _p(reason, C.c_int32))
    if np.any(reason < 0):
        raise RuntimeError("oracle replay failed: energy not conserved, or a source above the top energy bin")
    return xyz, reason


EV_VOXEL, EV_VACUUM, EV_STEP_END, EV_ESCAPE = 0, 1, 2, 3


def trace(db, ph, sp, spot, h, plan=0, seed=1, R=64, flags=0, table=None, cap=100_000):
    """The walk of one history as a list of events (kind, voxel, piece, axis,
    wel, move); see oracle_trace_history.  Returns (events, reason, end point)."""
    arrs, args = _common(db, ph, sp, table)
    ev = np.zeros((cap, 4), np.int64)
    evd = np.zeros((cap, 2), np.float64)
    reason = C.c_int32()
    ep = np.zeros(3, np.float64)
    with _Secondaries(db):
        n = lib().oracle_trace_history(*args, C.c_uint32(spot), C.c_uint64(h), C.c_uint32(plan), C.c_uint64(seed),
                                       C.c_uint32(R), C.c_uint32(flags), _p(ev, C.c_int64), _p(evd, C.c_double),
                                       C.c_int(cap), C.byref(reason), _p(ep, C.c_double))
    if n > cap:
        raise RuntimeError("trace longer than its buffer")
    out = [(int(a), int(b), int(c), int(d), float(w), float(m)) for (a, b, c, d), (w, m) in zip(ev[:n], evd[:n])]
    return out, int(reason.value), ep


# --------------------------------------------------------------------------
# quantities derived from the tallies (FP64)
# --------------------------------------------------------------------------
def voxel_mass_kg(ph, table=None):
    rho, _, _, vac = material(ph.hu, table)
    vol = float(np.prod(np.asarray(ph.voxel_cm, np.float64)))
    return (rho * vol * 1e-3).reshape(ph.hu.shape), vac.reshape(ph.hu.shape)


def dose_and_variance(E, E2, n_histories, ph, table=None):
    """Dose per primary (Gy) = E / m / N, and the Eq. (2) variance of that mean.

    S1 = sum_i D_i and S2 = sum_i D_i^2 over all N histories (zeros included):
    var = (S2/N - (S1/N)^2) / (N - 1).  E2 is in units of 2^-24 MeV^2."""
    m, vac = voxel_mass_kg(ph, table)
    N = float(n_histories)
    c = FP_LSB_MEV * MEV_J / np.where(vac, 1.0, m)
    S1 = E.astype(np.float64) * c
    S2 = E2.astype(np.float64) * FP_LSB_MEV * (MEV_J / np.where(vac, 1.0, m)) ** 2
    dose = np.where(vac, 0.0, S1 / N)
    var = np.where(vac, 0.0, (S2 / N - (S1 / N) ** 2) / max(N - 1.0, 1.0))
    return dose, var


def mean_uncertainty(dose, sigma, vacuum=None):
    """Mean of sigma/D over voxels with D > Dmax/2 (vacuum voxels excluded)."""
    d = dose if vacuum is None else np.where(vacuum, 0.0, dose)
    dmax = d.max()
    sel = d > 0.5 * dmax
    return float(np.mean(sigma[sel] / d[sel]))


def batch_uncertainty(doses):
    """Eq. (1): sqrt(sum_i (D_i - mean)^2 / (n (n-1))) over n independent batches."""
    D = np.stack([np.asarray(d, np.float64) for d in doses])
    n = D.shape[0]
    mean = D.mean(axis=0)
    return mean, np.sqrt(((D - mean) ** 2).sum(axis=0) / (n * (n - 1)))


def _upsample2(a):
    """Trilinear interpolation at half-voxel spacing: along each axis the new
    points are the voxel values and the midpoints between neighbours."""
    for ax in range(3):
        a = np.moveaxis(a, ax, 0)
        n = a.shape[0]
        u = np.empty((2 * n - 1,) + a.shape[1:])
        u[0::2] = a
        u[1::2] = 0.5 * (a[:-1] + a[1:])
        a = np.moveaxis(u, 0, ax)
    return a


def gamma_index(ref, ev, ph, dose_frac=0.02, dta_cm=0.2, cutoff_frac=0.1, search_cm=0.6, table=None):
    """Gamma index (Low et al. 1998), global dose criterion dose_frac * Dmax(ref).

    Evaluated voxels: non-vacuum reference voxels with D >= cutoff_frac * Dmax.
    gamma = min over points p of the evaluated dose upsampled twice per axis
    (trilinear) within search_cm of sqrt(|r - p|^2 / dta^2 + (D_e(p) - D_r)^2 /
    (dose_frac * Dmax)^2).  Returns (gamma array with -1 where not evaluated,
    pass rate = fraction of evaluated voxels with gamma <= 1)."""
    ref = np.asarray(ref, np.float64)
    ev = np.asarray(ev, np.float64)
    _, vac = voxel_mass_kg(ph, table)
    dmax = ref[~vac].max()
    sel = (~vac) & (ref >= cutoff_frac * dmax)
    U = _upsample2(ev)
    nz, ny, nx = ref.shape
    vx, vy, vz = (float(v) for v in ph.voxel_cm)
    z, y, x = np.nonzero(sel)
    dr = ref[sel]
    best = np.full(dr.shape, np.inf)
    rx, ry, rz = (int(np.floor(search_cm / (0.5 * v) + 1e-9)) for v in (vx, vy, vz))
    for c in range(-rz, rz + 1):
        for b in range(-ry, ry + 1):
            for a in range(-rx, rx + 1):
                d2 = (a * 0.5 * vx) ** 2 + (b * 0.5 * vy) ** 2 + (c * 0.5 * vz) ** 2
                if d2 > search_cm ** 2 * (1 + 1e-12):
                    continue
                pz, py, px = 2 * z + c, 2 * y + b, 2 * x + a
                ok = (pz >= 0) & (py >= 0) & (px >= 0) & (pz <= 2 * nz - 2) & (py <= 2 * ny - 2) & (px <= 2 * nx - 2)
                e = np.zeros_like(dr)
                e[ok] = U[pz[ok], py[ok], px[ok]]
                g2 = d2 / dta_cm ** 2 + (e - dr) ** 2 / (dose_frac * dmax) ** 2
                best = np.where(ok, np.minimum(best, g2), best)
    g = np.full(ref.shape, -1.0)
    g[sel] = np.sqrt(best)
    return g, float(np.mean(g[sel] <= 1.0)) if sel.any() else 0.0
