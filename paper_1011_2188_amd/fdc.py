"""Thin Python binding of libfdc.so (include/fdc.h).

Argument marshalling only: every step of the dose calculation runs in the
library's HIP kernels.  The library must have been built (`build.build()` or
`__graft_entry__.build()`); importing this module without it raises - there is
no fallback path.

The module-level functions carry the C names (`fdc_create`, `fdc_run_histories`
...) and take/return plain ctypes values; `Context` wraps them for numpy inputs
and torch device tensors.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfdc.so")

FDC_OK, FDC_E_ARG, FDC_E_STATE, FDC_E_NOMEM, FDC_E_HIP, FDC_E_RANGE, FDC_E_FORMAT, FDC_E_OVERFLOW = \
    0, -1, -2, -3, -4, -5, -6, -7
FDC_NO_DEVICE = -1
FDC_RUN_VARIANCE = 1
FDC_RUN_ROTATE_TRACKS = 2
FDC_RUN_COUNT_WORK = 4
ERROR_NAMES = {0: "FDC_OK", -1: "FDC_E_ARG", -2: "FDC_E_STATE", -3: "FDC_E_NOMEM", -4: "FDC_E_HIP",
               -5: "FDC_E_RANGE", -6: "FDC_E_FORMAT", -7: "FDC_E_OVERFLOW"}

# every entry point declared in include/fdc.h
EXPORTS = ["fdc_create", "fdc_destroy", "fdc_last_error", "fdc_set_allocator", "fdc_set_hu_table",
           "fdc_load_track_db", "fdc_load_secondaries", "fdc_load_track_db_file", "fdc_load_phantom", "fdc_add_beam_spots", "fdc_add_phase_space",
           "fdc_add_phase_space_file", "fdc_add_beam_device", "fdc_set_spot_device", "fdc_run_histories",
           "fdc_run_histories_noalloc", "fdc_prepare_run",
           "fdc_reset_plan", "fdc_read_work_counts", "fdc_plan_state_bytes", "fdc_save_plan_state",
           "fdc_restore_plan_state", "fdc_compute_dose", "fdc_read_dose_and_variance", "fdc_debug_endpoints",
           "fdc_debug_philox", "fdc_debug_material", "fdc_set_launch_config", "fdc_device_cus",
           "fdc_mean_uncertainty", "fdc_batch_uncertainty", "fdc_gamma_index",
           "fdc_graph_create", "fdc_graph_launch", "fdc_graph_destroy",
           "fdc_unet_num_params", "fdc_unet_create", "fdc_unet_destroy", "fdc_unet_last_error",
           "fdc_unet_set_params", "fdc_unet_get_params", "fdc_unet_get_grads", "fdc_unet_forward",
           "fdc_unet_backward", "fdc_unet_adam", "fdc_unet_debug_buffer", "fdc_density", "fdc_denoise_input",
           "fdc_unet_init_params", "fdc_set_timing", "fdc_transport_times"]
FDC_GRAPH_RESET_TALLIES = 1
FDC_GRAPH_DOSE = 2


class fdc_summary(C.Structure):
    _fields_ = [("n_histories", C.c_uint64), ("incident_fp", C.c_int64),
                ("deposited_fp", C.c_int64), ("escaped_fp", C.c_int64)]


class fdc_beam_device(C.Structure):
    _fields_ = [("origin_cm", C.c_float * 3), ("dir", C.c_float * 3), ("pitch_cm", C.c_float * 2),
                ("n", C.c_uint32 * 2), ("rsp", C.c_float), ("rscp", C.c_float)]


class fdc_launch_config(C.Structure):
    _fields_ = [("waves_per_block", C.c_uint32), ("blocks_per_cu", C.c_uint32),
                ("tally_slots", C.c_uint32), ("units_per_wave", C.c_uint32),
                ("tally_mode", C.c_uint32), ("source_order", C.c_uint32),
                ("reserved", C.c_uint32 * 2)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class FdcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None
_P = C.c_void_p


def lib():
    """Load libfdc.so; raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (paper_1011_2188_amd.build.build())")
    L = C.CDLL(LIB_PATH)
    sig = {
        "fdc_create": (C.c_int, [C.POINTER(_P), C.c_int, C.c_uint64, C.c_uint32]),
        "fdc_destroy": (C.c_int, [_P]),
        "fdc_last_error": (C.c_char_p, [_P]),
        "fdc_set_allocator": (C.c_int, [_P, ALLOC_FN, FREE_FN, _P]),
        "fdc_set_hu_table": (C.c_int, [_P, _P, _P, _P, _P, C.c_int, C.c_float]),
        "fdc_load_track_db": (C.c_int, [_P, _P, C.c_uint64, _P, C.c_uint32, _P, _P, C.c_uint32, _P]),
        "fdc_load_secondaries": (C.c_int, [_P, _P, _P, C.c_uint32, _P, C.c_uint64, _P, _P, _P]),
        "fdc_load_track_db_file": (C.c_int, [_P, C.c_char_p, _P]),
        "fdc_load_phantom": (C.c_int, [_P, C.POINTER(C.c_int32), _P, C.c_int, C.c_int, C.c_int, _P, _P, _P]),
        "fdc_add_beam_spots": (C.c_int, [_P, C.c_int32, _P, C.c_uint32]),
        "fdc_add_phase_space": (C.c_int, [_P, C.c_int32, _P, C.c_uint64, C.POINTER(C.c_uint32), _P]),
        "fdc_add_phase_space_file": (C.c_int, [_P, C.c_int32, C.c_char_p, C.POINTER(C.c_uint32), _P]),
        "fdc_add_beam_device": (C.c_int, [_P, C.POINTER(fdc_beam_device), _P, C.POINTER(C.c_int32), _P]),
        "fdc_set_spot_device": (C.c_int, [_P, C.c_int32, C.c_uint32, C.c_uint32, C.c_int32]),
        "fdc_run_histories": (C.c_int, [_P, _P, C.c_uint32, C.c_uint32, _P]),
        "fdc_run_histories_noalloc": (C.c_int, [_P, _P, C.c_uint32, C.c_uint32, _P]),
        "fdc_prepare_run": (C.c_int, [_P]),
        "fdc_reset_plan": (C.c_int, [_P, C.c_int32, C.c_int, _P]),
        "fdc_read_work_counts": (C.c_int, [_P, C.c_int32, _P, _P]),
        "fdc_plan_state_bytes": (C.c_int, [_P, C.c_int32, _P]),
        "fdc_save_plan_state": (C.c_int, [_P, C.c_int32, _P, C.c_uint64, _P]),
        "fdc_restore_plan_state": (C.c_int, [_P, C.c_int32, _P, C.c_uint64, _P]),
        "fdc_compute_dose": (C.c_int, [_P, C.c_int32, _P, _P, _P]),
        "fdc_read_dose_and_variance": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, C.POINTER(fdc_summary), _P]),
        "fdc_debug_endpoints": (C.c_int, [_P, C.c_int32, C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32,
                                          _P, _P, _P]),
        "fdc_debug_philox": (C.c_int, [_P, _P, _P, C.c_uint32, _P]),
        "fdc_debug_material": (C.c_int, [_P, _P, _P, _P, _P]),
        "fdc_set_launch_config": (C.c_int, [_P, C.POINTER(fdc_launch_config)]),
        "fdc_device_cus": (C.c_int, [_P, C.POINTER(C.c_int)]),
        "fdc_set_timing": (C.c_int, [_P, C.c_int]),
        "fdc_transport_times": (C.c_int, [_P, C.POINTER(C.c_float), C.c_uint32]),
        "fdc_mean_uncertainty": (C.c_int, [_P, C.c_int32, _P, _P, C.c_double, C.POINTER(C.c_double),
                                           C.POINTER(C.c_uint64), C.POINTER(C.c_double), _P]),
        "fdc_batch_uncertainty": (C.c_int, [_P, _P, C.c_uint32, C.c_uint64, _P, _P, _P]),
        "fdc_graph_create": (C.c_int, [_P, _P, C.c_uint32, C.c_uint32, C.c_uint32, _P, _P, C.POINTER(_P)]),
        "fdc_graph_launch": (C.c_int, [_P, _P]),
        "fdc_graph_destroy": (C.c_int, [_P]),
        "fdc_density": (C.c_int, [_P, C.c_int32, _P, _P]),
        "fdc_denoise_input": (C.c_int, [_P, C.c_int32, _P, _P, C.c_double, _P, _P]),
        "fdc_unet_num_params": (C.c_int64, []),
        "fdc_unet_create": (C.c_int, [C.POINTER(_P), C.c_int, C.c_int, C.c_int, C.c_int]),
        "fdc_unet_destroy": (C.c_int, [_P]),
        "fdc_unet_last_error": (C.c_char_p, [_P]),
        "fdc_unet_set_params": (C.c_int, [_P, _P, _P]),
        "fdc_unet_init_params": (C.c_int, [_P, C.c_uint64, _P]),
        "fdc_unet_get_params": (C.c_int, [_P, _P, _P]),
        "fdc_unet_get_grads": (C.c_int, [_P, _P, _P]),
        "fdc_unet_forward": (C.c_int, [_P, _P, _P, _P]),
        "fdc_unet_backward": (C.c_int, [_P, _P, _P, _P, C.POINTER(C.c_double), _P]),
        "fdc_unet_adam": (C.c_int, [_P, C.c_float, C.c_float, C.c_float, C.c_float, _P]),
        "fdc_unet_debug_buffer": (C.c_int, [_P, C.c_int, _P, C.POINTER(C.c_int64), C.POINTER(C.c_int32), _P]),
        "fdc_gamma_index": (C.c_int, [_P, C.c_int32, _P, _P, C.c_double, C.c_double, C.c_double, C.c_double,
                                      _P, C.POINTER(C.c_double), C.POINTER(C.c_uint64), _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if not a.flags.c_contiguous:
            raise ValueError("array arguments must be C-contiguous")
        return a.ctypes.data
    if not a.is_contiguous():   # torch tensor
        raise ValueError("tensor arguments must be contiguous")
    return a.data_ptr()


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                return torch.cuda.current_stream().cuda_stream
        except ImportError:
            pass
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---- C-named wrappers (argument marshalling only) -------------------------
def fdc_create(hip_device, seed, reuse_R):
    h = _P()
    rc = lib().fdc_create(C.byref(h), hip_device, seed, reuse_R)
    return rc, h


def fdc_last_error(ctx):
    m = lib().fdc_last_error(ctx)
    return m.decode() if m else ""


def _check(ctx, rc):
    if rc != FDC_OK:
        raise FdcError(rc, fdc_last_error(ctx))


class Graph:
    """A captured run (fdc_graph_*); launch() enqueues one replay."""

    def __init__(self, ctx, handle, keep):
        self.ctx, self.h, self._keep = ctx, handle, keep

    def launch(self, stream=None):
        _check(self.ctx.h, lib().fdc_graph_launch(self.h, _stream(stream)))

    def close(self):
        if self.h:
            lib().fdc_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One libfdc context (one device).  Inputs are numpy arrays on the host
    (copied by the loaders); dose outputs are numpy or torch device tensors."""

    def __init__(self, device=0, seed=1, reuse_R=64, torch_allocator=False, table=None):
        rc, h = fdc_create(device, seed, reuse_R)
        if rc != FDC_OK:
            raise FdcError(rc, f"fdc_create(device={device}) failed")
        self.h = h
        self.device = device
        self.plans = {}           # plan id -> shape (nz, ny, nx)
        self._keep = []
        self._graphs = []
        if torch_allocator:
            self._use_torch_allocator()
        if table is not None:
            self.set_hu_table(table)

    # -- lifetime
    def close(self):
        if self.h:
            for g in self._graphs:
                g.close()
            lib().fdc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _use_torch_allocator(self):
        import torch
        live = {}
        dev = torch.device("cuda", self.device)

        def _alloc(n, user):
            try:
                t = torch.empty(int(n), dtype=torch.uint8, device=dev)
            except RuntimeError:
                return None
            live[t.data_ptr()] = t
            return t.data_ptr()

        def _free(p, user):
            live.pop(p, None)

        fa, ff = ALLOC_FN(_alloc), FREE_FN(_free)
        self._keep += [fa, ff, live]
        _check(self.h, lib().fdc_set_allocator(self.h, fa, ff, None))

    # -- inputs
    def set_hu_table(self, t):
        cols = [np.ascontiguousarray(t[k], np.float32) for k in ("hu", "rho", "rsp", "rscp")]
        _check(self.h, lib().fdc_set_hu_table(self.h, *[c.ctypes.data for c in cols], cols[0].size,
                                              float(t["vacuum_below_hu"])))

    def load_track_db(self, db, stream=None):
        steps = np.ascontiguousarray(db.steps, np.float32)
        off = np.ascontiguousarray(db.track_off, np.uint64)
        be = np.ascontiguousarray(db.bin_E, np.float32)
        bf = np.ascontiguousarray(db.bin_first, np.uint32)
        _check(self.h, lib().fdc_load_track_db(self.h, steps.ctypes.data, steps.shape[0], off.ctypes.data,
                                               off.size - 1, be.ctypes.data, bf.ctypes.data, be.size,
                                               _stream(stream)))
        if getattr(db, "sec", None) is not None:
            self.load_secondaries(db.sec, stream)

    def load_secondaries(self, sec, stream=None):
        """The database's secondary trajectories (inputs.Secondaries)."""
        first = np.ascontiguousarray(sec.sec_first, np.uint32)
        off = np.ascontiguousarray(sec.off, np.uint64)
        st = np.ascontiguousarray(sec.steps, np.float32).reshape(-1, 4)
        br = np.ascontiguousarray(sec.branch, np.uint32)
        em = np.ascontiguousarray(sec.emit, np.float32).reshape(-1, 2)
        _check(self.h, lib().fdc_load_secondaries(self.h, first.ctypes.data, off.ctypes.data, br.size,
                                                  st.ctypes.data, st.shape[0], br.ctypes.data, em.ctypes.data,
                                                  _stream(stream)))

    def load_track_db_file(self, path, stream=None):
        _check(self.h, lib().fdc_load_track_db_file(self.h, os.fsencode(path), _stream(stream)))

    def load_phantom(self, ph, stream=None):
        hu = np.ascontiguousarray(ph.hu, np.int16)
        nz, ny, nx = hu.shape
        vox = np.ascontiguousarray(ph.voxel_cm, np.float32)
        org = np.ascontiguousarray(ph.origin_cm, np.float32)
        plan = C.c_int32()
        _check(self.h, lib().fdc_load_phantom(self.h, C.byref(plan), hu.ctypes.data, nx, ny, nz,
                                              vox.ctypes.data, org.ctypes.data, _stream(stream)))
        self.plans[plan.value] = (nz, ny, nx)
        return plan.value

    def add_beam_spots(self, plan, spots):
        from .inputs import SPOT_DTYPE
        s = np.ascontiguousarray(spots, SPOT_DTYPE)
        _check(self.h, lib().fdc_add_beam_spots(self.h, plan, s.ctypes.data, s.size))

    def add_beam_device(self, dev, stream=None):
        """A beam-line device (a dict from inputs.beam_device); returns its id."""
        d = fdc_beam_device()
        d.origin_cm[:] = [float(x) for x in dev["origin_cm"]]
        d.dir[:] = [float(x) for x in dev["dir"]]
        d.pitch_cm[:] = [float(x) for x in dev["pitch_cm"]]
        d.n[:] = [int(x) for x in dev["n"]]
        d.rsp, d.rscp = float(dev["rsp"]), float(dev["rscp"])
        pix = np.ascontiguousarray(dev["pixels"], np.float32)
        out = C.c_int32()
        _check(self.h, lib().fdc_add_beam_device(self.h, C.byref(d), pix.ctypes.data, C.byref(out), _stream(stream)))
        return out.value

    def set_spot_device(self, plan, first_spot, n_spots, device):
        _check(self.h, lib().fdc_set_spot_device(self.h, plan, first_spot, n_spots, device))

    def add_phase_space(self, plan, particles, stream=None):
        """Listed incident protons (inputs.PARTICLE_DTYPE); returns the number of
        sources (energy-bin groups) added to the plan."""
        from .inputs import PARTICLE_DTYPE
        q = np.ascontiguousarray(particles, PARTICLE_DTYPE)
        n = C.c_uint32()
        _check(self.h, lib().fdc_add_phase_space(self.h, plan, q.ctypes.data, q.size, C.byref(n), _stream(stream)))
        return n.value

    def add_phase_space_file(self, plan, path, stream=None):
        n = C.c_uint32()
        _check(self.h, lib().fdc_add_phase_space_file(self.h, plan, os.fsencode(path), C.byref(n), _stream(stream)))
        return n.value

    # -- the method
    def run_histories(self, plans, flags=FDC_RUN_VARIANCE, stream=None):
        p = np.ascontiguousarray(np.atleast_1d(plans), np.int32)
        _check(self.h, lib().fdc_run_histories(self.h, p.ctypes.data, p.size, flags, _stream(stream)))

    def run_histories_noalloc(self, plans, flags=FDC_RUN_VARIANCE, stream=None):
        p = np.ascontiguousarray(np.atleast_1d(plans), np.int32)
        _check(self.h, lib().fdc_run_histories_noalloc(self.h, p.ctypes.data, p.size, flags, _stream(stream)))

    def prepare_run(self):
        _check(self.h, lib().fdc_prepare_run(self.h))

    def save_plan_state(self, plan, stream=None):
        """The plan's state (tallies, summary, history counters) as bytes."""
        n = C.c_uint64()
        _check(self.h, lib().fdc_plan_state_bytes(self.h, plan, C.byref(n)))
        buf = np.empty(n.value, np.uint8)
        _check(self.h, lib().fdc_save_plan_state(self.h, plan, buf.ctypes.data, buf.size, _stream(stream)))
        return buf.tobytes()

    def restore_plan_state(self, plan, state, stream=None):
        buf = np.frombuffer(state, np.uint8)
        _check(self.h, lib().fdc_restore_plan_state(self.h, plan, buf.ctypes.data, buf.size, _stream(stream)))

    def read_work_counts(self, plan, stream=None):
        """Steps, non-vacuum voxel pieces and flushes of the plan's runs with
        FDC_RUN_COUNT_WORK since its last reset."""
        out = np.zeros(3, np.uint64)
        _check(self.h, lib().fdc_read_work_counts(self.h, plan, out.ctypes.data, _stream(stream)))
        return dict(steps=int(out[0]), visits=int(out[1]), flushes=int(out[2]))

    def reset_plan(self, plan, rewind=False, stream=None):
        _check(self.h, lib().fdc_reset_plan(self.h, plan, int(bool(rewind)), _stream(stream)))

    def compute_dose(self, plan, dose=None, var=None, stream=None):
        """Into torch float64 device tensors (either may be None)."""
        _check(self.h, lib().fdc_compute_dose(self.h, plan, _ptr(dose), _ptr(var), _stream(stream)))

    def read_dose_and_variance(self, plan, dose=True, var=True, raw=False, stream=None):
        shape = self.plans[plan]
        out = {}
        d = np.empty(shape, np.float64) if dose else None
        v = np.empty(shape, np.float64) if var else None
        e = np.empty(shape, np.int64) if raw else None
        e2 = np.empty(shape, np.uint64) if raw else None
        s = fdc_summary()
        _check(self.h, lib().fdc_read_dose_and_variance(self.h, plan, _ptr(d), _ptr(v), _ptr(e), _ptr(e2),
                                                        C.byref(s), _stream(stream)))
        out.update(dose=d, var=v, E=e, E2=e2, n_histories=s.n_histories, incident=s.incident_fp,
                   deposited=s.deposited_fp, escaped=s.escaped_fp)
        return out

    # -- testing aids
    def debug_endpoints(self, plan, spot, h0, n, flags=0, stream=None):
        xyz = np.empty((n, 3), np.float32)
        why = np.empty(n, np.int32)
        _check(self.h, lib().fdc_debug_endpoints(self.h, plan, spot, h0, n, flags, xyz.ctypes.data,
                                                 why.ctypes.data, _stream(stream)))
        return xyz, why

    def debug_philox(self, ctr, stream=None):
        c = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
        out = np.empty_like(c)
        _check(self.h, lib().fdc_debug_philox(self.h, c.ctypes.data, out.ctypes.data, c.shape[0], _stream(stream)))
        return out

    def debug_material(self, stream=None):
        rsp, g, rho = (np.empty(4096, np.float32) for _ in range(3))
        _check(self.h, lib().fdc_debug_material(self.h, rsp.ctypes.data, g.ctypes.data, rho.ctypes.data,
                                                _stream(stream)))
        return rsp, g, rho

    def set_launch_config(self, waves_per_block=4, blocks_per_cu=0, tally_slots=0, units_per_wave=0, tally_mode=0,
                          source_order=0):
        cfg = fdc_launch_config(waves_per_block, blocks_per_cu, tally_slots, units_per_wave, tally_mode, source_order)
        _check(self.h, lib().fdc_set_launch_config(self.h, C.byref(cfg)))

    # -- graphs
    def graph_create(self, plans, flags=FDC_RUN_VARIANCE, reset=True, doses=None, variances=None):
        """Capture a run over `plans` (optionally clearing tallies first and
        writing dose/variance into the given torch device tensors after)."""
        p = np.ascontiguousarray(np.atleast_1d(plans), np.int32)
        opts = (FDC_GRAPH_RESET_TALLIES if reset else 0) | (FDC_GRAPH_DOSE if (doses or variances) else 0)
        dp = (C.c_void_p * p.size)(*[_ptr(d) for d in doses]) if doses else None
        vp = (C.c_void_p * p.size)(*[_ptr(v) for v in variances]) if variances else None
        g = _P()
        _check(self.h, lib().fdc_graph_create(self.h, p.ctypes.data, p.size, flags, opts,
                                              C.cast(dp, _P) if dp is not None else None,
                                              C.cast(vp, _P) if vp is not None else None, C.byref(g)))
        gr = Graph(self, g, (doses, variances))
        self._graphs.append(gr)
        return gr

    def density(self, plan, rho, stream=None):
        _check(self.h, lib().fdc_density(self.h, plan, _ptr(rho), _stream(stream)))

    def denoise_input(self, plan, dose, rho, scale, out, stream=None):
        _check(self.h, lib().fdc_denoise_input(self.h, plan, _ptr(dose), _ptr(rho), float(scale), _ptr(out),
                                               _stream(stream)))

    # -- metrics (device arrays in, host scalars out)
    def mean_uncertainty(self, plan, dose, var, frac=0.5, stream=None):
        m, n, dmax = C.c_double(), C.c_uint64(), C.c_double()
        _check(self.h, lib().fdc_mean_uncertainty(self.h, plan, _ptr(dose), _ptr(var), frac, C.byref(m),
                                                  C.byref(n), C.byref(dmax), _stream(stream)))
        return m.value, n.value, dmax.value

    def batch_uncertainty(self, doses, mean=None, sigma=None, stream=None):
        """doses: torch float64 device tensor [n_batches, n_vox]."""
        _check(self.h, lib().fdc_batch_uncertainty(self.h, _ptr(doses), doses.shape[0], doses[0].numel(),
                                                   _ptr(mean), _ptr(sigma), _stream(stream)))

    def gamma_index(self, plan, ref, ev, dose_frac=0.02, dta_cm=0.2, cutoff_frac=0.1, search_cm=0.6,
                    gamma=None, stream=None):
        rate, n = C.c_double(), C.c_uint64()
        _check(self.h, lib().fdc_gamma_index(self.h, plan, _ptr(ref), _ptr(ev), dose_frac, dta_cm, cutoff_frac,
                                             search_cm, _ptr(gamma), C.byref(rate), C.byref(n), _stream(stream)))
        return rate.value, n.value

    def device_cus(self):
        n = C.c_int()
        _check(self.h, lib().fdc_device_cus(self.h, C.byref(n)))
        return n.value

    def set_timing(self, on=True):
        """Time the transport kernel of every following run (HIP events)."""
        _check(self.h, lib().fdc_set_timing(self.h, int(bool(on))))

    def transport_times(self, n):
        """Kernel milliseconds of the last n timed runs, oldest first."""
        out = np.zeros(n, np.float32)
        _check(self.h, lib().fdc_transport_times(self.h, out.ctypes.data_as(C.POINTER(C.c_float)), n))
        return out


UNET_BUFFERS = ["x", "e1a", "c1", "p1", "e2a", "c2", "p2", "ma", "m", "d2a", "d2", "d1a", "d1",
                "gd1", "gd1a", "gc1", "gd2", "gd2a", "gc2", "gm", "gma", "gp2", "ge2", "ge2a", "gp1", "ge1", "ge1a"]


class UNet:
    """The dose denoiser (fdc_unet_*): volumes of nz x ny x nx voxels."""

    def __init__(self, shape_zyx, device=0):
        nz, ny, nx = shape_zyx
        h = _P()
        rc = lib().fdc_unet_create(C.byref(h), device, nx, ny, nz)
        if rc != FDC_OK:
            raise FdcError(rc, f"fdc_unet_create({nx}, {ny}, {nz}) failed")
        self.h, self.shape = h, (nz, ny, nx)
        self.n_params = int(lib().fdc_unet_num_params())

    def _check(self, rc):
        if rc != FDC_OK:
            m = lib().fdc_unet_last_error(self.h)
            raise FdcError(rc, m.decode() if m else "")

    def close(self):
        if self.h:
            lib().fdc_unet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat, stream=None):
        v = np.ascontiguousarray(flat, np.float32)
        assert v.size == self.n_params
        self._check(lib().fdc_unet_set_params(self.h, v.ctypes.data, _stream(stream)))

    def init_params(self, seed, stream=None):
        self._check(lib().fdc_unet_init_params(self.h, seed, _stream(stream)))

    def get_params(self, stream=None):
        v = np.empty(self.n_params, np.float32)
        self._check(lib().fdc_unet_get_params(self.h, v.ctypes.data, _stream(stream)))
        return v

    def get_grads(self, stream=None):
        v = np.empty(self.n_params, np.float32)
        self._check(lib().fdc_unet_get_grads(self.h, v.ctypes.data, _stream(stream)))
        return v

    def forward(self, inp, out, stream=None):
        """inp: torch float32 [2, nz, ny, nx] on the device; out: [nz, ny, nx]."""
        self._check(lib().fdc_unet_forward(self.h, _ptr(inp), _ptr(out), _stream(stream)))

    def backward(self, inp, target, out=None, want_loss=True, stream=None):
        loss = C.c_double()
        self._check(lib().fdc_unet_backward(self.h, _ptr(inp), _ptr(target), _ptr(out),
                                            C.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self._check(lib().fdc_unet_adam(self.h, lr, beta1, beta2, eps, _stream(stream)))

    def debug_buffer(self, name, stream=None):
        """Internal bf16 buffer as float32 [voxels, pitch] (channels-last)."""
        i = UNET_BUFFERS.index(name)
        n, pitch = C.c_int64(), C.c_int32()
        self._check(lib().fdc_unet_debug_buffer(self.h, i, None, C.byref(n), C.byref(pitch), None))
        raw = np.empty(n.value * pitch.value, np.uint16)
        self._check(lib().fdc_unet_debug_buffer(self.h, i, raw.ctypes.data, C.byref(n), C.byref(pitch),
                                                _stream(stream)))
        return (raw.astype(np.uint32) << 16).view(np.float32).reshape(n.value, pitch.value)
