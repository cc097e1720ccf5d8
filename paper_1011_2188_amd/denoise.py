"""Learned denoising of low-history doses, trained on pairs the method makes.

Workflow (every numeric step runs in the library's kernels; torch only holds
device memory and cuts training crops):
  1. thorax-like plans with jittered anatomy and 1-3 fields (`denoise_plan`);
  2. for each plan a low-history dose and an independent high-history dose
     (the history counters continue, so the two never share a history);
  3. network input = (low dose / its Dmax, density / 2), target = high dose /
     the same Dmax; random crops train the U-Net (MSE, Adam) with the
     project's BF16 MFMA forward/backward kernels;
  4. evaluation: gamma pass rate (2%/2 mm, global, 10% cutoff) against an
     independent reference dose, plain vs denoised, and the histories each
     needs to reach the pass rate of the plain dose at 2% mean uncertainty.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import fdc as F
from . import inputs as I


def denoise_plan(seed, shape=(128, 128, 64), voxel_cm=0.4, e_range=(70.0, 200.0), spots=(200, 2000),
                 half_width_cm=3.0):
    """A thorax-like plan: the thorax anatomy scaled to the box, +-15% jitter of
    the body, lung and spine, 1-3 coplanar fields of spots on a square of half
    width half_width_cm at the right-lung centre.  Returns (phantom, spots)
    with n_histories = 1 per spot."""
    rng = np.random.default_rng([int(seed), 55])
    nx, ny, nz = shape
    sc = (nx * voxel_cm / 51.2, ny * voxel_cm / 51.2, nz * voxel_cm / 25.6)
    j = lambda: rng.uniform(0.85, 1.15)
    ph = I.thorax_phantom(shape, voxel_cm, seed=int(seed), scale=sc, body_axes=(17.0 * j(), 11.0 * j()),
                          lung_centre_x=7.0 * j(), lung_centre_y=-1.0 + rng.uniform(-1.0, 1.0),
                          lung_axes=(5.0 * j(), 7.0 * j(), 10.0 * j()), spine_centre_y=-8.0 * j(),
                          spine_radius=1.5 * j())
    n_fields = int(rng.integers(1, 4))
    gantries = rng.choice([0.0, 90.0, 180.0, 270.0], n_fields, replace=False)
    n_spots = int(rng.integers(spots[0], spots[1] + 1))
    iso = (7.0 * sc[0], -1.0 * sc[1], 0.0)
    per = np.diff(np.linspace(0, n_spots, n_fields + 1).astype(int))
    sp = np.concatenate([I.field_spots(iso, g, int(k), rng, half_width_cm=half_width_cm * sc[0], e_range=e_range,
                                       histories=np.ones(int(k), np.uint64)) for g, k in zip(gantries, per)])
    return ph, sp


class Simulator:
    """One library context running many plans; doses come back as device tensors."""

    def __init__(self, db, seed=1, launch=None, rotate=False):
        import torch
        self.torch = torch
        self.flags = F.FDC_RUN_ROTATE_TRACKS if rotate else 0
        self.ctx = F.Context(0, seed, table=I.HU_TABLE_DEFAULT)
        self.ctx.load_track_db(db)
        if launch:
            self.ctx.set_launch_config(**launch)
        self.per_pass = {}
        self.shape = {}

    def add(self, ph, sp, per_pass):
        """Load a plan whose spots share `per_pass` histories per pass."""
        sp = sp.copy()
        k = len(sp)
        base, extra = divmod(int(per_pass), k)
        sp["n_histories"] = base
        sp["n_histories"][:extra] += 1
        p = self.ctx.load_phantom(ph)
        self.ctx.add_beam_spots(p, sp)
        self.per_pass[p] = int(per_pass)
        self.shape[p] = ph.hu.shape
        return p

    def dose(self, plan, passes, variance=False):
        """Clear the tallies and run `passes` passes of NEW histories (the
        history counters continue, so successive doses are independent)."""
        torch = self.torch
        self.ctx.reset_plan(plan)
        flags = self.flags | (F.FDC_RUN_VARIANCE if variance else 0)
        for _ in range(int(passes)):
            self.ctx.run_histories([plan], flags)
        n = int(np.prod(self.shape[plan]))
        d = torch.empty(n, dtype=torch.float64, device="cuda")
        v = torch.empty(n, dtype=torch.float64, device="cuda") if variance else None
        self.ctx.compute_dose(plan, d, v)
        return d, v

    def density(self, plan):
        rho = self.torch.empty(int(np.prod(self.shape[plan])), dtype=self.torch.float32, device="cuda")
        self.ctx.density(plan, rho)
        return rho

    def net_input(self, plan, dose, rho):
        """(dose / Dmax, rho / 2) as a [2, nz, ny, nx] float32 tensor, and Dmax."""
        torch = self.torch
        _, _, dmax = self.ctx.mean_uncertainty(plan, dose, dose, 0.5)
        out = torch.empty((2,) + tuple(self.shape[plan]), dtype=torch.float32, device="cuda")
        self.ctx.denoise_input(plan, dose, rho, 1.0 / dmax if dmax > 0 else 1.0, out)
        return out, dmax

    def scaled(self, plan, dose, rho, dmax):
        """dose / dmax as a [nz, ny, nx] float32 tensor (the input kernel's channel 0)."""
        out = self.torch.empty((2,) + tuple(self.shape[plan]), dtype=self.torch.float32, device="cuda")
        self.ctx.denoise_input(plan, dose, rho, 1.0 / dmax if dmax > 0 else 1.0, out)
        return out[0]


def make_pairs(sim, plans, high_passes, levels=(1,)):
    """Per plan and input level k: (input [2,z,y,x], target [z,y,x]) float32
    device tensors; the input from k passes, the target from `high_passes`
    further passes, both divided by the input's Dmax (one target per level)."""
    pairs = []
    for p in plans:
        lows = [(k, sim.dose(p, k)[0]) for k in levels]
        high, _ = sim.dose(p, high_passes)
        rho = sim.density(p)
        for k, low in lows:
            x, dmax = sim.net_input(p, low, rho)
            pairs.append((x, sim.scaled(p, high, rho, dmax)))
    return pairs


def _dose_voxels(t, frac=0.1):
    """Flat indices of voxels above frac * max of a target (host copy, once per pair)."""
    a = t.detach().float().cpu().numpy().reshape(-1)
    m = float(a.max()) if a.size else 0.0
    return np.flatnonzero(a > frac * m) if m > 0 else np.zeros(0, np.int64)


def train(pairs, crop, steps, lr=1e-3, seed=0, init_params=None, log=None, log_every=200, focus=0.9,
          flips=True, lr_final=0.1):
    """Train on random crops (size `crop`, a tuple z, y, x) of the pairs.

    A crop is centred on a voxel of the target's dose region (> 10% of its
    maximum) with probability `focus`, else placed uniformly; with `flips`
    each crop is mirrored along random axes (a symmetry of transport in a
    mirrored phantom).  The learning rate decays on a cosine from lr to
    lr * lr_final."""
    import torch
    net = F.UNet(crop)
    if init_params is not None:
        net.set_params(init_params)
    else:
        net.init_params(seed)
    rng = np.random.default_rng(seed)
    hot = [_dose_voxels(t) for _, t in pairs]
    losses = []
    cz, cy, cx = crop
    t0 = time.perf_counter()
    for it in range(steps):
        k = int(rng.integers(len(pairs)))
        x, t = pairs[k]
        _, nz, ny, nx = x.shape
        if hot[k].size and rng.random() < focus:
            c = int(hot[k][int(rng.integers(hot[k].size))])
            centre = (c // (ny * nx), (c // nx) % ny, c % nx)
            z0, y0, x0 = (min(max(int(q) - s // 2 + int(rng.integers(-s // 4, s // 4 + 1)), 0), n - s)
                          for q, s, n in zip(centre, crop, (nz, ny, nx)))
        else:
            z0, y0, x0 = (int(rng.integers(0, n - c + 1)) for n, c in zip((nz, ny, nx), crop))
        xc = x[:, z0:z0 + cz, y0:y0 + cy, x0:x0 + cx]
        tc = t[z0:z0 + cz, y0:y0 + cy, x0:x0 + cx]
        if flips:
            axes = [a for a in (0, 1, 2) if rng.random() < 0.5]
            if axes:
                xc = torch.flip(xc, [a + 1 for a in axes])
                tc = torch.flip(tc, axes)
        want = (it % log_every == 0) or it == steps - 1
        loss = net.backward(xc.contiguous(), tc.contiguous(), want_loss=want)
        rate = lr * (lr_final + (1 - lr_final) * 0.5 * (1 + math.cos(math.pi * it / max(steps - 1, 1))))
        net.adam(rate)
        if want:
            losses.append((it, loss))
            if log:
                log(f"step {it} loss {loss:.4g} lr {rate:.3g} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return net, losses, time.perf_counter() - t0


def infer(params, x):
    """Denoised (normalised) dose of a full volume x [2, z, y, x]."""
    import torch
    net = F.UNet(tuple(x.shape[1:]))
    net.set_params(params)
    y = torch.empty(tuple(x.shape[1:]), dtype=torch.float32, device="cuda")
    net.forward(x, y)
    net.close()
    return y


# ---- the denoised route to the plain method's gamma pass rate -----------------

def with_total(sp, total):
    """The spots with `total` histories per run, split evenly (the first spots
    take the remainder)."""
    sp = sp.copy()
    base, extra = divmod(int(total), len(sp))
    sp["n_histories"] = base
    sp["n_histories"][:extra] += 1
    return sp


def plan_dose(ctx, ph, sp, total, flags=0):
    """A new plan of phantom ph with spots sp at `total` histories, run once;
    (plan id, dose, variance or None) as float64 device tensors.  A new plan id
    keys new random numbers, so doses of different plans are independent."""
    import torch
    p = ctx.load_phantom(ph)
    ctx.add_beam_spots(p, with_total(sp, total))
    ctx.run_histories([p], flags)
    n = ph.hu.size
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    v = torch.empty(n, dtype=torch.float64, device="cuda") if flags & F.FDC_RUN_VARIANCE else None
    ctx.compute_dose(p, d, v)
    return p, d, v


def normalised(ctx, plan, dose, rho, scale):
    """(dose * scale, rho / 2) as a [2, nz, ny, nx] float32 tensor (the network
    input, and with channel 0 alone a dose on the same normalisation)."""
    import torch
    shape = ctx.plans[plan]                          # (nz, ny, nx)
    out = torch.empty((2,) + tuple(shape), dtype=torch.float32, device="cuda")
    ctx.denoise_input(plan, dose, rho, scale, out)
    return out


def gamma_ladder(ctx, ph, sp, params, n2, rate, ref_total=400_000_000, rungs=7, plain=None, ref=None,
                 flags=F.FDC_RUN_ROTATE_TRACKS, log=None, above=0):
    """Seconds to the plain method's gamma pass rate, plain vs denoised.

    G* = gamma pass rate (2%/2 mm, global, 10% cutoff) of the plain dose of
    n2 histories (the histories to 2% mean uncertainty; `plain` = (plan, dose)
    if already run) against an independent reference of ref_total histories.
    The denoised dose is evaluated at N = n2 / 2^(rungs-1) ... n2 / 2, n2 (the
    ladder n2 * {1/64, ..., 1} for 7 rungs); N_d = the smallest N whose
    denoised dose reaches G*.  Times: histories / rate (the measured transport
    rate), plus the measured inference time for the denoised route.  Every rung
    is a new plan (independent histories); the plain dose of each rung is
    scored too.  `above` further rungs go past n2 (2 n2, 4 n2, ...): where the
    denoised route needs more histories than the plain one."""
    import torch
    if ref is None:
        pr, dref, _ = plan_dose(ctx, ph, sp, ref_total, flags)
    else:
        pr, dref = ref
    if plain is None:
        pp, dplain, _ = plan_dose(ctx, ph, sp, int(round(n2)), flags)
    else:
        pp, dplain = plain
    rho = torch.empty(ph.hu.size, dtype=torch.float32, device="cuda")
    ctx.density(pp, rho)
    g_star = ctx.gamma_index(pp, dref, dplain)[0]
    net = F.UNet(tuple(ph.hu.shape))
    net.set_params(params)
    y = torch.empty(tuple(ph.hu.shape), dtype=torch.float32, device="cuda")
    rows, n_d, t_inf_best = [], None, None
    for j in range(rungs + above):
        n = max(1, int(round(n2 * 2.0 ** (j - (rungs - 1)))))
        p, d, _ = plan_dose(ctx, ph, sp, n, flags)
        _, _, dmax = ctx.mean_uncertainty(p, d, d, 0.5)
        scale = 1.0 / dmax if dmax > 0 else 1.0
        x = normalised(ctx, p, d, rho, scale)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net.forward(x, y)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t0
        t_inf_best = t_inf if t_inf_best is None else min(t_inf_best, t_inf)
        r = normalised(ctx, p, dref, rho, scale)[0].reshape(-1).double()
        g_den = ctx.gamma_index(p, r, y.reshape(-1).double())[0]
        g_plain = ctx.gamma_index(p, r, x[0].reshape(-1).double())[0]
        rows.append({"histories": n, "gamma_denoised": g_den, "gamma_plain": g_plain, "inference_s": t_inf})
        if log:
            log(f"  rung {j}: {n} histories, gamma denoised {g_den:.5f} plain {g_plain:.5f} (G* {g_star:.5f})")
        if n_d is None and g_den >= g_star:
            n_d = (n, t_inf)
    net.close()
    return {"N_2pct": n2, "G_star": g_star, "reference_histories": ref_total, "t_plain_s": n2 / rate,
            "ladder": rows, "N_denoised": n_d[0] if n_d else None,
            "t_denoised_s": (n_d[0] / rate + n_d[1]) if n_d else None, "inference_s": t_inf_best}


def save_params(path, params, meta):
    """Network parameters (float32) and a JSON description, as an .npz (no pickles)."""
    import json
    np.savez(path, params=np.asarray(params, np.float32), meta=np.frombuffer(json.dumps(meta).encode(), np.uint8))


def load_params(path):
    """(params float32, meta dict) from save_params' file."""
    import json
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32), json.loads(bytes(z["meta"]).decode())
