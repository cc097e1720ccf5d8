"""Measurements beyond the benchmark's main line (run on one GPU):

  thorax_rate       histories/s on the 1e8-history synthetic thorax plan;
  paper_field_rate  the same on the paper's own kind of test case (121 MeV
                    field of circular cross-section, 1 x 1 x 2.5 mm voxels);
  batched           64 thorax-like plans in ONE captured graph launch vs 64
                    separate eager runs (same histories, same tallies);
  denoiser_study    seconds to 2% mean uncertainty, plain vs denoised at equal
                    gamma pass rate (2%/2 mm) against an independent reference;
  recycling_study   the database-recycling test of Section 3: mean uncertainty
                    against N with the history-by-history estimator (Eq. 2)
                    and with fully independent batches (Eq. 1), for several
                    track reuse factors R;
  denoiser_rate     the denoiser's forward pass over a 256x256x128 volume and
                    its training step on a 128^3 crop.

`python -m paper_1011_2188_amd.experiments denoiser [--reps K]` prints the
denoiser timings, one line per call, then a JSON summary.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import autotune as A
from . import denoise as D
from . import fdc as F
from . import inputs as I
from . import workloads as W


def _sync():
    import torch
    torch.cuda.synchronize()


def thorax_rate(db, reps=2, tune=True, log=print):
    ph, sp, _ = W.thorax()
    return workload_rate(ph, sp, db, reps, tune, log, "thorax")


def paper_field_rate(reps=2, tune=True, log=print, total=10_000_000):
    """The paper's test case with synthetic anatomy (Section 2.5): 121 MeV disk
    field of 4 cm radius on 1 x 1 x 2.5 mm voxels."""
    ph, sp, db = W.paper_field(total)
    return workload_rate(ph, sp, db, reps, tune, log, "paper field")


def workload_rate(ph, sp, db, reps=2, tune=True, log=print, name="workload"):
    """Histories/s of one plan (both tallies, dose included), its mean
    uncertainty and the seconds to 2% it implies (Eq. (2))."""
    import torch
    c = F.Context(0, 1, table=I.HU_TABLE_DEFAULT)
    c.load_track_db(db)
    p = c.load_phantom(ph)
    c.add_beam_spots(p, sp)
    cfg = A.tune(c, [p], F.FDC_RUN_VARIANCE, reps=1, log=None)[0] if tune else {}
    n = int(sp["n_histories"].sum())
    d = torch.empty(ph.hu.size, dtype=torch.float64, device="cuda")
    v = torch.empty(ph.hu.size, dtype=torch.float64, device="cuda")
    best = math.inf
    for _ in range(reps):
        c.reset_plan(p)
        _sync()
        t = time.perf_counter()
        c.run_histories([p], F.FDC_RUN_VARIANCE)
        c.compute_dose(p, d, v)
        _sync()
        best = min(best, time.perf_counter() - t)
    u, _, _ = c.mean_uncertainty(p, d, v, 0.5)
    n2 = n * (u / 0.02) ** 2
    out = {"histories": n, "seconds": best, "histories_per_s": n / best, "launch": cfg,
           "mean_uncertainty": u, "seconds_to_2pct": n2 / (n / best)}
    log(f"{name}: {out}")
    c.close()
    return out


def batched(db, log=print, hist_scale=1.0):
    """64 plans: one graph launch (all plans, tallies cleared, dose computed)
    against 64 separate eager runs of the same plans in a second context."""
    import torch
    plans = W.batched_plans(64, hist_scale=hist_scale)
    ctxs = []
    for k in range(2):
        c = F.Context(0, 1, table=I.HU_TABLE_DEFAULT)
        c.load_track_db(db)
        ids = []
        for ph, sp in plans:
            p = c.load_phantom(ph)
            c.add_beam_spots(p, sp)
            ids.append(p)
        ctxs.append((c, ids))
    (cg, ids), (ce, ide) = ctxs
    # the launch configuration both sides run, tuned on the whole batch (a
    # launch of several plans takes the rounds cache; the start-position order
    # is captured in the graph like the rest)
    cfg, _ = A.tune(cg, ids, F.FDC_RUN_VARIANCE, reps=1, candidates=A.CANDIDATES, use_cache=False)
    ce.set_launch_config(**cfg)
    doses = [torch.empty(ph.hu.size, dtype=torch.float64, device="cuda") for ph, _ in plans]
    vars_ = [torch.empty(ph.hu.size, dtype=torch.float64, device="cuda") for ph, _ in plans]
    g = cg.graph_create(ids, F.FDC_RUN_VARIANCE, reset=True, doses=doses, variances=vars_)
    n_hist = sum(int(sp["n_histories"].sum()) for _, sp in plans)
    g.launch()
    _sync()
    t = time.perf_counter()
    g.launch()
    _sync()
    t_graph = time.perf_counter() - t
    for p in ide:                                  # warm-up pass, then the timed one
        ce.run_histories([p], F.FDC_RUN_VARIANCE)
    _sync()
    for p in ide:
        ce.reset_plan(p)
    _sync()
    t = time.perf_counter()
    for p, d, v in zip(ide, doses, vars_):
        ce.run_histories([p], F.FDC_RUN_VARIANCE)
        ce.compute_dose(p, d, v)
    _sync()
    t_sep = time.perf_counter() - t
    # same histories on both sides (second pass of each context): tallies equal
    same = all(np.array_equal(cg.read_dose_and_variance(a, dose=False, var=False, raw=True)["E"],
                              ce.read_dose_and_variance(b, dose=False, var=False, raw=True)["E"])
               for a, b in zip(ids[:4], ide[:4]))
    out = {"plans": len(plans), "histories": n_hist, "graph_seconds": t_graph, "separate_seconds": t_sep,
           "graph_histories_per_s": n_hist / t_graph, "separate_histories_per_s": n_hist / t_sep,
           "launch": cfg, "first_plans_bitwise_equal": bool(same)}
    log(f"batched: {out}")
    g.close()
    cg.close()
    ce.close()
    return out


def denoiser_study(db, n_train=128, n_test=6, shape=(256, 256, 128), voxel_cm=0.2, per_pass=1_000_000,
                   high_passes=100, crop=(128, 128, 128), steps=6000, lr=1e-3, log=print, levels=(1, 2, 4),
                   launch=dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=1, tally_mode=1),
                   step_passes=2):
    """Plain vs denoised seconds to 2% at equal gamma pass rate (2%/2 mm).

    Training pairs: k passes (per_pass histories each, k in `levels`) as input,
    high_passes further passes as target, track rotation on.  For each held-out plan: N_2% from
    the Eq. (2) mean uncertainty of one pass; the plain dose at N_2% and its
    gamma pass rate G* against an independent reference of
    4 * N_2% + high_passes * per_pass histories; the denoised dose at k passes,
    k = 1, 2, 4, ... (or 1, 2, 3, ... with step_passes=1) up to the passes of
    N_2%, until its pass rate reaches G*.
    Times = histories / the measured transport rate (+ inference)."""
    import torch
    sim = D.Simulator(db, seed=7, rotate=True, launch=launch)
    plans = []
    t = time.perf_counter()
    for k in range(n_train + n_test):
        ph, sp = D.denoise_plan(10_000 + k if k < n_train else 20_000 + k, shape, voxel_cm)
        plans.append(sim.add(ph, sp, per_pass))
    log(f"{len(plans)} plans loaded in {time.perf_counter() - t:.1f} s")
    t = time.perf_counter()
    pairs = []
    for i, p in enumerate(plans[:n_train]):
        pairs += D.make_pairs(sim, [p], high_passes, levels)
        if i % 16 == 15:
            _sync()
            log(f"pairs {i + 1}/{n_train} ({time.perf_counter() - t:.1f} s)")
    _sync()
    t_pairs = time.perf_counter() - t
    rate = n_train * (sum(levels) + high_passes) * per_pass / t_pairs
    log(f"pairs: {n_train} plans x {(sum(levels) + high_passes) * per_pass:.3g} histories in {t_pairs:.1f} s "
        f"({rate:.3g} histories/s)")
    net, losses, t_train = D.train(pairs, crop, steps, lr, seed=0, log=log, log_every=500)
    params = net.get_params()
    net.close()
    del pairs
    rows = []
    for p in plans[n_train:]:
        d1, v1 = sim.dose(p, 1, variance=True)
        u1, _, _ = sim.ctx.mean_uncertainty(p, d1, v1, 0.5)
        n2 = per_pass * (u1 / 0.02) ** 2                       # histories to 2%
        passes_2 = max(1, int(math.ceil(n2 / per_pass)))
        rho = sim.density(p)
        ref, _ = sim.dose(p, 4 * passes_2 + high_passes)
        plain, _ = sim.dose(p, passes_2)
        x, dmax = sim.net_input(p, plain, rho)
        r = sim.scaled(p, ref, rho, dmax)
        g_star = sim.ctx.gamma_index(p, r.reshape(-1).double(), x[0].reshape(-1).double())[0]
        best, tried = None, []
        k = 1
        while k <= passes_2:
            low, _ = sim.dose(p, k)
            xl, dl = sim.net_input(p, low, rho)
            _sync()
            ti = time.perf_counter()
            den = D.infer(params, xl)
            _sync()
            t_inf = time.perf_counter() - ti
            rl = sim.scaled(p, ref, rho, dl)
            g = sim.ctx.gamma_index(p, rl.reshape(-1).double(), den.reshape(-1).double())[0]
            gp = sim.ctx.gamma_index(p, rl.reshape(-1).double(), xl[0].reshape(-1).double())[0]
            tried.append((k, g, gp))
            if g >= g_star:
                best = (k * per_pass, g, t_inf)
                break
            k = k + 1 if step_passes == 1 else k * 2
        row = {"plan": int(p), "u_one_pass": u1, "N_2pct": n2, "passes_2pct": passes_2, "G_star": g_star,
               "t_plain_s": passes_2 * per_pass / rate, "tried_passes_gamma_denoised_plain": tried,
               "N_denoised": best[0] if best else None, "G_denoised": best[1] if best else None,
               "t_denoised_s": (best[0] / rate + best[2]) if best else None}
        log(f"denoise eval: {row}")
        rows.append(row)
    ok = [r for r in rows if r["t_denoised_s"] is not None]
    out = {"train_plans": n_train, "test_plans": n_test, "shape_xyz": shape, "voxel_cm": voxel_cm, "levels": levels,
           "per_pass": per_pass, "high_passes": high_passes, "train_steps": steps, "crop_zyx": crop,
           "train_seconds": t_train, "pair_seconds": t_pairs, "rate_histories_per_s": rate,
           "final_losses": losses[-5:],
           "t_plain_mean_s": float(np.mean([r["t_plain_s"] for r in rows])),
           "t_denoised_mean_s": float(np.mean([r["t_denoised_s"] for r in ok])) if ok else None,
           "reached": len(ok), "rows": rows}
    log(f"denoiser study: {out}")
    return out


C5_LAUNCH = dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=2, tally_mode=2,
                 source_order=1)


def c5_pairs(db, seeds, shape, voxel_cm, base, levels, high, launch, log, e_range=(70.0, 230.0), t_high=None):
    """Training samples of the given plan seeds: per plan the density / 2
    (bf16) and the high-history target divided by its own Dmax (float32); per
    input level k the dose of k * base histories divided by its own Dmax (bf16)
    and the ratio of the two Dmax values (the target on the input's
    normalisation is target * ratio).  Plans run in contexts of 25 plans
    (closed afterwards); track rotation on; every dose is a new plan id, so
    inputs and targets never share a history."""
    import concurrent.futures as cf

    import torch
    out = []
    t_high = [] if t_high is None else t_high          # wall time of each target run (load, run, dose)
    # the phantoms are generated on the host two plans ahead of the GPU work
    pool = cf.ThreadPoolExecutor(2)
    make = lambda sd: D.denoise_plan(sd, shape, voxel_cm, e_range=e_range, half_width_cm=4.0)
    futs = {sd: pool.submit(make, sd) for sd in seeds[:2]}
    for c0 in range(0, len(seeds), 25):
        ctx = F.Context(0, 7, table=I.HU_TABLE_DEFAULT)
        ctx.load_track_db(db)
        ctx.set_launch_config(**launch)
        for i, sd in enumerate(seeds[c0:c0 + 25]):
            for nxt in seeds[c0 + i + 1:c0 + i + 3]:
                if nxt not in futs:
                    futs[nxt] = pool.submit(make, nxt)
            ph, sp = futs.pop(sd).result()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ph_, hd, _ = D.plan_dose(ctx, ph, sp, high, F.FDC_RUN_ROTATE_TRACKS)
            torch.cuda.synchronize()
            t_high.append(time.perf_counter() - t0)
            rho = torch.empty(ph.hu.size, dtype=torch.float32, device="cuda")
            ctx.density(ph_, rho)
            _, _, dmax_h = ctx.mean_uncertainty(ph_, hd, hd, 0.5)
            th = D.normalised(ctx, ph_, hd, rho, 1.0 / dmax_h)
            sample = {"rho": th[1].to(torch.bfloat16), "target": th[0].clone(), "levels": []}
            del th, hd
            for k in levels:
                pl, ld, _ = D.plan_dose(ctx, ph, sp, k * base, F.FDC_RUN_ROTATE_TRACKS)
                _, _, dmax_l = ctx.mean_uncertainty(pl, ld, ld, 0.5)
                xl = D.normalised(ctx, pl, ld, rho, 1.0 / dmax_l)
                sample["levels"].append((xl[0].to(torch.bfloat16), dmax_h / dmax_l))
                del xl, ld
            out.append(sample)
        torch.cuda.synchronize()
        ctx.close()
        log(f"c5 pairs: {min(c0 + 25, len(seeds))}/{len(seeds)} plans")
    pool.shutdown()
    return out


def train_samples(samples, crop, steps, lr=1e-3, seed=0, log=None, log_every=500, focus=0.9, lr_final=0.1):
    """D.train on c5_pairs samples: a step picks a plan and an input level,
    crops (x = (input, density), target * ratio) around the dose region with
    probability focus, and mirrors the crop along random axes."""
    import torch
    net = F.UNet(crop)
    net.init_params(seed)
    rng = np.random.default_rng(seed)
    hot = [D._dose_voxels(s["target"]) for s in samples]
    losses = []
    cz, cy, cx = crop
    t0 = time.perf_counter()
    for it in range(steps):
        k = int(rng.integers(len(samples)))
        s = samples[k]
        low, ratio = s["levels"][int(rng.integers(len(s["levels"])))]
        nz, ny, nx = s["target"].shape
        if hot[k].size and rng.random() < focus:
            c = int(hot[k][int(rng.integers(hot[k].size))])
            centre = (c // (ny * nx), (c // nx) % ny, c % nx)
            z0, y0, x0 = (min(max(int(q) - w // 2 + int(rng.integers(-w // 4, w // 4 + 1)), 0), n - w)
                          for q, w, n in zip(centre, crop, (nz, ny, nx)))
        else:
            z0, y0, x0 = (int(rng.integers(0, n - w + 1)) for n, w in zip((nz, ny, nx), crop))
        sl = (slice(z0, z0 + cz), slice(y0, y0 + cy), slice(x0, x0 + cx))
        xc = torch.stack([low[sl], s["rho"][sl]]).float()
        tc = s["target"][sl] * float(ratio)
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
    params = net.get_params()
    net.close()
    return params, losses, time.perf_counter() - t0


def c5_study(db, n_train=500, n_val=50, shape=(256, 256, 128), voxel_cm=0.2, base=250_000, levels=(1, 2, 4, 8),
             high=100_000_000, ref_total=400_000_000, crop=(128, 128, 128), steps=16000, lr=1e-3,
             launch=C5_LAUNCH, weights_out=None, json_out=None, log=print):
    """The learned denoiser at full scale: n_train thorax-like training plans
    (seeds 10000..) and n_val validation plans (seeds 20000..), 256x256x128 of
    2 mm, 1-3 fields of 200-2000 spots, 70-230 MeV, over 8x8 cm at the right
    lung.  Inputs: doses of k * base histories (k in levels: 2.5e5 .. 2e6, the
    1e6-history input among them); targets 1e8 histories; 128^3 crops, MSE,
    Adam (lr 1e-3, cosine to 1e-4).  Each validation plan: N_2% from the Eq.
    (2) mean uncertainty of 1e6 histories, G* of the plain dose at N_2% against
    an independent 4e8-history reference, the denoised ladder N_2% * {1/64 ..
    1} (gamma_ladder).  Times use the transport rate measured on the pairs.
    With json_out, the result so far is written after every validation plan."""
    import torch
    t = time.perf_counter()
    t_high = []
    samples = c5_pairs(db, [10_000 + k for k in range(n_train)], shape, voxel_cm, base, levels, high, launch, log,
                       t_high=t_high)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t
    n_hist = n_train * (high + sum(levels) * base)
    rate = high / float(np.median(t_high))              # a target run: load, 1e8 histories, dose
    log(f"c5 pairs: {n_train} plans, {n_hist:.3g} histories in {t_pairs:.1f} s; target runs at {rate:.3g} "
        f"histories/s (median, loading and dose included)")
    params, losses, t_train = train_samples(samples, crop, steps, lr, seed=0, log=log)
    del samples
    torch.cuda.empty_cache()
    meta = {"train_plans": n_train, "seeds": [10_000, 10_000 + n_train - 1], "shape_xyz": list(shape),
            "voxel_cm": voxel_cm, "input_histories": [k * base for k in levels], "target_histories": high,
            "crop_zyx": list(crop), "steps": steps, "lr": lr, "n_params": int(params.size)}
    if weights_out:
        D.save_params(weights_out, params, meta)
        log(f"weights written to {weights_out}")
    rows = []
    ctx = None
    for j in range(n_val):
        if ctx is not None:
            ctx.close()
        ctx = F.Context(0, 11, table=I.HU_TABLE_DEFAULT)
        ctx.load_track_db(db)
        ctx.set_launch_config(**launch)
        ph, sp = D.denoise_plan(20_000 + j, shape, voxel_cm, e_range=(70.0, 230.0), half_width_cm=4.0)
        p1, d1, v1 = D.plan_dose(ctx, ph, sp, 1_000_000, F.FDC_RUN_VARIANCE | F.FDC_RUN_ROTATE_TRACKS)
        u1, _, _ = ctx.mean_uncertainty(p1, d1, v1, 0.5)
        n2 = 1_000_000 * (u1 / 0.02) ** 2
        row = D.gamma_ladder(ctx, ph, sp, params, n2, rate, ref_total=ref_total)
        row.update(plan_seed=20_000 + j, u_1e6=u1)
        rows.append(row)
        lad = " ".join(f"{r['histories']:.3g}:{r['gamma_denoised']:.4f}/{r['gamma_plain']:.4f}" for r in row["ladder"])
        log(f"c5 val {j}: N_2% {n2:.3g}, G* {row['G_star']:.5f}, N_d {row['N_denoised']}, ladder {lad}")
        del d1, v1
        if json_out:
            import json
            with open(json_out, "w") as f:
                json.dump({**meta, "rate_histories_per_s": rate, "pair_seconds": t_pairs, "train_seconds": t_train,
                           "final_losses": losses[-5:], "rows": rows}, f, default=float)
    if ctx is not None:
        ctx.close()
    reached = [r for r in rows if r["N_denoised"] is not None]
    out = {**meta, "val_plans": n_val, "pair_seconds": t_pairs, "train_seconds": t_train,
           "rate_histories_per_s": rate, "final_losses": losses[-5:], "reached": len(reached),
           "t_plain_mean_s": float(np.mean([r["t_plain_s"] for r in rows])),
           "t_denoised_mean_s_reached": float(np.mean([r["t_denoised_s"] for r in reached])) if reached else None,
           "rows": rows}
    return out


# multiply-adds of one voxel through the network (all layers, forward), times 2
UNET_FLOP_PER_VOXEL = 94_880


def denoiser_rate(reps=3, vol=(128, 256, 256), crop=(128, 128, 128), log=None):
    """Best-of-`reps` (after a warm-up) wall time of the denoiser's forward pass
    over `vol` and of one training step (forward, backward, Adam) on `crop`,
    random inputs and He-initialised weights; sizes are (z, y, x)."""
    import torch

    def best(f):
        f()
        _sync()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            f()
            _sync()
            ts.append(time.perf_counter() - t)
            if log:
                log(f"{f.__name__}: {ts[-1] * 1e3:.2f} ms")
        return min(ts)

    g = torch.Generator(device="cuda").manual_seed(0)
    net = F.UNet(vol)
    net.init_params(1)
    x = torch.rand((2,) + tuple(vol), device="cuda", generator=g)
    y = torch.empty(vol, device="cuda")

    def forward():
        net.forward(x, y)
    tf = best(forward)
    net.close()
    net = F.UNet(crop)
    net.init_params(1)
    xc = torch.rand((2,) + tuple(crop), device="cuda", generator=g)
    tc = xc[0].clone()

    def train_step():
        net.backward(xc, tc, want_loss=False)
        net.adam(1e-3)
    ts = best(train_step)
    net.close()
    vox_f, vox_c = float(np.prod(vol)), float(np.prod(crop))
    return {"forward_ms": tf * 1e3, "forward_volume_zyx": list(vol),
            "forward_tflops": UNET_FLOP_PER_VOXEL * vox_f / tf / 1e12,
            "train_step_ms": ts * 1e3, "train_crop_zyx": list(crop),
            "train_tflops": 3 * UNET_FLOP_PER_VOXEL * vox_c / ts / 1e12, "peak_tflops_bf16": 2500.0}


def _c_over_sqrt(ns, us):
    """The line C / sqrt(N) through the point of lowest N (as in the paper's
    recycling figure) and the largest relative deviation of the points from it."""
    c = us[0] * math.sqrt(ns[0])
    dev = max(abs(u / (c / math.sqrt(n)) - 1.0) for n, u in zip(ns, us))
    return c, dev


def recycling_study(R_values=(1, 64, 320), db_seeds=(101, 102, 103, 104, 105, 106), hbh_db_seed=2188,
                    n_min=1_500_000, doublings=5, n_tracks=10_000, log=print,
                    workload=None):
    """The recycling test (Section 3): does re-tracing each stored track many
    times correlate the histories?

    For each reuse factor R (histories of a spot per shared track) and each N in
    n_min * 2^k (k = 0..doublings) on the slab workload:
      * history-by-history: one run of N histories (database seed hbh_db_seed,
        run seed 1), mean over voxels above Dmax/2 of sigma/D from Eq. (2);
      * batch method: n = len(db_seeds) fully independent batches of N/n
        histories, each with its own synthetic database (seed db_seeds[i]) and
        its own run seed, combined with Eq. (1); also with the first half of the
        batches (their total N/2), and with n batches that share the
        history-by-history database (different run seeds only).
    Hidden correlations would show as a departure from 1/sqrt(N) of the
    history-by-history curve and as history-by-history values below the batch
    values.  Each curve gets the line C/sqrt(N) through its lowest-N point and
    the largest relative deviation from it.  Doses of one N are snapshots of
    one accumulating run (k doubles the passes), so successive points share
    histories.  `workload` = (phantom, spots) replaces the slab (the spots'
    n_histories are replaced)."""
    import torch
    ph, sp0 = workload if workload is not None else (I.slab_phantom(128, 0.1), W.slab_spots(1))
    n_b = len(db_seeds)
    n_spots = len(sp0)
    if n_min % (n_b * n_spots):
        raise ValueError("n_min must split evenly over the batches and the spots")
    ks = [2 ** j for j in range(doublings + 1)]
    ns = [n_min * k for k in ks]
    nvox = int(np.prod(ph.hu.shape))
    t0 = time.perf_counter()
    bins = list(W.DB_BINS_FULL)
    dbs = {}
    for seed in (hbh_db_seed,) + tuple(db_seeds):
        dbs[seed] = I.make_water_track_db(bins, n_tracks, seed)
        log(f"recycling: database seed {seed} ready ({time.perf_counter() - t0:.0f} s)")

    def spots(per_pass):
        sp = sp0.copy()
        sp["n_histories"] = per_pass // n_spots
        return sp

    def snapshots(db, run_seed, R, per_pass, variance):
        """Doses (and Eq. (2) variances) after k passes for every k in ks."""
        c = F.Context(0, run_seed, reuse_R=R, table=I.HU_TABLE_DEFAULT)
        c.load_track_db(db)
        p = c.load_phantom(ph)
        c.add_beam_spots(p, spots(per_pass))
        flags = F.FDC_RUN_VARIANCE if variance else 0
        out, done = [], 0
        for k in ks:
            for _ in range(k - done):
                c.run_histories([p], flags)
            done = k
            d = torch.empty(nvox, dtype=torch.float64, device="cuda")
            v = torch.empty(nvox, dtype=torch.float64, device="cuda") if variance else None
            c.compute_dose(p, d, v)
            out.append((d, v))
        return c, p, out

    result = {"n": ns, "n_min": n_min, "batches": n_b, "db_seeds": list(db_seeds), "hbh_db_seed": hbh_db_seed,
              "n_tracks_per_bin": n_tracks, "R": {}}
    for R in R_values:
        t = time.perf_counter()
        c, p, hb = snapshots(dbs[hbh_db_seed], 1, R, n_min, True)
        u_hbh = [c.mean_uncertainty(p, d, v, 0.5)[0] for d, v in hb]
        c.close()
        indep = []
        for i, seed in enumerate(db_seeds):
            cb, pb, sn = snapshots(dbs[seed], seed, R, n_min // n_b, False)
            indep.append([d for d, _ in sn])
            if i < n_b - 1:
                cb.close()
        shared = []
        for i in range(n_b):
            cs, _, sn = snapshots(dbs[hbh_db_seed], 1000 + i, R, n_min // n_b, False)
            shared.append([d for d, _ in sn])
            cs.close()

        def eq1(doses):
            stack = torch.stack(doses)
            mean = torch.empty(nvox, dtype=torch.float64, device="cuda")
            sig = torch.empty(nvox, dtype=torch.float64, device="cuda")
            cb.batch_uncertainty(stack, mean, sig)
            return cb.mean_uncertainty(pb, mean, sig.square(), 0.5)[0]

        u_b = [eq1([indep[b][j] for b in range(n_b)]) for j in range(len(ks))]
        u_half = [eq1([indep[b][j] for b in range(n_b // 2)]) for j in range(len(ks))]
        u_sh = [eq1([shared[b][j] for b in range(n_b)]) for j in range(len(ks))]
        cb.close()
        torch.cuda.synchronize()
        rec = {"hbh_eq2": u_hbh, "batch_eq1_indep": u_b, "batch_eq1_indep_half": u_half,
               "n_half": [n // 2 for n in ns], "batch_eq1_shared_db": u_sh,
               "ratio_hbh_over_batch": [a / b for a, b in zip(u_hbh, u_b)], "seconds": time.perf_counter() - t}
        for key, xs in (("hbh_eq2", ns), ("batch_eq1_indep", ns), ("batch_eq1_indep_half", rec["n_half"]),
                        ("batch_eq1_shared_db", ns)):
            cc, dev = _c_over_sqrt(xs, rec[key])
            rec[key + "_fit"] = {"C": cc, "max_rel_deviation": dev}
        result["R"][R] = rec
        log(f"recycling R={R}: hbh {['%.4f' % u for u in u_hbh]} batch {['%.4f' % u for u in u_b]} "
            f"({rec['seconds']:.1f} s)")
        del indep, shared, hb
    return result


def _main():
    import argparse
    import json
    ap = argparse.ArgumentParser(prog="python -m paper_1011_2188_amd.experiments")
    ap.add_argument("what", choices=["denoiser", "c5"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--train", type=int, default=500, help="c5: training plans")
    ap.add_argument("--val", type=int, default=50, help="c5: validation plans")
    ap.add_argument("--steps", type=int, default=16000, help="c5: training steps")
    ap.add_argument("--weights", default=None, help="c5: write the trained parameters here (.npz)")
    ap.add_argument("--json", default=None, help="c5: write the result here")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the experiments need a GPU"
    torch.cuda.init()
    log = lambda m: print(m, flush=True)
    if args.what == "denoiser":
        out = denoiser_rate(args.reps, log=log)
    else:
        out = c5_study(W.multi_bin_db(), n_train=args.train, n_val=args.val, steps=args.steps,
                       weights_out=args.weights, json_out=args.json, log=log)
        if args.json:
            with open(args.json, "w") as f:
                json.dump(out, f, default=float)
    print(json.dumps(out, default=float), flush=True)


if __name__ == "__main__":
    _main()
