"""Benchmark: proton histories/s of the track-repeating dose engine on one MI355X.

One step = one complete dose calculation of the thorax workload (synthetic
thorax CT of 256 x 256 x 128 voxels of 2 mm; three coplanar fields at gantry
0, 90 and 180 degrees with 2000 spots each at 70..230 MeV; 1e8 histories;
database of 33 energy bins x 1e4 synthetic water tracks): clear the tallies,
re-trace every history with the energy and squared-energy tallies, and convert
to dose and Eq. (2) variance on the device.  Inputs (database, phantom, spots)
are resident in HBM before timing starts.  The launch configuration is
autotuned before the warm-up (untimed; only knobs that cannot change a result
bit), or fixed with --launch.

Prints ONE JSON line.  Also reported: seconds to 2% mean dose uncertainty
(Eq. (2), voxels above half the maximum dose; extrapolated from the step, then
verified by running that many histories), the transport kernel against the HBM
roofline (HIP-event kernel time; HBM traffic from the committed rocprofv3
counter summary when it matches this kernel and launch), the CPU oracle timed
on this host on a bounded sample (one thread and all threads), and as extras
the slab and paper-field workloads, the batch estimator of Eq. (1) and the
denoiser.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "proton histories/sec and seconds to 2% dose uncertainty, plain vs denoised, 1 MI355X"
HBM_PEAK_GBS = 8000.0
LAUNCH_KEYS = ("waves_per_block", "blocks_per_cu", "tally_slots", "units_per_wave", "tally_mode", "source_order")

# Work per history, counted exactly by the oracle (steps S, non-vacuum voxel
# visits C, vacuum voxel visits Cv, tally flushes G) on a sample of every spot
# of each workload (thorax: 6000 spots x 64 histories; slab: 25 x 2000).
COUNTS = {
    "thorax": dict(S=109.73, C=212.74, Cv=111.67, G=104.01),
    "slab": dict(S=95.03, C=205.38, Cv=0.0, G=111.71),
}


def bytes_per_history(counts, variance, shared=64.0):
    """Algorithmic HBM bytes per history: 16 B per step record / the histories
    sharing one read of it (64: a chunk of 64 histories re-traces one track) +
    2 B voxel index per non-vacuum voxel visit + 8 B per tally update (one per
    flush, two with the squared-energy tally).  Vacuum visits are ALU work
    (their index reads are not counted)."""
    return (16.0 * counts["S"] / shared + 2.0 * counts["C"]
            + 8.0 * counts["G"] * (2.0 if variance else 1.0))


def measured_traffic(launch, profile):
    """HBM bytes per launch of the transport kernel from a committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, if it holds an entry for this launch
    configuration and the kernel sources are unchanged since; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile)
    try:
        lines = [line.strip().split(": ", 1) for line in open(path) if line.startswith("    ") and ": " in line]
        src = b"".join(open(os.path.join(ROOT, "paper_1011_2188_amd", "csrc", f), "rb").read()
                       for f in ("transport.hip", "fdc_device.h"))
    except (OSError, ValueError):
        return None
    sha = dict(kv for kv in lines if len(kv) == 2).get("kernel_source_sha1")
    if sha != hashlib.sha1(src).hexdigest():
        return None
    want = ",".join(str(launch.get(k, 0)) for k in LAUNCH_KEYS)
    cur = None
    for kv in lines:
        if len(kv) != 2:
            continue
        if kv[0] == "launch":
            cur = kv[1]
        elif kv[0] == "traffic_bytes_per_launch" and cur == want:
            return float(kv[1])
    return None


def kernel_name(launch):
    return ("transport_kernel" if not launch.get("tally_slots", 0) else
            "transport_cache_kernel" if launch.get("tally_mode", 0) == 2 else "transport_lds_kernel")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# LDS-cache launch candidates (the autotuner's best family on every workload measured)
CACHE_CANDS = ([dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=1, tally_mode=m,
                     source_order=0) for m in (1, 2)]
               + [dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=u, tally_mode=2,
                       source_order=1) for u in (1, 2, 4, 8)])


def best_of(f, n=3):
    import torch
    f()
    torch.cuda.synchronize()
    ts = []
    for _ in range(n):
        t = time.perf_counter()
        f()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return min(ts)


def timed_kernel_ms(c, f, n=3):
    """Mean HIP-event time of the transport kernel over n runs of f."""
    import numpy as np
    import torch
    f()
    torch.cuda.synchronize()
    c.set_timing(True)
    for _ in range(n):
        f()
    torch.cuda.synchronize()
    ms = float(np.mean(c.transport_times(n)))
    c.set_timing(False)
    return ms


def mean_unc(c, plan, dose, var):
    u, _, _ = c.mean_uncertainty(plan, dose, var, 0.5)
    return u


def extras(c, plan, nvox, hist_per_step, launch, variance, ph_thorax, sp_thorax):
    """Other rows of the path, timed live: the batch estimator of Eq. (1) on the
    thorax (six batches of new histories, energy tally only, as the paper's batch
    method; the batches share the database, whose own variance the recycling
    study measures); the slab workload (1e7 histories, both tallies); the
    paper's kind of test case (121 MeV disk field, 1 x 1 x 2.5 mm voxels, 1e7
    histories); the denoiser's forward pass (256x256x128 volume) and training
    step (128^3 crop: forward, backward, Adam), each the best of three after a
    warm-up.  Each workload gets its own tuned launch configuration (untimed)."""
    import torch
    from paper_1011_2188_amd import autotune as A
    from paper_1011_2188_amd import fdc as F
    from paper_1011_2188_amd import inputs as I
    from paper_1011_2188_amd import workloads as W

    out = {}
    # Eq. (1) batch method on the thorax
    nb = 6
    doses = torch.empty((nb, nvox), dtype=torch.float64, device="cuda")
    eq1_launch, _ = A.tune(c, [plan], 0, use_cache=False, candidates=CACHE_CANDS, reps=1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for b in range(nb):                       # new histories each batch (counters continue)
        c.reset_plan(plan)
        c.run_histories([plan], 0)
        c.compute_dose(plan, doses[b], None)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    mean = torch.empty(nvox, dtype=torch.float64, device="cuda")
    sigma = torch.empty(nvox, dtype=torch.float64, device="cuda")
    c.batch_uncertainty(doses, mean, sigma)
    ub, _, _ = c.mean_uncertainty(plan, mean, sigma.square(), 0.5)
    n_tot = nb * hist_per_step
    n2 = n_tot * (ub / 0.02) ** 2
    out["batch_method_eq1"] = {"batches": nb, "histories": n_tot, "seconds": tb, "histories_per_s": n_tot / tb,
                               "launch": eq1_launch, "mean_uncertainty": ub, "histories_to_2pct": n2,
                               "seconds_to_2pct": n2 / (n_tot / tb)}
    log(f"batch method: {ub:.4%} at {n_tot} histories -> 2% in {n2 / (n_tot / tb):.4g} s")
    del doses
    c.set_launch_config(**launch)

    # slab workload, in its own context
    flags = F.FDC_RUN_VARIANCE if variance else 0
    ph, sp, db = W.slab()
    cs = F.Context(0, 1, table=I.HU_TABLE_DEFAULT)
    cs.load_track_db(db)
    ps = cs.load_phantom(ph)
    cs.add_beam_spots(ps, sp)
    sl_launch, _ = A.tune(cs, [ps], flags, use_cache=False, candidates=CACHE_CANDS, reps=2)
    n = int(sp["n_histories"].sum())
    d = torch.empty(ph.hu.size, dtype=torch.float64, device="cuda")
    v = torch.empty(ph.hu.size, dtype=torch.float64, device="cuda")

    def slab_run():
        cs.reset_plan(ps)
        cs.run_histories([ps], flags)
        cs.compute_dose(ps, d, v if variance else None)
    t = best_of(slab_run)
    kms = timed_kernel_ms(cs, slab_run)
    u = mean_unc(cs, ps, d, v) if variance else None
    bph = bytes_per_history(COUNTS["slab"], variance)
    out["slab_1e7"] = {"seconds": t, "histories_per_s": n / t, "launch": sl_launch, "kernel_ms": kms,
                       "roofline_frac": bph * n / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, "bytes_per_history": bph,
                       "mean_uncertainty": u, "seconds_to_2pct": (n * (u / 0.02) ** 2 / (n / t)) if u else None,
                       "workload": "slab phantom 128^3 x 1 mm (bone z 4-6 cm, lung z 8-12 cm), 25 spots "
                                   "70-230 MeV x 4e5 histories, both tallies"}
    log(f"slab: {n / t:.4g} histories/s, kernel {kms:.3f} ms")
    cs.close()
    del d, v

    # the paper's kind of test case: 121 MeV disk field (radius 4 cm) on 1 x 1 x 2.5 mm voxels;
    # its own database (1e5 tracks at 121 MeV)
    ph, sp, db_pf = W.paper_field()
    c2 = F.Context(0, 1, table=I.HU_TABLE_DEFAULT)
    c2.load_track_db(db_pf)
    p2 = c2.load_phantom(ph)
    c2.add_beam_spots(p2, sp)
    pf_launch, _ = A.tune(c2, [p2], use_cache=False, candidates=CACHE_CANDS, reps=1)
    n2 = int(sp["n_histories"].sum())
    d2 = torch.empty(ph.hu.size, dtype=torch.float64, device="cuda")
    v2 = torch.empty(ph.hu.size, dtype=torch.float64, device="cuda")

    def pf_run():
        c2.reset_plan(p2)
        c2.run_histories([p2], F.FDC_RUN_VARIANCE)
    t2 = best_of(pf_run)
    c2.compute_dose(p2, d2, v2)
    u2 = mean_unc(c2, p2, d2, v2)
    c2.close()
    out["paper_field_1e7"] = {"seconds": t2, "histories_per_s": n2 / t2, "launch": pf_launch,
                              "mean_uncertainty": u2, "seconds_to_2pct": n2 * (u2 / 0.02) ** 2 / (n2 / t2),
                              "workload": "thorax 352x240x72 x 1x1x2.5 mm, one 121 MeV field of circular "
                                          "cross-section (radius 4 cm), 1e7 histories, DB 1e5 tracks at 121 MeV, "
                                          "both tallies"}
    log(f"paper field: {n2 / t2:.4g} histories/s, {u2:.4%} at 1e7")
    del d2, v2

    # the thorax with secondary trajectories in its database (protons from
    # non-elastic nuclear interactions, about 1%/cm above 20 MeV), the
    # headline's launch configuration
    t = time.perf_counter()
    db_s = W.multi_bin_db(secondaries=True)
    log(f"database with secondaries: {db_s.sec.n} secondaries, {db_s.sec.steps.shape[0]} steps "
        f"({time.perf_counter() - t:.1f} s)")
    c3 = F.Context(0, 1, table=I.HU_TABLE_DEFAULT)
    c3.load_track_db(db_s)
    c3.set_launch_config(**launch)
    p3 = c3.load_phantom(ph_thorax)
    c3.add_beam_spots(p3, sp_thorax)
    flags3 = F.FDC_RUN_VARIANCE if variance else 0

    def sec_run():
        c3.reset_plan(p3)
        c3.run_histories([p3], flags3)
    t3 = best_of(sec_run)
    k3 = timed_kernel_ms(c3, sec_run)
    r3 = c3.read_dose_and_variance(p3, raw=True)
    c3.close()
    out["thorax_1e8_secondaries"] = {
        "seconds": t3, "histories_per_s": hist_per_step / t3, "kernel_ms": k3, "launch": launch,
        "secondaries": db_s.sec.n, "secondary_steps": int(db_s.sec.steps.shape[0]),
        "escaped_fraction": r3["escaped"] / max(r3["incident"], 1),
        "workload": "the headline thorax workload with a database of 33 bins x 1e4 tracks carrying "
                    "secondary proton trajectories (nuclear interactions 1.2%/cm above 20 MeV)"}
    log(f"thorax with secondaries: {hist_per_step / t3:.4g} histories/s, kernel {k3:.3f} ms")
    del db_s

    from paper_1011_2188_amd import experiments as X
    den = X.denoiser_rate(3)
    out["denoiser"] = {"forward_ms_256x256x128": den["forward_ms"], "forward_tflops": den["forward_tflops"],
                       "train_step_ms_128cube": den["train_step_ms"], "train_tflops": den["train_tflops"],
                       "peak_tflops_bf16": den["peak_tflops_bf16"]}
    log(f"denoiser: forward {den['forward_ms']:.2f} ms, training step {den['train_step_ms']:.2f} ms")
    return out


WEIGHTS = os.path.join(ROOT, "paper_1011_2188_amd", "weights", "denoiser_thorax.npz")


def denoised_route(c, ph, sp, plain_plan, plain_dose, n2, rate):
    """The denoised half of the metric on this workload: G* = gamma pass rate
    (2%/2 mm) of the plain dose at N_2% (the verification run) against an
    independent reference of 4e8 histories; the trained denoiser (parameters
    from the full-scale training study, if present) on doses of N_2% * {1/64,
    ..., 1, 2, 4} histories; seconds = the first rung reaching G*, at this
    run's histories/s, plus the measured inference time (null when no rung
    reaches it; the ladder, the denoised pass rate at N_2% and the best one are
    reported either way).  Untimed for `value`."""
    from paper_1011_2188_amd import denoise as D
    if not os.path.exists(WEIGHTS):
        return {"seconds_to_2pct_denoised": None,
                "denoised": {"note": "no trained denoiser parameters (run the training study first)"}}
    params, meta = D.load_params(WEIGHTS)
    t = time.perf_counter()
    r = D.gamma_ladder(c, ph, sp, params, n2, rate, ref_total=400_000_000, plain=(plain_plan, plain_dose),
                       log=log, above=2)
    at_n2 = next(row for row in r["ladder"] if row["histories"] == max(1, int(round(n2))))
    r["gamma_denoised_at_N_2pct"] = at_n2["gamma_denoised"]
    r["best_gamma_denoised"] = max(row["gamma_denoised"] for row in r["ladder"])
    r["reached_G_star"] = r["N_denoised"] is not None
    # The ladder's doses use track rotation (as the denoiser's training data did);
    # G* is the benchmarked plain method's (no rotation).  The same comparison
    # against the rotated plain dose of N_2% histories, and the histories the
    # rotated plain dose alone needs to reach G*, both from the ladder's rungs:
    g_rot = at_n2["gamma_plain"]
    first = lambda key, g: next((row["histories"] for row in r["ladder"] if row[key] >= g), None)
    r["rotated_plain"] = {"G_star": g_rot, "N_denoised": first("gamma_denoised", g_rot),
                          "histories_to_G_star": first("gamma_plain", r["G_star"])}
    log(f"denoised route: G* {r['G_star']:.5f}, N_d {r['N_denoised']}, t_den {r['t_denoised_s']} "
        f"({time.perf_counter() - t:.1f} s)")
    r["weights"] = {k: meta[k] for k in ("train_plans", "input_histories", "target_histories", "steps")
                    if k in meta}
    return {"seconds_to_2pct_denoised": r["t_denoised_s"], "denoised": r}


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, os.cpu_count() or 1, avail


def cpu_baseline(ph, sp, db, target_s=12.0):
    """The oracle as it stands (plain C, FP64, OpenMP over history ranges with
    per-thread integer tallies) on a bounded sample of the same workload: every
    spot with the same number of histories, sized from a short probe for about
    target_s seconds, once on one thread and once on all threads of this host's
    share (at most 16), scaled to histories/s."""
    import numpy as np
    from oracle import oracle as O
    model, n_cpu, n_avail = host_cpu()
    threads = int(os.environ.get("ORACLE_THREADS", min(n_avail, 16)))

    def rate(th, per_spot):
        t = time.perf_counter()
        r = O.replay(db, ph, sp, h_count=np.full(len(sp), per_spot, np.uint64), threads=th)
        dt = time.perf_counter() - t
        return r["n_histories"] / dt, r["n_histories"], dt

    probe, _, _ = rate(threads, 4)
    per_all = int(max(4, min(int(sp["n_histories"].max()), probe * target_s / len(sp))))
    v_all, n_all, dt_all = rate(threads, per_all)
    if dt_all < 0.5 * target_s:               # the short probe underestimated the threaded rate
        per_all = int(max(4, min(int(sp["n_histories"].max()), v_all * target_s / len(sp))))
        v_all, n_all, dt_all = rate(threads, per_all)
    per_one = int(max(1, min(per_all, v_all / threads * target_s / len(sp))))
    v_one, n_one, dt_one = rate(1, per_one)
    return {"value": v_all, "unit": "histories/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sp)} spots x {per_all} histories of the same workload ({n_all} histories, "
                      f"{dt_all:.1f} s on {threads} threads); one thread: {len(sp)} x {per_one} "
                      f"({n_one} histories, {dt_one:.1f} s)",
            "one_thread_value": v_one, "cpu_model": model, "nproc": n_cpu, "cpus_available": n_avail}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-variance", action="store_true", help="energy tally only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 2%% verification run and the slab, paper-field, Eq. (1) and denoiser timings")
    ap.add_argument("--launch", default="tune",
                    help="'tune' (autotune before the warm-up, untimed) or waves_per_block,blocks_per_cu,"
                         "tally_slots,units_per_wave[,tally_mode[,source_order]]")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(histories are independent: more GPUs would take disjoint history ranges and "
              "sum the int64 tallies once)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1011_2188_amd import fdc as F
    from paper_1011_2188_amd import inputs as I
    from paper_1011_2188_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.init()
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    variance = not args.no_variance
    flags = F.FDC_RUN_VARIANCE if variance else 0

    t = time.perf_counter()
    ph, sp, db = W.thorax()
    log(f"inputs generated in {time.perf_counter() - t:.1f} s: DB {db.steps.shape[0]} steps, "
        f"{db.n_tracks} tracks, {db.n_bins} bins; phantom {ph.hu.shape}, {len(sp)} spots")
    c = F.Context(device=0, seed=1, table=I.HU_TABLE_DEFAULT)
    t = time.perf_counter()
    c.load_track_db(db, stream)
    plan = c.load_phantom(ph, stream)
    c.add_beam_spots(plan, sp)
    torch.cuda.synchronize()
    log(f"loaded into HBM in {time.perf_counter() - t:.2f} s")
    if args.launch == "tune":
        from paper_1011_2188_amd import autotune as A
        t = time.perf_counter()
        launch, timings = A.tune(c, [plan], flags, reps=2, use_cache=False, candidates=CACHE_CANDS)
        log(f"autotuned in {time.perf_counter() - t:.1f} s: {launch}")
        for k, v in sorted(timings.items(), key=lambda kv: kv[1]):
            log(f"  {v * 1e3:8.2f} ms  {k}")
    else:
        v = [int(x) for x in args.launch.split(",")]
        launch = dict(zip(LAUNCH_KEYS, v))
        c.set_launch_config(**launch)
    nvox = ph.hu.size
    hist_per_step = int(sp["n_histories"].sum())
    dose = torch.empty(nvox, dtype=torch.float64, device=dev)
    var = torch.empty(nvox, dtype=torch.float64, device=dev) if variance else None

    def step():
        c.reset_plan(plan, stream=stream)
        c.run_histories([plan], flags, stream=stream)
        c.compute_dose(plan, dose, var, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the library brackets each run's transport kernel with HIP events on the
    # run's stream (read back after the timed region)
    c.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    value = hist_per_step * args.steps / wall
    kern_ms = float(np.mean(c.transport_times(min(args.steps, 64))))
    c.set_timing(False)
    log(f"{args.steps} steps in {wall:.3f} s: {value:.4g} histories/s; transport {kern_ms:.3f} ms per launch")

    # seconds to 2% mean uncertainty (Eq. (2), voxels above Dmax/2), from the last step
    out = {}
    # the work of one launch counted on the device (untimed, its own run): steps
    # S, non-vacuum voxel pieces C and flushes G per history, against the
    # oracle's counts on a sample that the roofline's byte figure uses
    if variance:
        u_step, _, _ = c.mean_uncertainty(plan, dose, var, 0.5, stream=stream)
    c.reset_plan(plan, stream=stream)
    c.run_histories([plan], flags | F.FDC_RUN_COUNT_WORK, stream=stream)
    wk = c.read_work_counts(plan, stream=stream)
    live = {"S": wk["steps"] / hist_per_step, "C": wk["visits"] / hist_per_step, "G": wk["flushes"] / hist_per_step}
    out["work_per_history"] = {"device": live, "oracle_sample": COUNTS["thorax"],
                               "bytes_per_history_device": bytes_per_history(live, variance)}
    log(f"work per history on the device: S {live['S']:.2f}, C {live['C']:.2f}, G {live['G']:.2f} "
        f"(oracle sample {COUNTS['thorax']['S']}, {COUNTS['thorax']['C']}, {COUNTS['thorax']['G']})")
    if variance:
        u0 = u_step
        n2 = hist_per_step * (u0 / 0.02) ** 2
        out["mean_uncertainty_at_step"] = u0
        out["histories_to_2pct"] = n2
        out["seconds_to_2pct"] = n2 / value
        r = c.read_dose_and_variance(plan, dose=False, var=False, raw=False, stream=stream)
        assert r["deposited"] + r["escaped"] == r["incident"], "energy identity violated"
        log(f"mean uncertainty {u0:.4%} at {hist_per_step} histories -> 2% at {n2:.3g} histories, "
            f"{n2 / value:.3g} s")
    if variance and not args.no_extras:
        # verification: a plan of the same spots with N_2% histories in total, run
        # and finalised (dose, Eq. (2) variance, mean uncertainty on the device),
        # best of three after a warm-up
        sp2 = sp.copy()
        base, extra = divmod(int(np.ceil(n2)), len(sp))
        sp2["n_histories"] = base
        sp2["n_histories"][:extra] += 1
        plan2 = c.load_phantom(ph)
        c.add_beam_spots(plan2, sp2)
        n2_run = int(sp2["n_histories"].sum())
        times = []
        for rep in range(4):
            c.reset_plan(plan2, stream=stream)
            torch.cuda.synchronize()
            t = time.perf_counter()
            c.run_histories([plan2], flags, stream=stream)
            c.compute_dose(plan2, dose, var, stream=stream)
            u2, _, _ = c.mean_uncertainty(plan2, dose, var, 0.5, stream=stream)
            torch.cuda.synchronize()
            if rep:
                times.append(time.perf_counter() - t)
        out["verify_2pct"] = {"histories": n2_run, "mean_uncertainty": u2, "seconds": min(times),
                              "in_band": bool(0.019 <= u2 <= 0.021)}
        log(f"verification: {n2_run} histories -> {u2:.4%} in {min(times):.4g} s")
        out.update(denoised_route(c, ph, sp, plan2, dose.clone(), n2_run, value))

    so = launch.get("source_order", 0)
    bph = bytes_per_history(COUNTS["thorax"], variance)
    achieved = bph * hist_per_step / (kern_ms * 1e-3) / 1e9
    issued = bytes_per_history(COUNTS["thorax"], variance, shared=1.0 if so else 64.0)
    updates = COUNTS["thorax"]["G"] * (2.0 if variance else 1.0) * hist_per_step / (kern_ms * 1e-3)
    traffic = measured_traffic(launch, "transport_thorax_1e8_pmc.md")
    result = {
        "metric": METRIC, "value": value, "unit": "histories/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "thorax CT 256x256x128 x 2 mm (body ellipse, lungs, spine), 3 fields (gantry "
                               "0/90/180) x 2000 spots 70-230 MeV, 1e8 histories per step, DB 33 bins x 1e4 "
                               "tracks, int64 fixed-point tallies" + (" + squared-energy tally" if variance else ""),
                   "histories_per_step": hist_per_step, "variance": variance, "launch": launch},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel_name(launch), "kernel_ms": kern_ms,
                     "bytes_per_history": bph, "issued_bytes_per_history": issued,
                     "tally_updates_per_s": updates},
        **out,
    }
    if not args.no_extras:
        result["extras"] = extras(c, plan, nvox, hist_per_step, launch, variance, ph, sp)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        result["cpu_baseline"] = cpu_baseline(ph, sp, db)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
