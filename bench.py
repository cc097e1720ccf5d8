"""Benchmark: proton histories/s of the track-repeating dose engine on one MI355X.

One step = one complete dose calculation of the slab workload (128^3 voxels of
1 mm with a bone and a lung slab, 25 pencil-beam spots at 70..230 MeV, 4e5
histories each = 1e7 histories, database of 33 energy bins x 1e4 synthetic
water tracks): clear the tallies, re-trace every history with the energy and
squared-energy tallies, and convert to dose and Eq. (2) variance on the device.
Inputs (database, phantom, spots) are resident in HBM before timing starts.
The launch configuration is autotuned before the warm-up (untimed; only knobs
that cannot change a result bit), or fixed with --launch.

Prints ONE JSON line.  Also reported: seconds to 2% mean dose uncertainty
(Eq. (2), voxels above half the maximum dose; extrapolated from the step, then
verified by running that many histories), the transport kernel against the
HBM roofline (HIP-event kernel time; HBM traffic from the committed rocprofv3
counter summary when it matches this kernel and launch), and the CPU oracle
timed on this host on a bounded sample.
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

# Algorithmic work per history of the slab workload, counted exactly by
# replaying a 25 x 2000-history sample: steps S = 95.03, voxel-walk iterations
# C = 205.38 (no vacuum), flushes G = 111.71.  Bytes per history =
# 16 B per step record / the histories sharing one read of it (64 when a wave
# replays one track; 1 when the histories run in start-position order, each
# lane on its own track) + 2 B voxel index per walk iteration + 8 B per tally
# update (G, doubled with the squared-energy tally).
SLAB_S, SLAB_C, SLAB_G = 95.03, 205.38, 111.71
LAUNCH_KEYS = ("waves_per_block", "blocks_per_cu", "tally_slots", "units_per_wave", "tally_mode", "source_order")


def slab_bytes_per_history(variance: bool, source_order: int = 0) -> float:
    shared = 1.0 if source_order else 64.0
    return 16.0 * SLAB_S / shared + 2.0 * SLAB_C + 8.0 * SLAB_G * (2.0 if variance else 1.0)


def measured_traffic(launch):
    """HBM bytes per launch of the transport kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, if it holds an entry for this launch
    configuration and the kernel sources are unchanged since; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "transport_slab_1e7_pmc.md")
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


def extras(c, plan, nvox, hist_per_step, launch, log):
    """Other rows of the path, timed live: seconds to 2% with the batch
    estimator of Eq. (1) (six batches of new histories of the slab workload
    with the energy tally only, as the paper's batch method; the batches share
    the database, whose own variance the recycling study measures); the 1e8-history thorax
    plan and the 1e7-history paper-field plan (both tallies, each with its own
    tuned launch configuration); the denoiser's
    forward pass (256x256x128 volume) and training step (128^3 crop: forward,
    backward, Adam), each the best of three after a warm-up."""
    import numpy as np
    import torch
    from paper_1011_2188_amd import fdc as F
    from paper_1011_2188_amd import inputs as I
    from paper_1011_2188_amd import workloads as W

    def best(f, n=3):
        f()
        torch.cuda.synchronize()
        ts = []
        for _ in range(n):
            t = time.perf_counter()
            f()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return min(ts)

    from paper_1011_2188_amd import autotune as A
    out = {}
    nb = 6
    doses = torch.empty((nb, nvox), dtype=torch.float64, device="cuda")
    # the energy-tally-only runs get their own launch configuration (untimed tuning)
    cache_cands = ([dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=1, tally_mode=m,
                         source_order=0) for m in (1, 2)]
                   + [dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=u, tally_mode=2,
                           source_order=1) for u in (1, 2, 4, 8)])
    eq1_launch, _ = A.tune(c, [plan], 0, use_cache=False, candidates=cache_cands, reps=1)
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
    c.set_launch_config(**launch)
    out["batch_method_eq1"] = {"batches": nb, "histories": n_tot, "seconds": tb, "histories_per_s": n_tot / tb,
                               "launch": eq1_launch,
                               "mean_uncertainty": ub, "histories_to_2pct": n2,
                               "seconds_to_2pct": n2 / (n_tot / tb)}
    log(f"batch method: {ub:.4%} at {n_tot} histories -> 2% in {n2 / (n_tot / tb):.4g} s")
    ph, sp, _ = W.thorax()
    p = c.load_phantom(ph)
    c.add_beam_spots(p, sp)
    n = int(sp["n_histories"].sum())

    # the thorax plan gets its own launch configuration (untimed tuning over the
    # LDS-cache candidates), then the slab's is restored
    th_launch, _ = A.tune(c, [p], use_cache=False, candidates=cache_cands, reps=1)

    def thorax_run():
        c.reset_plan(p)
        c.run_histories([p], F.FDC_RUN_VARIANCE)
    t = best(thorax_run)
    out["thorax_1e8"] = {"seconds": t, "histories_per_s": n / t, "launch": th_launch,
                         "workload": "thorax 256x256x128 x 2 mm, 3 fields x 2000 spots, 1e8 histories, both tallies"}
    log(f"thorax: {n / t:.4g} histories/s")
    # the paper's kind of test case: 121 MeV disk field (radius 4 cm) on 1 x 1 x 2.5 mm voxels;
    # its own database (1e5 tracks at 121 MeV) in a second context
    ph, sp, db_pf = W.paper_field()
    c2 = F.Context(0, 1, table=I.HU_TABLE_DEFAULT)
    c2.load_track_db(db_pf)
    p2 = c2.load_phantom(ph)
    c2.add_beam_spots(p2, sp)
    pf_launch, _ = A.tune(c2, [p2], use_cache=False, candidates=cache_cands, reps=1)
    n2 = int(sp["n_histories"].sum())
    d2 = torch.empty(ph.hu.size, dtype=torch.float64, device="cuda")
    v2 = torch.empty(ph.hu.size, dtype=torch.float64, device="cuda")

    def pf_run():
        c2.reset_plan(p2)
        c2.run_histories([p2], F.FDC_RUN_VARIANCE)
    t2 = best(pf_run)
    c2.compute_dose(p2, d2, v2)
    u2, _, _ = c2.mean_uncertainty(p2, d2, v2, 0.5)
    c2.close()
    out["paper_field_1e7"] = {"seconds": t2, "histories_per_s": n2 / t2, "launch": pf_launch,
                              "mean_uncertainty": u2, "seconds_to_2pct": n2 * (u2 / 0.02) ** 2 / (n2 / t2),
                              "workload": "thorax 352x240x72 x 1x1x2.5 mm, one 121 MeV field of circular "
                                          "cross-section (radius 4 cm), 1e7 histories, DB 1e5 tracks at 121 MeV, "
                                          "both tallies"}
    log(f"paper field: {n2 / t2:.4g} histories/s, {u2:.4%} at 1e7")
    c.set_launch_config(**launch)
    from paper_1011_2188_amd import experiments as X
    den = X.denoiser_rate(3)
    out["denoiser"] = {"forward_ms_256x256x128": den["forward_ms"], "forward_tflops": den["forward_tflops"],
                       "train_step_ms_128cube": den["train_step_ms"], "train_tflops": den["train_tflops"],
                       "peak_tflops_bf16": den["peak_tflops_bf16"],
                       "seconds_to_2pct_denoised": None,
                       "note": "denoised time to 2% at equal gamma pass rate: not reached (the plain method is "
                               "faster on thorax-like plans; see profiles/denoiser_study_thorax.md)"}
    log(f"denoiser: forward {den['forward_ms']:.2f} ms, training step {den['train_step_ms']:.2f} ms")
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(ph, sp, db, target_s=20.0):
    """The oracle as it stands, all host threads, on a bounded sample of the
    same workload (every spot, up to its full history count, sized for about
    target_s seconds from a probe run), scaled to histories/s."""
    import numpy as np
    from oracle import oracle as O
    threads = int(os.environ.get("ORACLE_THREADS", min(os.cpu_count() or 1, 16)))
    probe = 4000
    t = time.perf_counter()
    O.replay(db, ph, sp, h_count=np.full(len(sp), probe, np.uint64), threads=threads)
    rate = probe * len(sp) / (time.perf_counter() - t)
    per_spot = int(max(probe, min(400_000, rate * target_s / len(sp))))
    t = time.perf_counter()
    O.replay(db, ph, sp, h_count=np.full(len(sp), per_spot, np.uint64), threads=threads)
    dt = time.perf_counter() - t
    n = per_spot * len(sp)
    return {"value": n / dt, "unit": "histories/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sp)} spots x {per_spot} histories of the same workload ({n} histories, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-variance", action="store_true", help="energy tally only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 2%% verification run and the thorax, paper-field and denoiser timings")
    ap.add_argument("--launch", default="tune",
                    help="'tune' (autotune before the warm-up, untimed) or waves_per_block,blocks_per_cu,"
                         "tally_slots,units_per_wave[,tally_mode]")
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
    ph, sp, db = W.slab()
    log(f"inputs generated in {time.perf_counter() - t:.1f} s: DB {db.steps.shape[0]} steps, "
        f"{db.n_tracks} tracks, {db.n_bins} bins")
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
        launch, timings = A.tune(c, [plan], flags, reps=2, use_cache=False)
        log(f"autotuned in {time.perf_counter() - t:.1f} s: {launch}")
        for k, v in sorted(timings.items(), key=lambda kv: kv[1]):
            log(f"  {v * 1e3:8.2f} ms  {k}")
    else:
        v = [int(x) for x in args.launch.split(",")]
        launch = dict(zip(LAUNCH_KEYS, v))
        c.set_launch_config(**launch)
    kernel = ("transport_kernel" if not launch.get("tally_slots", 0) else
              "transport_cache_kernel" if launch.get("tally_mode", 0) == 2 else "transport_lds_kernel")
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
    if variance:
        r = c.read_dose_and_variance(plan, raw=False, stream=stream)
        d, v = r["dose"], r["var"]
        sel = d > 0.5 * d.max()
        u0 = float(np.mean(np.sqrt(np.maximum(v[sel], 0)) / d[sel]))
        n2 = hist_per_step * (u0 / 0.02) ** 2
        out["mean_uncertainty_at_1e7"] = u0
        out["histories_to_2pct"] = n2
        out["seconds_to_2pct"] = n2 / value
        assert r["deposited"] + r["escaped"] == r["incident"], "energy identity violated"
        log(f"mean uncertainty {u0:.4%} at {hist_per_step} histories -> 2% at {n2:.3g} histories, "
            f"{n2 / value:.3g} s")
    if variance and not args.no_extras:
        # verification: a plan of the same spots with N_2% histories in total, run
        # and finalised (dose, Eq. (2) variance, mean uncertainty on the device),
        # best of three after a warm-up
        sp2 = sp.copy()
        per = int(np.ceil(n2 / len(sp)))
        sp2["n_histories"] = per
        plan2 = c.load_phantom(ph)
        c.add_beam_spots(plan2, sp2)
        n2_run = per * len(sp)
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

    bph = slab_bytes_per_history(variance, launch.get("source_order", 0))
    achieved = bph * hist_per_step / (kern_ms * 1e-3) / 1e9
    updates = SLAB_G * (2.0 if variance else 1.0) * hist_per_step / (kern_ms * 1e-3)
    traffic = measured_traffic(launch)
    result = {
        "metric": METRIC, "value": value, "unit": "histories/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "slab phantom 128^3 x 1 mm (bone z 4-6 cm, lung z 8-12 cm), 25 spots "
                               "70-230 MeV, 1e7 histories per step, DB 33 bins x 1e4 tracks, int64 "
                               "fixed-point tallies" + (" + squared-energy tally" if variance else ""),
                   "histories_per_step": hist_per_step, "variance": variance, "launch": launch},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel, "kernel_ms": kern_ms,
                     "bytes_per_history": bph, "tally_updates_per_s": updates},
        **out,
    }
    if not args.no_extras:
        result["extras"] = extras(c, plan, nvox, hist_per_step, launch, log)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        result["cpu_baseline"] = cpu_baseline(ph, sp, db)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
