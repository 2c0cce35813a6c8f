#!/usr/bin/env python
"""Benchmark of the LSRTM hot path on one MI355X.

Workload (default): the 2D data-domain LSRTM configuration -- seeded
faulted-layered model, 737 x 240 nodes at 12.5 m (280 x 777 padded with a
20-cell CPML), 120 shots at 25 m depth every 75 m, 369 receivers, 15 Hz
Ricker, nt = 4000, dt = 1 ms, FP32 propagation -- solved by CGNR.  Observed
data are Born data of the seeded true perturbation (synthetic).

One "step" = one CGNR iteration over all 120 shots: a Born pass, a migration
pass (checkpoint replay + adjoint + imaging), FP64 inner products and vector
updates, all in the HIP library.  Timed region: K iterations after W warm-up
iterations, bracketed by device synchronisation, every pass of every launch
group replayed from its captured HIP graph.

value = grid-point updates per second of the two operator passes
        2 * (sum over shots of padded nodes) * nt * K / time   [Gpts/s]

Launch configuration: 32 shots per launch group (balanced to 4 groups of 30)
and 32 x 16 tiles for every phase, the autotuner's pick for this workload on
MI355X; --shots-per-launch -1 --tile -1 --tile-adj-a -1 tunes again (per-phase
shapes included).

Also reported: the roofline of the dominant time step (its minimum bytes per
padded node plus the strips' CPML memories, times the nodes of a launch group,
over the summed average durations of the step's kernels, against the 8 TB/s
HBM peak; kernel durations from one further, untimed iteration in which the
runtime stamps the start and end of every 16th step's kernels), the streaming
rate of a 1 GiB axpy and of the stencils' array mixes without the stencil
(lsrtm_stream_mix: in order, and for a 3D workload in the 3D tiles' order),
the Born and migration passes timed on their own (grid-point updates per
second, and field updates per second counting the two wavefields of every
time step), the plain per-shot CG-iteration time (one launch per
shot, measured on a sample of shots and scaled by the shot count), the
uneven-aperture workload batched against shot by shot, and the FP64 oracle
timed on the host cores on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gpts/s Born+adjoint stencil & % HBM peak; CG-iter time batched vs plain FP32"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per padded node and launch (FP32, interior node,
# every array read once and written once; CPML strips excluded).
BYTES_PER_PT = {
    2: {"born_v": 48, "born_p": 40, "bg_v": 32, "bg_p": 24, "adj_a": 36, "adj_b": 36},
    3: {"born_v": 64, "born_p": 48, "bg_v": 44, "bg_p": 28, "adj_a": 44, "adj_b": 44},
    # fused 2D schedule: one kernel per step, reported under the velocity-phase class
    "2f": {"born_v": 64, "bg_v": 44, "adj_a": 64},
}
KERNEL_SYMBOL = {"born_v": "k2_v<*, true, false>", "born_p": "k2_p<*, true, false>",
                 "bg_v": "k2_v<*, false, true>", "bg_p": "k2_p<*, false, true>",
                 "adj_a": "k2_a", "adj_b": "k2_b"}
# Minimum HBM bytes of one whole time step per padded node (every array of
# the step read once and written once), and the kernels that make up the
# step in the two-phase schedule.  Every node of a CPML strip adds 16 B per
# axis whose strip it lies in (two memories read and written).
STEP_BYTES = {2: {"born": 68, "replay": 48, "adjoint": 64}, 3: {"born": 88, "replay": 64, "adjoint": 80}}
STEP_KERNELS = {"born": ("born_v", "born_p"), "replay": ("bg_v", "bg_p"), "adjoint": ("adj_a", "adj_b")}
STRIP_BYTES = 16


def strip_nodes(w):
    """Sum over shots and axes of the padded nodes inside that axis' two
    absorbing strips."""
    tot = 0
    for win in w.win:
        N = [(hi - lo) + 2 * w.npml for lo, hi in win]
        for a in range(len(N)):
            other = 1
            for b in range(len(N)):
                if b != a:
                    other *= N[b]
            tot += 2 * min(w.npml, N[a]) * other
    return tot


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources of the stencil kernels a workload runs (a change to any of them
# makes its committed counter profile stale).
KERNEL_SOURCES = {2: ("common.h", "kern2d.hip", "kern2f.hip"),
                  3: ("common.h", "kern3d.hip")}


def kernel_source_hash(ndim=2):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[ndim]:
        h.update(open(os.path.join(ROOT, "paper_2508_10405_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def read_traffic(workload_tag, kernel, pts_per_launch, ndim=2):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC
    summary (calibrated bytes per padded node times the nodes of a launch),
    or None when it is missing or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", f"pmc_{workload_tag}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        line = line.strip()
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha") != kernel_source_hash(ndim):
        return None
    v = vals.get(f"traffic_bytes_per_point.{kernel}")
    return float(v) * pts_per_launch if v not in (None, "", "null") else None


# Array mixes of the stencil phases (reads, writes per node): the 3D Born
# velocity phase reads 10 arrays and writes 6, its pressure phase 10 and 2,
# the replay phases 5 and 6 / 5 and 2.
MIXES = ((10, 6), (10, 2), (5, 6), (5, 2))


def mix_calibration(ctx, torch, dev, w, reps=3):
    """Streaming rate of the stencils' array mixes without the stencil
    (lsrtm_stream_mix: every element of nread arrays read once, of nwrite
    arrays written once), walking the elements in order and, for a 3D
    workload, in the 3D tiles' y-march order over its padded grid; the best
    of reps passes per mix."""
    grid = None
    if w.ndim == 3:
        N = [(hi - lo) + 2 * w.npml for lo, hi in w.win[0]]
        ldz = (N[0] + 31) // 32 * 32
        grid = (N[0], N[1], N[2], ldz)
        n = ldz * N[1] * N[2]
    else:
        n = 1 << 26
    buf = torch.zeros(16 * n, device=dev)
    out = {"floats_per_array": n, "grid": list(grid) if grid else None}
    for nr, nw in MIXES:
        for order, g in (("flat", None), ("march", grid)):
            if order == "march" and g is None:
                continue
            ctx.stream_mix(buf, n, nr, nw, g)
            ms = min(ctx.stream_mix(buf, n, nr, nw, g) for _ in range(reps))
            out[f"{nr}r{nw}w_{order}_GBs"] = 4.0 * (nr + nw) * n / (ms * 1e-3) / 1e9
    del buf
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
def cpu_worker(args):
    """FP64 oracle on one shot of the workload: Born + migration of nt_s steps."""
    os.environ["OMP_NUM_THREADS"] = "1"
    import numpy as np
    from oracle import lsrtm_oracle as O
    from paper_2508_10405_amd import synth
    shot, nt_s = args
    w = synth.config2(nt=nt_s)
    prob = O.Problem(w.h, w.dt, nt_s, w.npml, w.pml_R, w.pml_freq, [w.win[shot]], [w.src[shot]],
                     [w.rec[shot]], w.wavelet[shot:shot + 1].astype(np.float64))
    lnvp, lnip = w.lnvp.astype(np.float64), w.lnip.astype(np.float64)
    t0 = time.perf_counter()
    dd = O.born(prob, lnvp, lnip, w.dm.astype(np.float64))
    O.adjoint(prob, lnvp, lnip, dd)
    return time.perf_counter() - t0


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(nt_s, workers, padded_per_shot):
    from multiprocessing import get_context
    ctx = get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        times = pool.map(cpu_worker, [(s, nt_s) for s in range(workers)])
    wall = time.perf_counter() - t0
    busy = max(times)
    gpts = workers * 2 * padded_per_shot * nt_s / busy / 1e9
    return {"value": gpts, "unit": "Gpts/s", "cores": workers, "kind": "oracle", "cpu": cpu_model(),
            "host_cores": os.cpu_count(),
            "sample": f"{workers} shots x {nt_s} of 4000 steps (Born + migration, one shot per "
                      f"process, FP64 numpy); slowest process {busy:.1f} s, wall {wall:.1f} s; "
                      f"{workers} processes = the host cores allotted to one GPU "
                      f"({os.cpu_count()} logical cores on the host)"}


# ---------------------------------------------------------------------------
CONFIG3_SHOTS_PER_LAUNCH = 52


def form2_block(lsrtm, synth, torch, dev, steps=2, plain_shots=16):
    """Uneven-aperture workload (256 shots, windows of 200..737 x 240 nodes,
    nt = 4000): CG-iteration time of the batched form (launch groups of up to
    52 shots over one tile table -- 5 groups, about as many padded nodes per
    launch as config 2's groups of 30; about 1.5 % faster than groups of 32 on
    average over interleaved runs, whose spread is 2-4 %, and faster than
    groups of 64 --, every pass replayed from its HIP graph,
    checkpoints and replay cache reused) against the plain form (one launch
    per shot, no graphs, no replay cache) on the same GPU.  The plain form is
    timed on the first plain_shots shots and scaled by padded nodes (per-shot
    passes run one after another); its Born data for those shots are
    compared bit for bit with the batched form's, so both forms have the same
    error against the oracle."""
    import numpy as np
    w = synth.config3()
    padded = w.padded_points()
    ctx = lsrtm.context_for(w, shots_per_launch=CONFIG3_SHOTS_PER_LAUNCH, tile=1, replay_cache_mb=1 << 30)
    sz = ctx.sizes()
    dm = torch.from_numpy(w.dm).to(dev)
    d_obs = ctx.born(dm)
    x = ctx.cgnr_begin(d_obs)
    ctx.cgnr_iterate(x)                       # captures the graphs of the reading passes
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.cgnr_iterate(x)
    torch.cuda.synchronize()
    batched = (time.perf_counter() - t0) / steps
    d_b = [p.cpu().numpy() for p in ctx.split(d_obs)[:plain_shots]]
    ctx.close()
    del ctx, d_obs, x
    torch.cuda.empty_cache()
    P = min(plain_shots, w.nshot)
    wp = synth.Workload(w.name, w.h, w.dt, w.nt, w.npml, w.f0, w.lnvp, w.lnip, w.dm,
                        w.win[:P], w.src[:P], w.rec[:P], w.wavelet[:P])
    cp = lsrtm.context_for(wp, shots_per_launch=1, tile=1, graph=False)
    dp = cp.born(dm)
    same = all(np.array_equal(a.cpu().numpy(), b) for a, b in zip(cp.split(dp), d_b))
    xp = cp.cgnr_begin(dp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cp.cgnr_iterate(xp)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    cp.close()
    del cp, dp, xp
    torch.cuda.empty_cache()
    plain = tp * padded / wp.padded_points()
    return {"workload": "2D LSRTM, 256 shots on uneven windows of 200..737 x 240 nodes, nt=4000, 15 Hz",
            "shots": w.nshot, "padded_points": padded, "groups": sz["groups"],
            "shots_per_launch": sz["shots_per_launch"], "ckpt_every": sz["ckpt_every"],
            "replay_cache_segments": sz["replay_cache_segments"], "graphs": True,
            "cg_iter_s_batched": batched, "gpts_batched": 2.0 * padded * w.nt / batched / 1e9,
            "cg_iter_s_plain": plain, "plain_sample": f"{P} shots, one launch per shot, scaled by padded nodes",
            "speedup": plain / batched, "plain_bitwise_equal_to_batched": same}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plain-shots", type=int, default=12,
                    help="shots of the plain per-shot CG iteration sample (0 = skip)")
    ap.add_argument("--cpu-steps", type=int, default=100, help="time steps of the oracle sample")
    ap.add_argument("--cpu-workers", type=int, default=0, help="oracle processes (0 = min(16, cores))")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-passes", action="store_true",
                    help="skip the separately timed Born and migration passes (long 3D runs)")
    ap.add_argument("--no-config3", action="store_true",
                    help="skip the uneven-aperture (batched vs per-shot) block of the default run")
    ap.add_argument("--calibrate", action="store_true",
                    help="accepted for the counter-profile commands; the 1 GiB axpy of known traffic "
                         "(streaming rate, counter calibration) always runs")
    ap.add_argument("--shots-per-launch", type=int, default=None,
                    help="shots per launch group; -1 = autotuned together with the tile shape "
                         "(default: 32 for the 2D workloads, the autotuner's pick on MI355X; "
                         "autotuned for config5)")
    ap.add_argument("--tile", type=int, default=None,
                    help="tile shape id; -1 = autotuned (default: 1 = 32 x 16 for the 2D workloads)")
    ap.add_argument("--tile-v", type=int, default=None,
                    help="tile shape id of the velocity phases (-1 = the stencil tile; default: -1 for "
                         "the 2D workloads, 1 = 64 x 8 x 32 for config5)")
    ap.add_argument("--tile-adj-a", type=int, default=None,
                    help="tile shape id of the adjoint A phase (-1 = the stencil tile, the default; the "
                         "autotuner's pick for the 2D workloads on MI355X)")
    ap.add_argument("--replay-cache-gb", type=float, default=-1,
                    help="HBM that may keep the background replays of the last checkpoint segments across "
                         "CG iterations (they depend on the background only); -1 = what the memory plan "
                         "leaves (default), 0 = off")
    ap.add_argument("--fused", action="store_true",
                    help="2D: one fused kernel per time step instead of the two-phase step (default two-phase)")
    ap.add_argument("--tune-steps", type=int, default=24)
    ap.add_argument("--pcgnr", type=int, default=0,
                    help="also run N CGNR and N pseudo-Hessian-preconditioned CGNR iterations from x = 0 "
                         "and report both misfit curves (untimed for value)")
    ap.add_argument("--psf", type=int, default=0,
                    help="also run image-domain LSRTM with the PSF Hessian: scatterers every N nodes, "
                         "10 multi- and 10 monoparameter CGNR iterations on the RTM image (untimed for value)")
    ap.add_argument("--wiener", type=int, default=0,
                    help="also run the nonstationary Wiener deblurring of the RTM image with blocks of N "
                         "nodes (untimed for value)")
    ap.add_argument("--nt", type=int, default=0,
                    help="truncate the time axis to nt steps (0 = the workload's own); for counter "
                         "profiles, whose per-launch figures do not depend on nt")
    ap.add_argument("--workload", default="config2", choices=("config2", "config3", "config5"),
                    help="config2 = the benchmark workload; config3 (uneven apertures) and config5 (3D, "
                         "BF16 checkpoints) are measured on request")
    args = ap.parse_args()
    if args.shots_per_launch is None:
        args.shots_per_launch = -1 if args.workload == "config5" else 32
    if args.tile is None:
        args.tile = -1 if args.workload == "config5" else 1
    if args.tile_v is None:
        args.tile_v = 1 if args.workload == "config5" else -1
    if args.tile_adj_a is None:
        args.tile_adj_a = -1
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the shot-parallel "
              "multi-GPU layout is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2508_10405_amd import lsrtm, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    make = {"config2": synth.config2, "config3": synth.config3, "config5": synth.config5}[args.workload]
    w = make(nt=args.nt) if args.nt > 0 else make()
    tag = f"{args.workload}_batched"
    nd = w.ndim
    ckdt = "bf16" if args.workload == "config5" else "f32"
    log(f"[bench] workload {w.name}: {w.nshot} shots, nt={w.nt}, padded points {w.padded_points()}")
    # the timed iterations run as the library runs them for a user: every
    # pass of every launch group replayed from its captured HIP graph
    ctx = lsrtm.context_for(w, shots_per_launch=max(0, args.shots_per_launch), tile=args.tile, timing=False,
                            tile_v=args.tile_v, tile_adj_a=args.tile_adj_a,
                            replay_cache_mb=1 << 30 if args.replay_cache_gb < 0 else int(args.replay_cache_gb * 1024),
                            ckpt_dtype=ckdt, progress=nd == 3, fused=args.fused)
    if args.tile < 0:
        t0 = time.perf_counter()
        tuned = ctx.autotune(nsteps=args.tune_steps, groups=args.shots_per_launch < 0)
        log(f"[bench] autotune {tuned} in {time.perf_counter() - t0:.1f} s")
    sz = ctx.sizes()
    log(f"[bench] plan {sz}")
    btab = BYTES_PER_PT["2f" if (nd == 2 and sz["fused"]) else nd]
    dm = torch.from_numpy(w.dm).to(dev)
    d_obs = ctx.born(dm)
    torch.cuda.synchronize()
    log("[bench] observed data done")
    x = ctx.cgnr_begin(d_obs)
    torch.cuda.synchronize()
    log("[bench] initial migration done")
    for i in range(args.warmup):
        m = ctx.cgnr_iterate(x)
        log(f"[bench] warmup iteration {i}: misfit {m:.6f}")
    torch.cuda.synchronize()
    misfit = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        misfit.append(ctx.cgnr_iterate(x))
        log(f"[bench] step {i}: misfit {misfit[-1]:.6f}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / args.steps
    padded = sz["padded_points"]
    value = 2.0 * padded * w.nt / sec / 1e9

    # per-kernel times: one more CG iteration (untimed for value) with plain
    # launches, every 16th step's stencil kernels stamped with their own start
    # and end by the runtime
    ctx.set_option(lsrtm.OPT_TIMING, 1)
    torch.cuda.synchronize()
    ts0 = time.perf_counter()
    ctx.cgnr_iterate(x)
    torch.cuda.synchronize()
    sec_direct = time.perf_counter() - ts0
    st = ctx.stats()
    ctx.set_option(lsrtm.OPT_TIMING, 0)
    kms = {k: st[k][0] for k in lsrtm.KERNEL_NAMES}
    kcnt = {k: st[k][1] for k in lsrtm.KERNEL_NAMES}
    log(f"[bench] sampled iteration (direct launches, events): {sec_direct:.3f} s")

    # streaming rate of this GPU: a 1 GiB axpy (reads 8 B, writes 4 B per element)
    n_ax = 1 << 28
    a_ax = torch.ones(n_ax, device=dev)
    b_ax = torch.ones(n_ax, device=dev)
    ctx.axpy(0.5, a_ax, b_ax)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        ctx.axpy(0.5, a_ax, b_ax)
    e1.record()
    torch.cuda.synchronize()
    ms_ax = e0.elapsed_time(e1) / 5
    stream_gbs = 12 * n_ax / (ms_ax * 1e-3) / 1e9
    calib = {"kernel": "k_axpy", "elements": n_ax, "read_bytes": 8 * n_ax, "write_bytes": 4 * n_ax,
             "avg_ms": ms_ax, "GBs": stream_gbs}
    del a_ax, b_ax
    log(f"[bench] streaming axpy {stream_gbs:.0f} GB/s")
    calib["stream_mix"] = mix_calibration(ctx, torch, dev, w)
    log(f"[bench] streaming mixes {calib['stream_mix']}")

    # roofline: the dominant time step of the plan, priced at the step's
    # minimum bytes per padded node (each array of one time step read and
    # written once) plus the CPML strip surcharge, over the summed average
    # durations of the step's kernels
    pts_per_launch = padded / sz["groups"]
    strip_per_launch = STRIP_BYTES * strip_nodes(w) / sz["groups"]
    ptag = tag + ("_fused" if (nd == 2 and sz["fused"]) else "")
    kernels = {}
    for k in lsrtm.KERNEL_NAMES:
        if kcnt[k] == 0:
            continue
        t = kms[k] / kcnt[k] * 1e-3
        tr = read_traffic(ptag, k, pts_per_launch, nd) if k in btab else None
        gbs = btab[k] * pts_per_launch / t / 1e9 if k in btab else None
        kernels[k] = {"avg_ms": t * 1e3, "launches_timed": kcnt[k], "GBs": gbs,
                      "frac": gbs / HBM_PEAK_GBS if gbs else None,
                      "counter_GBs": tr / t / 1e9 if tr else None,
                      "above_streaming_rate": (gbs > stream_gbs) if gbs else None}
    steps = {}
    fused = nd == 2 and sz["fused"]
    for name, ks in STEP_KERNELS.items():
        ks = tuple(k for k in ks if k in btab) if fused else ks
        if not ks or any(kcnt[k] == 0 for k in ks):
            continue
        t = sum(kms[k] / kcnt[k] for k in ks) * 1e-3
        byt = STEP_BYTES[nd][name] * pts_per_launch + strip_per_launch
        trs = [read_traffic(ptag, k, pts_per_launch, nd) for k in ks]
        steps[name] = {"kernels": list(ks), "step_ms": t * 1e3, "bytes_per_launch": byt,
                       "GBs": byt / t / 1e9, "frac": byt / t / 1e9 / HBM_PEAK_GBS,
                       "traffic": sum(trs) if all(trs) else None}
    # the dominant step by the event time the sampled iteration spent in it
    dom = max(steps, key=lambda n: sum(kms[k] for k in steps[n]["kernels"])) if steps else None
    ds = steps.get(dom, {})
    dk = max((k for k in btab if kcnt[k]), key=lambda k: kms[k])
    # per-pass rates (outside the timed region): one Born pass, one migration
    # pass, each run once first so that its graphs are captured
    passes = None
    if not args.no_passes:
        dtmp = torch.empty(ctx.data_len, device=dev)
        itmp = torch.empty_like(x)
        ctx.born(x, d=dtmp)
        ctx.adjoint(dtmp, img=itmp)
        torch.cuda.synchronize()
        tb0 = time.perf_counter()
        ctx.born(x, d=dtmp)
        torch.cuda.synchronize()
        tb1 = time.perf_counter()
        ctx.adjoint(dtmp, img=itmp)
        torch.cuda.synchronize()
        tb2 = time.perf_counter()
        del dtmp, itmp
        # per pass: grid-point updates, and field updates counting the two
        # wavefields every time step of the pass stands for (Born: background
        # and scattered; migration: background history and adjoint field,
        # whether the history is replayed or read from the replay cache)
        passes = {"born_s": tb1 - tb0, "migration_s": tb2 - tb1,
                  "born_gpts": padded * w.nt / (tb1 - tb0) / 1e9,
                  "migration_gpts": padded * w.nt / (tb2 - tb1) / 1e9,
                  "born_field_updates_gps": 2 * padded * w.nt / (tb1 - tb0) / 1e9,
                  "migration_field_updates_gps": 2 * padded * w.nt / (tb2 - tb1) / 1e9}
        log(f"[bench] passes {passes}")

    pcg = None
    if args.pcgnr > 0:
        tp0 = time.perf_counter()
        _, minv = ctx.pseudo_hessian(eps_rel=1e-3)
        torch.cuda.synchronize()
        t_ph = time.perf_counter() - tp0
        log(f"[bench] pseudo-Hessian pass {t_ph:.2f} s")
        curves = {}
        for name, pre in (("cgnr", None), ("pcgnr", minv)):
            ctx.set_preconditioner(pre)
            xx = ctx.cgnr_begin(d_obs)
            mm = [1.0]
            for i in range(args.pcgnr):
                mm.append(ctx.cgnr_iterate(xx))
                log(f"[bench] {name} iteration {i}: misfit {mm[-1]:.6f}")
            curves[name] = mm
            del xx
        ctx.set_preconditioner(None)
        pcg = {"iterations": args.pcgnr, "pseudo_hessian_s": t_ph, "eps_rel": 1e-3,
               "cgnr_misfit": curves["cgnr"], "pcgnr_misfit": curves["pcgnr"]}

    psf_out = None
    if args.psf > 0:
        sp = args.psf
        torch.cuda.synchronize()
        ts0 = time.perf_counter()
        psf = ctx.psf_images(sp)
        torch.cuda.synchronize()
        t_img = time.perf_counter() - ts0
        m_rtm = ctx.adjoint(d_obs)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ctx.psf_apply(psf, sp, m_rtm)                     # warm-up
        e0.record()
        for _ in range(5):
            ctx.psf_apply(psf, sp, m_rtm)
        e1.record()
        torch.cuda.synchronize()
        t_mv = e0.elapsed_time(e1) / 5
        res = {}
        for mono in (False, True):
            rhs = m_rtm[1].contiguous() if mono else m_rtm
            tc0 = time.perf_counter()
            _, hist = ctx.psf_cgnr(psf, sp, rhs, 10, mono=mono)
            torch.cuda.synchronize()
            res["mono" if mono else "multi"] = {"misfit": hist, "s": time.perf_counter() - tc0}
        psf_out = {"spacing": sp, "window": 2 * ((sp - 1) // 2) + 1, "psf_images_s": t_img,
                   "matvec_ms": t_mv, "cgnr_multi": res["multi"], "cgnr_mono": res["mono"]}
        log(f"[bench] psf {psf_out}")

    wiener_out = None
    if args.wiener > 0:
        m_rtm = ctx.adjoint(d_obs)
        torch.cuda.synchronize()
        tw0 = time.perf_counter()
        m_rem = ctx.adjoint(ctx.born(m_rtm))
        torch.cuda.synchronize()
        tw1 = time.perf_counter()
        ctx.wiener(m_rtm, m_rem, block=args.wiener)        # plans and buffers
        torch.cuda.synchronize()
        tw2 = time.perf_counter()
        out = ctx.wiener(m_rtm, m_rem, block=args.wiener)
        torch.cuda.synchronize()
        tw3 = time.perf_counter()
        dmt = torch.from_numpy(w.dm).to(dev)
        corr = [float((out[k] * dmt[k]).sum() / (out[k].norm() * dmt[k].norm() + 1e-30)) for k in range(2)]
        corr_rtm = [float((m_rtm[k] * dmt[k]).sum() / (m_rtm[k].norm() * dmt[k].norm() + 1e-30)) for k in range(2)]
        wiener_out = {"block": args.wiener, "remigration_s": tw1 - tw0, "first_call_s": tw2 - tw1,
                      "filter_s": tw3 - tw2, "corr_with_true_dm": corr, "corr_rtm_with_true_dm": corr_rtm}
        log(f"[bench] wiener {wiener_out}")
    ctx.close()
    del ctx, d_obs, x
    torch.cuda.empty_cache()

    # the same batched plan without the replay cache: one CG iteration after a
    # Born pass and the initial migration (checkpoints reused as above)
    no_cache = None
    if sz["replay_cache_segments"] > 0:
        cn = lsrtm.context_for(w, shots_per_launch=sz["shots_per_launch"], tile=sz["tile"],
                               tile_v=sz["tile_v"], tile_adj_a=sz["tile_adj_a"], ckpt_dtype=ckdt, timing=True)
        dn = cn.born(dm)
        xn = cn.cgnr_begin(dn)
        torch.cuda.synchronize()
        tn0 = time.perf_counter()
        cn.cgnr_iterate(xn)
        torch.cuda.synchronize()
        no_cache = time.perf_counter() - tn0
        log(f"[bench] CG iteration without the replay cache: {no_cache:.2f} s")
        cn.close()
        del cn, dn, xn
        torch.cuda.empty_cache()

    # plain per-shot form on a sample of shots
    plain = None
    if args.plain_shots > 0 and nd == 2:
        P = min(args.plain_shots, w.nshot)
        wp = synth.Workload(w.name, w.h, w.dt, w.nt, w.npml, w.f0, w.lnvp, w.lnip, w.dm,
                            w.win[:P], w.src[:P], w.rec[:P], w.wavelet[:P])
        cp = lsrtm.context_for(wp, shots_per_launch=1, tile=args.tile, graph=False)
        dp = cp.born(dm)
        xp = cp.cgnr_begin(dp)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        cp.cgnr_iterate(xp)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp0
        plain = {"cg_iter_s": tp * w.nshot / P, "sample_shots": P, "sample_s": tp}
        log(f"[bench] plain per-shot CG iteration: {tp:.2f} s for {P} shots")
        cp.close()

    form2 = None
    if not args.no_config3 and args.workload == "config2" and args.nt == 0:
        form2 = form2_block(lsrtm, synth, torch, dev)
        log(f"[bench] config3 {form2}")

    cpu = None
    if not args.no_cpu_baseline and args.workload == "config2":
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(args.cpu_steps, workers, padded // w.nshot)
        log(f"[bench] cpu baseline {cpu}")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Gpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": {"config2": "2D LSRTM 737x240 @12.5 m (280x777 padded), 120 shots, 369 receivers, "
                                           "nt=4000, 15 Hz, CGNR step = Born + migration",
                                "config3": "2D LSRTM, 256 shots on uneven windows of 200..737 x 240 nodes, "
                                           "nt=4000, 15 Hz, CGNR step = Born + migration",
                                "config5": "3D LSRTM 400x400x200 @12.5 m (440x440x240 padded), 16 shots, "
                                           "80x80 receivers, nt=2500, 20 Hz, BF16 checkpoints, "
                                           "CGNR step = Born + migration"}[args.workload]
                               + (f" [time axis truncated to nt={w.nt}]" if args.nt > 0 else ""),
                   "shots": w.nshot, "nt": w.nt, "padded_points": padded,
                   "shots_per_launch": sz["shots_per_launch"], "ckpt_every": sz["ckpt_every"],
                   "replay_cache_segments": sz["replay_cache_segments"],
                   "tile": list(lsrtm.tile_shape(nd, sz["tile"])),
                   "tile_v": list(lsrtm.tile_shape(nd, sz["tile_v"])) if sz["tile_v"] >= 0 else None,
                   "tile_adj_a": list(lsrtm.tile_shape(nd, sz["tile_adj_a"])) if sz["tile_adj_a"] >= 0 else None,
                   "ckpt_dtype": ckdt,
                   "ckpt_per_group": bool(sz["ckpt_per_group"]),
                   "schedule": "fused step" if sz["fused"] else "two-phase step",
                   "parallelism": "shots batched on 1 GPU"},
        "roofline": {"bound": "hbm", "kernel": f"{dom} step ({' + '.join(ds['kernels'])})" if ds else None,
                     "achieved": ds.get("GBs"), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ds.get("frac"), "traffic": ds.get("traffic"),
                     "bytes_per_launch": ds.get("bytes_per_launch"), "avg_launch_ms": ds.get("step_ms"),
                     "accounting": "minimum bytes of one time step per padded node plus 16 B per node and "
                                   "axis in the absorbing strips, times the nodes of one launch group, over "
                                   "the summed average durations of the step's kernels",
                     "dominant_kernel": {"kernel": dk, "GBs": kernels[dk]["GBs"], "frac": kernels[dk]["frac"],
                                         "above_streaming_rate": kernels[dk]["above_streaming_rate"]},
                     "streaming_GBs": stream_gbs},
        "steps": steps,
        "cpu_baseline": cpu,
        "cg_iter_s_batched": sec,
        "cg_iter_s_direct_launches": sec_direct,
        "cg_iter_s_plain": plain,
        "cg_iter_s_no_replay_cache": no_cache,
        "speedup_batched_vs_plain": (plain["cg_iter_s"] / sec) if plain else None,
        "config3": form2,
        "misfit": misfit,
        "passes": passes,
        "pcgnr": pcg,
        "psf": psf_out,
        "wiener": wiener_out,
        "kernels": kernels,
        "calibration": calib,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
