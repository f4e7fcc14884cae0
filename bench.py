#!/usr/bin/env python3
"""Benchmark of the FP64 ELBO + gradient hot path on one MI355X.

Workload: the SDSS-shaped field (5 bands of 2048 x 1489 px, 2000 sources, 40% stars,
patch side log-uniform in [21, 101] px, r-band flux log-normal in [50, 1e5] e-), all
sources evaluated per step by the batched path (table build, tile-binned render, one
grid-stride fused adjoint launch, finalize) replayed as a HIP graph.  One step = one
ELBO + gradient of every source; the metric counts (source, pixel) visits per second.

Also reported: the plain per-source form on the same field (one launch per source,
overlapping sources evaluated on the fly), per-phase device times from HIP events, the
roofline of the dominant kernel (the fused adjoint, FP64 ALU bound) and the FP64 CPU
oracle timed on a bounded sample of the same sources on this host's cores, with the
parity of the GPU result on that sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "source-pixel ELBO+grad evals/s (FP64), % FP64 peak; batched vs plain at 1e-9"
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector peak (vendor figure)

# Algorithmic FP64 operations, counted from the formulas the kernels evaluate (add, sub,
# mul, div = 1 each, FMA = 2).  The strip kernels' own elementary functions: table-driven
# exp (256/ln2 scaling, two-part reduction, degree-4 polynomial, table product: 14 FLOPs),
# table-driven log (breakpoint, reduced argument, degree-6 log1p, m ln2 recombination:
# 20 FLOPs), reciprocal (hardware estimate + two Newton steps: 9 FLOPs).  Elsewhere exp = 27
# and log = 78, the FP64 operations of one call of the ROCm device library's exp and log on
# gfx950 (counted in the compiled gfx950 ISA).
EXP_FLOPS = 27
LOG_FLOPS = 78
FEXP_FLOPS = 14
FLOG_FLOPS = 20
FRCP_FLOPS = 9
N_STAR, N_GAL = 3, 42                   # Gaussians per (source, image): 3 star, 3 x (8 + 6) galaxy

# Strip algorithm (what runs): per strip of L rows and per Gaussian, the value and the
# first row ratio at the top row, then per row 2 multiplies for the recurrence plus the
# accumulation.  Both strip passes take the box's table staged in LDS, with the offsets from
# each PSF group's shared centre formed once per group and strip (12 FLOPs), so a seed costs
# 9 FLOPs + 2 exps.  Pass A (profile values) runs in the render's strip pass and its values
# are stored; the fused adjoint runs the pixel terms and pass B (seed again; per row one FMA
# and one (star) or two (galaxy) running-sum adds; per strip the moments from the running
# sums and the fold into the ten intermediates: 11 FLOPs per star, 46 per galaxy component).
# The strip kernels leave out of a work item the Gaussians below exp(-50) of their peak on
# all of its pixels, so the count is taken per evaluated (live) component from the library's
# own work counts (celeste_work_counts); the zero components that pad an odd group to a pair
# are overhead, not counted.
SEED = 9 + 2 * FEXP_FLOPS
GROUP = 12
PASS_A_STRIP = {"star": SEED, "gal": SEED}
PASS_A_VISIT = {"star": 3, "gal": 4}
PASS_B_STRIP = {"star": SEED + 11, "gal": SEED + 46}
PASS_B_VISIT = {"star": 5, "gal": 6}
PIXEL_PER_VISIT = 40 + FLOG_FLOPS + FRCP_FLOPS
GATHER_PER_VISIT = 11


def pass_flops(wc, per_strip, per_visit):
    return (wc["group_strips"] * GROUP + wc["star_strips"] * per_strip["star"]
            + wc["galaxy_strips"] * per_strip["gal"] + wc["star_visits"] * per_visit["star"]
            + wc["galaxy_visits"] * per_visit["gal"])


def full_counts(strips, visits):
    """Work counts with every Gaussian evaluated on every strip (no culling)."""
    return {"strips": strips, "visits": visits, "group_strips": 3 * strips, "star_strips": N_STAR * strips,
            "galaxy_strips": N_GAL * strips, "pad_strips": 0, "star_visits": N_STAR * visits,
            "galaxy_visits": N_GAL * visits, "pad_visits": 0}


def step_flops(wc, render_mode):
    """(fused adjoint, render) algorithmic FLOPs of one step.  Render modes 2 and 3 store the
    own values in the render's strip pass; modes 0 and 1 recompute them in the adjoint (their
    render is counted as the same strip values plus the plane accumulation)."""
    visits = wc["visits"]
    a = pass_flops(wc, PASS_A_STRIP, PASS_A_VISIT)
    b = pass_flops(wc, PASS_B_STRIP, PASS_B_VISIT) + visits * PIXEL_PER_VISIT
    if render_mode in (2, 3):
        return b, a + visits * GATHER_PER_VISIT
    return a + b, a + visits * GATHER_PER_VISIT


# Direct evaluation of the same quantities (one exp per Gaussian per visit), for context.
GAUSS_VALUE = 13 + EXP_FLOPS
DIRECT_ADJ_PER_VISIT = N_STAR * (GAUSS_VALUE + 5) + N_GAL * (GAUSS_VALUE + 21) + 62 + LOG_FLOPS
DIRECT_RENDER_PER_VISIT = N_STAR * (GAUSS_VALUE + 1) + N_GAL * (GAUSS_VALUE + 2) + 12
# Algorithmic HBM bytes per visit of the fused adjoint: x, E, V (float64) read once, plus the
# visit's own stored star/galaxy profile values (2 x float64) in render modes 2 and 3.
ADJOINT_BYTES_PER_VISIT = {0: 24, 1: 24, 2: 40, 3: 40}


def measured_profile(decomposition):
    """The committed rocprofv3 counter summary of the fused adjoint, if it was taken on the
    current kernel sources and the same work decomposition (strips per work item, strip
    rows, render mode: these fix what each wave reads; the launch shape does not); else
    None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "fused_adjoint_sdss_field_2000src.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        prof = json.load(fh)
    h = hashlib.sha256()
    for fn in ("strips.hip", "model.h", "internal.h", "dual.h"):
        with open(os.path.join(ROOT, "paper_1801_10277_amd", "csrc", fn), "rb") as fh:
            h.update(fh.read())
    if prof.get("source_sha256") != h.hexdigest() or prof.get("decomposition") != decomposition:
        return None
    return prof


def strip_count(f, L):
    import numpy as np
    b = f.boxes.astype(np.int64)
    return int(np.sum(b[:, 4] * ((b[:, 3] + L - 1) // L)))


LAUNCH_KEYS = ("chunk", "waves_per_block", "grid_blocks", "dynamic_queue", "strip_rows", "render_mode",
               "n_classes", "tile_h", "tile_w")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(f, theta_gpu_grad, elbo_gpu, seconds, seconds_single):
    """The oracle as it stands on this host, on bounded samples of the same field: OpenMP over
    sources on the host cores OMP_NUM_THREADS allows, then one thread (the oracle's
    per-source gradient called source by source), each with the parity of the GPU result on
    the sources it covered."""
    import numpy as np
    from oracle import oracle as O
    O.build()
    P = O.Problem(f)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    batch = max(cores, 8)
    done, visits, t0 = 0, 0, time.perf_counter()
    rel_e, rel_g = 0.0, 0.0

    def check(s, val3, gi):
        ref = val3[0] + val3[1]
        return abs(elbo_gpu[s] - ref) / abs(ref), float(np.max(np.abs(theta_gpu_grad[s, :27] - gi)) / np.abs(gi).max())

    while time.perf_counter() - t0 < seconds and done < f.n_src:
        srcs = np.arange(done, min(done + batch, f.n_src))
        val, g = O.grad_many(P, srcs)
        b = f.boxes[f.patch_ptr[srcs[0]]:f.patch_ptr[srcs[-1] + 1]]
        visits += int((b[:, 3].astype(np.int64) * b[:, 4]).sum())
        for k, s in enumerate(srcs):
            e_, g_ = check(s, val[k], g[k])
            rel_e, rel_g = max(rel_e, e_), max(rel_g, g_)
        done = srcs[-1] + 1
    dt = time.perf_counter() - t0
    # one thread: the last sources of the field, one oracle call each
    s1, v1, t1 = f.n_src - 1, 0, time.perf_counter()
    n1 = 0
    while time.perf_counter() - t1 < seconds_single and s1 >= done:
        val3, gi, _ = O.source_grad(P, s1)
        b = f.boxes[f.patch_ptr[s1]:f.patch_ptr[s1 + 1]]
        v1 += int((b[:, 3].astype(np.int64) * b[:, 4]).sum())
        e_, g_ = check(s1, val3, gi)
        rel_e, rel_g = max(rel_e, e_), max(rel_g, g_)
        s1 -= 1
        n1 += 1
    dt1 = time.perf_counter() - t1
    return {"value": visits / dt, "unit": "source-pixel ELBO+grad evals/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": "first %d of %d sources of the same field (%d visits, %.1f s), FP64 dual-number "
                      "gradient, OpenMP over sources on %d threads" % (done, f.n_src, visits, dt, cores),
            "single_thread": {"value": v1 / dt1 if dt1 > 0 else None, "cores": 1,
                              "sample": "last %d sources of the field (%d visits, %.1f s), one oracle call "
                                        "per source" % (n1, v1, dt1)}}, rel_e, rel_g, done + n1


def apply_launch(plan, text):
    """--launch chunk,waves_per_block,grid,dynamic,strip_rows,render_mode[,tile_h,tile_w]"""
    vals = [int(v) for v in text.split(",")]
    ch, wpb, grid, dyn, rows, rmode = vals[:6]
    th, tw = vals[6:8] if len(vals) >= 8 else (16, 16)
    plan.set_launch(chunk=ch, waves_per_block=wpb, grid_blocks=grid, dynamic=dyn, strip_rows=rows,
                    render_mode=rmode, tile_h=th, tile_w=tw)


def run_newton(args):
    """Config 3: 1024 sources of the field generator, N trust-region Newton iterations of
    every source (others held at their entry values), all on the device."""
    import numpy as np
    import torch
    from paper_1801_10277_amd import binding as B, synth
    f = synth.field_1024src()
    if args.color_mixture:
        f = synth.with_color_mixture(f, seed=3)
    dev = torch.device("cuda:0")
    plan = B.Plan(f, check_status=False)
    if args.launch:
        apply_launch(plan, args.launch)
    plan.set_hessian_mode(args.hessian_mode)
    theta0 = torch.tensor(f.theta, dtype=torch.float64, device=dev)
    src = np.arange(f.n_src, dtype=np.int32)
    params = B.tr_params()
    e0 = plan.elbo(theta0).cpu().numpy()
    warm = theta0.clone()
    plan.newton(warm, src, 1, params)                       # untimed warm-up
    theta = theta0.clone()
    radius = torch.full((f.n_src,), params.radius0, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e1, radius = plan.newton(theta, src, args.newton_steps, params, radius)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.check_status = True
    plan._status("celeste_newton")
    e1 = e1.cpu().numpy()
    visits = plan.info()["n_visits"]
    npar = plan.info()["n_params"]
    out = {"metric": "Newton trust-region iterations per second (ELBO + gradient + %dx%d Hessian + TR solve per "
                     "source)" % (npar, npar), "value": f.n_src * args.newton_steps / dt, "unit": "source-iterations/s",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "1024 sources, 5 bands x 2048x1489 px, %d iterations, others fixed"
                                  % args.newton_steps, "visits_per_evaluation": visits,
                      "seconds": dt, "visit_iterations_per_s": visits * args.newton_steps / dt,
                      "launch": {k: plan.info()[k] for k in LAUNCH_KEYS}, "hessian_mode": args.hessian_mode,
                      "n_params": npar,
                      "mean_elbo_gain": float(np.mean(e1 - e0)), "min_elbo_gain": float(np.min(e1 - e0)),
                      "sources_improved": int(np.sum(e1 > e0))}}
    print(json.dumps(out), flush=True)


def run_sweep(args):
    """Config 4: 16 overlapping fields x 2 epochs x 5 bands (160 images), 20 000 sources,
    conflict-free batches, block-coordinate-ascent sweeps of Newton steps."""
    import numpy as np
    import torch
    from paper_1801_10277_amd import binding as B, synth
    log("generating the sky region ...")
    t = time.perf_counter()
    f = synth.sky_region_20000src()
    if args.color_mixture:
        f = synth.with_color_mixture(f, seed=3)
    log("region ready in %.1f s: %d images, %d sources, %d boxes, %d visits" % (
        time.perf_counter() - t, f.n_img, f.n_src, len(f.boxes), f.visits()))
    dev = torch.device("cuda:0")
    plan = B.Plan(f, check_status=False)
    if args.launch:
        apply_launch(plan, args.launch)
    plan.set_hessian_mode(args.hessian_mode)
    plan.use_graph(not args.no_graph)
    log("plan: %s" % plan.info())
    theta = torch.tensor(f.theta, dtype=torch.float64, device=dev)
    params = B.tr_params(newton_steps=args.newton_steps)
    if args.schedule == "colour":
        ptr, srcl = plan.color_batches(seed=4)
        sched = "%d conflict-free batches (greedy colouring)" % (len(ptr) - 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        trace = plan.sweep(theta, ptr, srcl, args.sweeps, params)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        trace = trace.cpu().numpy()
        rounds = [len(ptr) - 1] * args.sweeps
    else:
        # Cyclades: a fresh sampling order every epoch, its schedule built inside the timed region
        graph = plan.conflict_graph()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        parts, rounds = [], []
        for k in range(args.sweeps):
            bp, bs, nc, _ = plan.cyclades_batches(seed=4 + k, sample_size=args.sample_size, graph=graph)
            parts.append(plan.sweep(theta, bp, bs, 1, params))
            rounds.append(len(bp) - 1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        trace = np.array([float(parts[0][0])] + [float(t[1]) for t in parts])
        sched = "Cyclades samples of %d sources, %s rounds per epoch" % (
            args.sample_size, "/".join(str(r) for r in rounds))
    plan.check_status = True
    plan._status("celeste_sweep")
    out = {"metric": "block-coordinate-ascent sweeps per second", "value": args.sweeps / dt, "unit": "sweeps/s",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "16 fields x 2 epochs x 5 bands (160 images of 2048x1489 px), %d sources, "
                                  "%s, %d Newton steps per batch visit"
                                  % (f.n_src, sched, args.newton_steps),
                      "schedule": args.schedule, "batches_per_sweep": rounds,
                      "n_params": plan.info()["n_params"],
                      "sweep_graph": not args.no_graph,
                      "launch": {k: plan.info()[k] for k in LAUNCH_KEYS}, "hessian_mode": args.hessian_mode,
                      "seconds": dt, "visits_per_evaluation": plan.info()["n_visits"],
                      "elbo_trace": [float(v) for v in trace],
                      "monotone": bool(np.all(np.diff(trace) >= 0))}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-seconds-single", type=float, default=8.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-hvp", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the one- and 16-source configurations")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner and time the plan's default launch")
    ap.add_argument("--sources", type=int, default=2000)
    ap.add_argument("--launch", type=str, default=None,
                    help="fixed launch chunk,waves_per_block,grid,dynamic,strip_rows,render_mode[,tile_h,tile_w] "
                         "(skips autotune)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 512 MiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--workload", choices=("elbo_grad", "newton", "sweep"), default="elbo_grad")
    ap.add_argument("--realistic", action="store_true",
                    help="field with per-image astrometry, sky maps and brightness-sized patches")
    ap.add_argument("--newton-steps", type=int, default=None)
    ap.add_argument("--sweeps", type=int, default=3)
    ap.add_argument("--schedule", choices=("colour", "cyclades"), default="colour",
                    help="sweep workload: greedy colouring, or Cyclades sampling (Section IV-D)")
    ap.add_argument("--sample-size", type=int, default=2000, help="Cyclades sample size")
    ap.add_argument("--no-graph", action="store_true",
                    help="sweep workload: run the sweeps eagerly instead of replaying a captured sweep graph")
    ap.add_argument("--color-mixture", action="store_true",
                    help="newton / sweep workloads: the 43-parameter model (colour prior as a Gaussian "
                         "mixture per type, component responsibilities in each source's row)")
    ap.add_argument("--hessian-mode", type=int, default=0, choices=(0, 1),
                    help="Newton / sweep Hessian rows: 0 closed form (default), 1 tangent passes")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload == "newton":
        args.newton_steps = args.newton_steps or 20
        return run_newton(args)
    if args.workload == "sweep":
        args.newton_steps = args.newton_steps or 5
        return run_sweep(args)

    import numpy as np
    import torch
    from paper_1801_10277_amd import binding as B, synth

    log("generating the field ...")
    t = time.perf_counter()
    f = synth.sdss_field(args.sources, realistic=args.realistic)
    log("field ready in %.1f s: %d sources, %d boxes, %d visits" % (time.perf_counter() - t, f.n_src,
                                                                    len(f.boxes), f.visits()))
    dev = torch.device("cuda:0")
    theta = torch.tensor(f.theta, dtype=torch.float64, device=dev)
    plan = B.Plan(f, check_status=False)
    info = plan.info()
    visits = info["n_visits"]
    elbo = torch.zeros(f.n_src, dtype=torch.float64, device=dev)
    grad = torch.zeros(f.n_src, 48, dtype=torch.float64, device=dev)

    default_launch = {k: info[k] for k in LAUNCH_KEYS}
    tuned = None
    if args.launch:
        apply_launch(plan, args.launch)
        info = plan.info()
    elif not args.no_tune:
        t_tune = time.perf_counter()
        ms = plan.autotune(theta, reps=5)
        info = plan.info()
        tuned = {"launch": {k: info[k] for k in LAUNCH_KEYS}, "median_ms": round(ms, 4),
                 "seconds": round(time.perf_counter() - t_tune, 2),
                 "equals_default": {k: info[k] for k in LAUNCH_KEYS} == default_launch}
        log("autotuned: %s (%.3f ms)" % (tuned["launch"], ms))

    # correctness of this configuration before timing
    plan.check_status = True
    plan.elbo_grad(theta, mode=B.CELESTE_BATCHED, elbo=elbo, grad=grad)
    plan.check_status = False

    plan.use_graph(True)
    for _ in range(args.warmup):
        plan.elbo_grad(theta, elbo=elbo, grad=grad)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.elbo_grad(theta, elbo=elbo, grad=grad)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    value = visits * args.steps / dt
    log("batched: %.3f ms/step, %.3e visits/s" % (ms_step, value))
    # each replay bracketed by HIP events on the launch stream (after the timed region)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in evs:
        e0.record()
        plan.elbo_grad(theta, elbo=elbo, grad=grad)
        e1.record()
    torch.cuda.synchronize()
    replay_ms = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    median_ms = replay_ms[len(replay_ms) // 2]
    log("replays (HIP events): median %.4f ms, min %.4f, max %.4f" % (median_ms, replay_ms[0], replay_ms[-1]))

    # per-phase device time with HIP events on the launch stream (outside the graph)
    plan.use_graph(False)
    plan.profile(True, reset=True)
    n_prof = max(5, min(args.steps, 20))
    for _ in range(n_prof):
        plan.elbo_grad(theta, elbo=elbo, grad=grad)
    phase_ms, calls = plan.profile(False, reset=True)
    phase = [m / calls for m in phase_ms]
    log("phases (ms): tables %.3f render %.3f adjoint %.3f finalize %.3f" % tuple(phase))
    adj_ms = phase[2]
    L = info["strip_rows"]
    strips = strip_count(f, L)
    wc = plan.work_counts(theta)
    assert wc["strips"] == strips and wc["visits"] == visits, (wc, strips, visits)
    adj_flops, render_flops = step_flops(wc, info["render_mode"])
    adj_full, render_full = step_flops(full_counts(strips, visits), info["render_mode"])
    live_per_strip = (wc["star_strips"] + wc["galaxy_strips"]) / strips
    log("live Gaussians per strip %.2f of 45 (+%.2f zero pads); adjoint %.3e FLOPs per launch (%.3e without culling)"
        % (live_per_strip, wc["pad_strips"] / strips, adj_flops, adj_full))
    achieved = adj_flops / (adj_ms * 1e-3) / 1e12
    decomposition = "chunk %d, strip rows %d, render mode %d" % (info["chunk"], info["strip_rows"],
                                                                  info["render_mode"])
    # the committed counter profile was taken on the default field only
    prof = None if (args.realistic or f.n_src != 2000) else measured_profile(decomposition)
    traffic = None if prof is None else prof["bytes_per_launch"]
    counted = None if prof is None else prof["counters"][prof["kernel"]].get("fp64_flops_counted")
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": None if traffic is None else round(traffic),
                "traffic_algorithmic": ADJOINT_BYTES_PER_VISIT[info["render_mode"]] * visits,
                "counted_fp64_tflops": None if counted is None else round(counted / (adj_ms * 1e-3) / 1e12, 3),
                "kernel": "k_adjoint_strips<double, planes, grad, L=%d> (fused own-source forward + adjoint)" % L,
                "flops_per_launch": adj_flops, "flops_per_visit": round(adj_flops / visits, 1),
                "live_gaussians_per_strip": round(live_per_strip, 3),
                "flops_per_launch_without_culling": adj_full,
                "visits_per_launch": visits, "strips_per_launch": strips, "avg_launch_ms": round(adj_ms, 4)}
    whole = (adj_flops + render_flops) / visits * value / 1e12
    direct_equiv = (DIRECT_ADJ_PER_VISIT + DIRECT_RENDER_PER_VISIT) * value / 1e12

    plain = None
    if not args.no_plain:
        plan.elbo_grad(theta, mode=B.CELESTE_PLAIN, elbo=elbo, grad=grad)
        torch.cuda.synchronize()
        n_plain = 3
        t0 = time.perf_counter()
        for _ in range(n_plain):
            plan.elbo_grad(theta, mode=B.CELESTE_PLAIN, elbo=elbo, grad=grad)
        torch.cuda.synchronize()
        pdt = (time.perf_counter() - t0) / n_plain
        plain = {"visits_per_s": visits / pdt, "ms_per_step": 1e3 * pdt}
        log("plain: %.3f ms/step, %.3e visits/s" % (1e3 * pdt, visits / pdt))

    # Hessian-vector products of every source (one tangent pass of the whole path), same field
    hvp = None
    if not args.no_hvp:
        v = torch.zeros_like(grad)
        v[:, :27] = torch.randn(f.n_src, 27, dtype=torch.float64, generator=torch.Generator().manual_seed(7)).to(dev)
        plan.hvp(theta, v)
        torch.cuda.synchronize()
        n_hvp = 10
        t0 = time.perf_counter()
        for _ in range(n_hvp):
            plan.hvp(theta, v)
        torch.cuda.synchronize()
        hdt = (time.perf_counter() - t0) / n_hvp
        hvp = {"ms_per_call": round(1e3 * hdt, 4), "visits_per_s": visits / hdt}
        log("hvp: %.3f ms per call, %.3e visits/s" % (1e3 * hdt, visits / hdt))

    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # the small configurations (one source; 16 sources): plain and batched, eager calls
    small = {}
    if not args.no_small:
        for name, g in (("single_source", synth.single_source()), ("region_16src", synth.region_16src())):
            sp = B.Plan(g, check_status=False)
            th = torch.tensor(g.theta, dtype=torch.float64, device=dev)
            row = {"visits": sp.info()["n_visits"]}
            for mode, label in ((B.CELESTE_PLAIN, "plain"), (B.CELESTE_BATCHED, "batched")):
                sp.elbo_grad(th, mode=mode)
                torch.cuda.synchronize()
                reps = 20
                t0 = time.perf_counter()
                for _ in range(reps):
                    sp.elbo_grad(th, mode=mode)
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t0) / reps
                row[label] = {"ms_per_eval": round(ms, 4), "visits_per_s": row["visits"] / (ms * 1e-3)}
            small[name] = row
            log("%s: plain %.3f ms, batched %.3f ms" % (name, row["plain"]["ms_per_eval"],
                                                        row["batched"]["ms_per_eval"]))
            del sp

    # batched result for the parity sample
    plan.elbo_grad(theta, mode=B.CELESTE_BATCHED, elbo=elbo, grad=grad)
    torch.cuda.synchronize()
    cpu, parity = None, None
    if not args.no_cpu:
        cpu, rel_e, rel_g, n_checked = cpu_baseline(f, grad.cpu().numpy(), elbo.cpu().numpy(), args.cpu_seconds,
                                                    args.cpu_seconds_single)
        parity = {"sources_checked": int(n_checked), "max_rel_err_elbo": rel_e, "max_rel_err_grad": rel_g}
        log("cpu oracle: %.3e visits/s on %d cores" % (cpu["value"], cpu["cores"]))

    out = {"metric": METRIC, "value": value, "unit": "source-pixel ELBO+grad evals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "SDSS-shaped field%s, %d sources, 5 bands x 2048x1489 px, batched "
                                  "fused launch replayed as a HIP graph"
                                  % (" with astrometry, sky maps and brightness-sized patches" if args.realistic
                                     else "", f.n_src),
                      "sources": f.n_src, "visits_per_step": visits, "form": "batched",
                      "launch": {k: info[k] for k in LAUNCH_KEYS}, "autotune": tuned,
                      "replay_ms_hip_events": {"median": round(median_ms, 4), "min": round(replay_ms[0], 4),
                                               "max": round(replay_ms[-1], 4), "n": len(replay_ms),
                                               "visits_per_s_at_median": visits / (median_ms * 1e-3)},
                      "phase_ms": [round(v, 4) for v in phase],
                      "path_flops_per_visit": round((adj_flops + render_flops) / visits, 1),
                      "path_tflops": round(whole, 3),
                      "path_frac_fp64_peak": round(whole / FP64_PEAK_TFLOPS, 4),
                      "direct_formula_flops_per_visit": DIRECT_ADJ_PER_VISIT + DIRECT_RENDER_PER_VISIT,
                      "direct_formula_equivalent_tflops": round(direct_equiv, 3),
                      "plain": plain,
                      "batched_vs_plain": (value / plain["visits_per_s"]) if plain else None,
                      "hvp_all_sources": hvp,
                      "small_configs": small or None,
                      "parity_vs_oracle": parity},
           "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
