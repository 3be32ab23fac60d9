"""Benchmark of the StePS direct-summation hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 3]
                    [--no-cpu-baseline] [--no-modes] [--no-batch] [--no-glass]

A step is one comoving KDK step (kick + drift, one O(N^2) pair sum, kick) of
the whole particle set, with state resident in HBM.  Default workload
(workload 3): N = 2^21 stereographically projected particles, D = 300 Mpc,
r_max = 3000 Mpc, LCDM (0.3089 / 0.6911 / 67.74), sigma 1%, Zel'dovich
velocities, FP64, stepping along a log-uniform grid from a = 0.02 (200 steps
to a = 1, the step of workload 2).  The value is ordered pair interactions
per second over the timed steps, N^2 per step: an ordered-pair equivalent,
since the default kernels evaluate each unordered pair once for both
particles; N(N - 1) per step is reported beside it.

Also reported on the same JSON line:
  roofline     -- force kernel: 20 flop per ordered pair (convention) over
                  its average launch time (HIP events on its own stream),
                  against the FP64 vector peak 78.6 TFLOP/s (FP64 vector and
                  FP64 matrix-core instructions issue through one pipe on
                  gfx950, whose peak that is), or the FP32 one in mixed mode;
  cpu_baseline -- the CPU FP64 oracle on a bounded seeded sample of i rows
                  against all N j, on every host thread and on one;
  modes        -- force-kernel pair rate in FP64 and both mixed modes at the
                  same N, with the relative force error against the oracle
                  on 65 536 sampled rows (median, max, binned);
  workload2    -- the same step timing and modes table at N = 2^18;
  config2_200  -- workload 2 as specified: all 200 KDK steps a 0.02 -> 1.0
                  at N = 2^18, with energies and momentum at both ends;
  batch, batch_small, glass, periodic -- the ensemble, glass-relaxation and
                  periodic-box legs.

--workload 2 makes workload 2 the headline; --workload 5 runs N = 2^22 for
50 steps in mixed precision and in FP64 with the energy checks.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TF = 78.6
FP32_PEAK_TF = 157.3
FLOP_PER_PAIR = 20
NOMINAL_CLOCK_GHZ = 2.4
METRIC = "pair interactions/s (ordered-pair equivalent, whole KDK step)"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=3, choices=[2, 3, 5])
    ap.add_argument("--no-glass", action="store_true",
                    help="skip the glass-relaxation and periodic legs")
    ap.add_argument("--no-li-study", action="store_true",
                    help="workload 5: skip the Layzer-Irvine step-convergence "
                         "study at N = 2^17")
    ap.add_argument("--li-study-only", action="store_true",
                    help="workload 5: only the Layzer-Irvine step-convergence "
                         "study at N = 2^17")
    ap.add_argument("--precision", default="fp64",
                    choices=["fp64", "mixed", "kahan"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the precision-mode tables and their oracle rows")
    ap.add_argument("--oracle-rows", type=int, default=65536,
                    help="oracle rows behind the headline's modes table")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the workload-2 and 200-step legs")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-member ensemble comparison")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched 64-member ensemble (no "
                         "sequential comparison; for profiling its kernels)")
    ap.add_argument("--periodic-only", action="store_true",
                    help="run only the periodic-box leg (for profiling its "
                         "kernels)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the single-thread oracle sample")
    ap.add_argument("--tile", default=None, metavar="R,TJ,JSPLIT,VARIANT",
                    help="force the force kernel's launch shape (a compiled "
                         "variant; JSPLIT 0 = the built-in split), e.g. "
                         "1,256,0,6 for the one-sided matrix-core kernel")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="finish with one device copy of MIB MiB (a kernel of "
                         "known traffic, to scale HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kdk_grid(ps, workload):
    """The step grid of a workload: its own log-uniform grid, or for
    workload 3 (one evaluation per mode as specified) the 200-step grid
    a 0.02 -> 1.0 of workload 2."""
    import numpy as np
    if workload != 3:
        return ps.a_grid()
    k = np.arange(201, dtype=np.float64)
    g = ps.a0 * (1.0 / ps.a0) ** (k / 200)
    g[-1] = 1.0
    return g


def kdk_leg(st, dev, ps, grid, steps, warmup, precision, tile=None,
            workload=None):
    """Times `steps` KDK steps after `warmup` untimed ones, from the set's
    initial state along `grid`; returns the timing, the force kernel's
    roofline and the final state."""
    import torch
    n = ps.n
    c = ps.cosmo
    cosmo = st.Cosmology(c.H0, c.omega_m, c.omega_l, c.omega_r)
    stream = torch.cuda.current_stream()
    ctx = st.Context(0, precision=precision, flags=st.STEPS_PROFILE,
                     stream=stream)
    if tile:
        ctx.set_tile(*(int(x) for x in tile.split(",")))
    pos, vel, mass, soft = dev(ps.pos), dev(ps.vel), dev(ps.mass), dev(ps.soft)
    acc = st.steps_forces(pos, mass, soft, ctx=ctx)
    if warmup + steps > len(grid) - 1:
        raise SystemExit("at most %d steps on this grid" % (len(grid) - 1))
    k = 0
    for _ in range(warmup):
        st.steps_step(pos, vel, mass, soft, acc, grid[k], grid[k + 1] - grid[k],
                      cosmo, ctx=ctx)
        k += 1
    torch.cuda.synchronize()
    ctx.force_timing(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        st.steps_step(pos, vel, mass, soft, acc, grid[k], grid[k + 1] - grid[k],
                      cosmo, ctx=ctx)
        k += 1
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    force_ms, force_cnt = ctx.force_timing(reset=True)
    t = ctx.get_tile(n)
    ctx.close()
    assert bool(torch.isfinite(pos).all()) and bool(torch.isfinite(acc).all())
    pairs = float(n) * n
    kern_ms = force_ms / max(1, force_cnt)
    achieved = FLOP_PER_PAIR * pairs / (kern_ms * 1e-3) / 1e12
    peak = FP64_PEAK_TF if precision == "fp64" else FP32_PEAK_TF
    log("n=%d %s: %d steps, %.2f ms/step, %.3e pairs/s; force kernel %.2f ms "
        "(%d launches), %.3f of peak"
        % (n, precision, steps, 1e3 * elapsed / steps, pairs * steps / elapsed,
           kern_ms, force_cnt, achieved / peak))
    name = force_kernel_name(precision, t)
    return {
        "n": n, "steps": steps, "warmup": warmup,
        "a_range": [float(grid[warmup]), float(grid[warmup + steps])],
        "ms_per_step": 1e3 * elapsed / steps,
        "pairs_per_s": pairs * steps / elapsed,
        "pairs_distinct_per_s": float(n) * (n - 1) * steps / elapsed,
        "tile": t,
        "roofline": {
            # the FP64 kernels (vector or matrix-core) are priced at the FP64
            # vector peak: on gfx950 FP64 vector and FP64 matrix-core
            # instructions issue through the one FP64 pipe with that peak
            "bound": "alu", "pipe": "fp64" if precision == "fp64" else "fp32",
            "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": profiled_traffic(precision, t, workload),
            "kernel": name, "kernel_ms": kern_ms,
            "kernel_launches": force_cnt,
            "flop_per_pair": FLOP_PER_PAIR,
            "pair_convention": "N^2 ordered pairs per evaluation (ordered-pair "
                               "equivalent: the symmetric kernels evaluate "
                               "N(N-1)/2 unordered pairs)",
            "counters": counter_roofline(profile_path(precision, t, workload),
                                         achieved / peak)},
    }, (pos, vel, acc)


def oracle_rows(ps, rows, seed, chunk=8192, first_timed=0):
    """The oracle's S and kappa on `rows` seeded-sampled i of the set (all j),
    in chunks of `chunk` rows on every host thread.  Returns ((idx, S,
    kappa), timing) where timing covers the first `first_timed` rows."""
    import numpy as np
    import oracle
    idx = np.sort(np.random.default_rng(seed).choice(ps.n, rows, replace=False))
    refs, kaps = [], []
    t0 = time.perf_counter()
    timed = None
    for k in range(0, rows, chunk):
        r, kp = oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx[k:k + chunk],
                              want_kappa=True)
        refs.append(r)
        kaps.append(kp)
        done = min(rows, k + chunk)
        if timed is None and first_timed and done >= first_timed:
            timed = (done, time.perf_counter() - t0)
        log("oracle rows %d/%d (%.0f s)" % (done, rows, time.perf_counter() - t0))
    return (idx, np.concatenate(refs, axis=1), np.concatenate(kaps)), timed


def cpu_baseline(ps, timed, seconds):
    """The oracle's pair rate on every host thread (from the first chunks of
    the parity rows, `timed` = (rows, seconds)) and on one thread (a
    bounded sample of about `seconds`), with the extrapolated time of one
    full evaluation."""
    import numpy as np
    import oracle
    n = ps.n
    rng = np.random.default_rng(12345)
    probe = rng.choice(n, 64, replace=False)
    t = time.perf_counter()
    oracle.forces(ps.pos, ps.mass, ps.soft, idx=probe, nthreads=1)
    rate1 = 64 * n / (time.perf_counter() - t)
    m1 = int(min(n, max(64, rate1 * seconds / n)))
    idx1 = np.sort(rng.choice(n, m1, replace=False))
    t = time.perf_counter()
    oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx1, nthreads=1)
    dt1 = time.perf_counter() - t
    single = m1 * float(n) / dt1
    if timed is None:
        m = int(min(n, max(256, 8 * m1)))
        idx = np.sort(rng.choice(n, m, replace=False))
        t = time.perf_counter()
        oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx)
        timed = (m, time.perf_counter() - t)
    rows, dt = timed
    value = rows * float(n) / dt
    log("cpu baseline: %.3e pairs/s on %d threads, %.3e on one"
        % (value, oracle.num_threads(), single))
    return {"value": value, "unit": "pairs/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "FP64 oracle pair sums for %d seeded-sampled i of the "
                      "N=%d set against all j (%.1f s)" % (rows, n, dt),
            "single_thread": {"value": single, "unit": "pairs/s", "cores": 1,
                              "sample": "%d seeded-sampled i against all j "
                                        "(%.1f s)" % (m1, dt1)},
            "extrapolated_full_evaluation_s": float(n) * n / value,
            "extrapolated_full_evaluation_s_single_thread": float(n) * n / single,
            "note": "extrapolated from the sampled rows: every row costs N "
                    "pair terms"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU "
              "path (each GPU would own a block of i-rows and all-gather "
              "positions once per step).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1811_05903_amd as st
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()

    if args.workload == 5:
        print(json.dumps(workload5(st, dev, args)), flush=True)
        return
    if args.batch_only:
        out = {"batch": batch_leg(st, dev, args.batch_steps, sequential=False)}
        copy_calibration(args.copy_calibration)
        print(json.dumps(out), flush=True)
        return
    if args.periodic_only:
        out = {"periodic": periodic_leg(st, dev)}
        copy_calibration(args.copy_calibration)
        print(json.dumps(out), flush=True)
        return

    ps = synth.config(args.workload)
    n = ps.n
    grid = kdk_grid(ps, args.workload)
    log("workload %d: n=%d precision=%s" % (args.workload, n, args.precision))
    leg, _ = kdk_leg(st, dev, ps, grid, args.steps, args.warmup,
                     args.precision, args.tile, args.workload)
    out = {
        "metric": METRIC,
        "value": leg["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-pair/f64-acc",
        "data": "synthetic",
        "config": {"workload": "stereographic sphere N=%d D=%g r_max=%g LCDM, "
                               "%s, KDK steps a %.4f -> %.4f"
                               % (n, ps.params["D"], ps.params["r_max"],
                                  args.precision, leg["a_range"][0],
                                  leg["a_range"][1]),
                   "n": n, "precision": args.precision, "tile": leg["tile"],
                   "parallelism": "single GPU"},
        "pairs_distinct_per_s": leg["pairs_distinct_per_s"],
        "roofline": leg["roofline"],
    }

    rows, timed = None, None
    if not args.no_modes:
        rows, timed = oracle_rows(ps, args.oracle_rows, seed=33,
                                  first_timed=16384)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ps, timed, args.cpu_seconds)
    if not args.no_modes:
        out["modes"] = mode_table(st, ps, rows, dev, reps=3, workload=args.workload)
    if not args.no_extras and args.workload == 3:
        w2 = synth.config(2)
        leg2, _ = kdk_leg(st, dev, w2, w2.a_grid(), 20, 3, "fp64", None, 2)
        w2rows = None
        if not args.no_modes:
            w2rows, _ = oracle_rows(w2, 4096, seed=22)
        leg2["modes"] = mode_table(st, w2, w2rows, dev, reps=3, workload=2)
        out["workload2"] = leg2
    if not args.no_extras:
        out["config2_200"] = config2_full(st, dev)
    if not args.no_batch:
        out["batch"] = batch_leg(st, dev, args.batch_steps)
        # many small members (N_b ~ 256 ... 4096): where one launch per
        # member and step would leave the GPU idle
        out["batch_small"] = batch_leg(st, dev, args.batch_steps, members=256,
                                       n_scale=1.0 / 32)
    if not args.no_glass:
        out["glass"] = glass_leg(st, dev)
        out["periodic"] = periodic_leg(st, dev)
    copy_calibration(args.copy_calibration)
    print(json.dumps(out), flush=True)


def copy_calibration(mib):
    """One device copy of `mib` MiB (a kernel of known traffic, to scale HBM
    byte counters), if mib > 0."""
    import torch
    if not mib:
        return
    src = torch.ones((mib << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log("copy calibration: %d MiB read + %d MiB written" % (mib, mib))


def config2_full(st, dev):
    """Workload 2 as specified: N = 2^18, all 200 log-uniform KDK steps
    a 0.02 -> 1.0, FP64.  Whole-run pair rate; energies (K, W) at both ends;
    the pair-force momentum |sum m S| / sum |m S| at the end (zero up to
    rounding by Newton's third law) and the peculiar momentum."""
    import numpy as np
    import torch
    import synth
    ps = synth.config(2)
    n, grid, c = ps.n, ps.a_grid(), ps.cosmo
    cosmo = st.Cosmology(c.H0, c.omega_m, c.omega_l, c.omega_r)
    ctx = st.Context(0, precision="fp64")
    p, v, m, h = dev(ps.pos), dev(ps.vel), dev(ps.mass), dev(ps.soft)
    acc = st.steps_forces(p, m, h, ctx=ctx)
    e0 = st.steps_energy(p, v, m, h, grid[0], cosmo, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(len(grid) - 1):
        st.steps_step(p, v, m, h, acc, grid[k], grid[k + 1] - grid[k], cosmo,
                      ctx=ctx)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    e1 = st.steps_energy(p, v, m, h, grid[-1], cosmo, ctx=ctx)
    ctx.close()
    ms = (m[None, :] * acc).cpu().numpy()
    pair_p = float(np.linalg.norm(ms.sum(axis=1)) / np.abs(ms).sum())
    steps = len(grid) - 1
    out = {"n": n, "steps": steps, "a_range": [float(grid[0]), float(grid[-1])],
           "seconds": elapsed, "ms_per_step": 1e3 * elapsed / steps,
           "pairs_per_s": float(n) * n * steps / elapsed,
           "start": {"a": float(grid[0]), "K": e0["K"], "W": e0["W"], "P": e0["P"]},
           "end": {"a": float(grid[-1]), "K": e1["K"], "W": e1["W"], "P": e1["P"]},
           "pair_momentum_rel_end": pair_p,
           "finite": bool(torch.isfinite(p).all()) and bool(torch.isfinite(v).all())}
    log("workload 2, 200 steps: %.2f s (%.3e pairs/s); K %.4e -> %.4e, "
        "W %.4e -> %.4e; |sum m S|/sum|m S| %.2e"
        % (elapsed, out["pairs_per_s"], e0["K"], e1["K"], e0["W"], e1["W"], pair_p))
    return out


def force_kernel_name(precision, tile):
    """Name of the force kernel a launch shape runs (as rocprofv3 lists it)."""
    if precision != "fp64":
        return "k_force_mixed_sym" if tile["variant"] & 8 else "k_force_mixed"
    if tile["variant"] & 8:
        return "k_force_f64_symq" if tile["variant"] & 16 else "k_force_f64_sym"
    return "k_force_f64_mfma" if tile["variant"] & 4 else "k_force_f64"


def profile_path(precision, tile, workload):
    """The committed rocprofv3 summary of this kernel, launch shape and
    workload (which may not exist)."""
    return os.path.join(ROOT, "profiles", "%s_r%d_tj%d_v%d_workload%d.md"
                        % (force_kernel_name(precision, tile), tile["r"],
                           tile["tj"], tile["variant"], workload))


def profiled_traffic(precision, tile, workload):
    """HBM bytes per force launch from the committed rocprofv3 summary of
    this kernel and launch shape, or None if there is none or the kernel
    source has changed since it was taken."""
    return profile_traffic(profile_path(precision, tile, workload))


def counter_roofline(path, frac):
    """Counter-based figures of a committed rocprofv3 summary (None if there
    is none or its kernel source has changed): the measured clock and the
    fraction `frac` of the nominal-clock peak restated at it, the executed
    flops per ordered pair and the counter-weighted fraction (executed flops
    instead of the 20-flop convention), VALU busy, and the FP64 pipe busy
    (FP64 kernels) or the VALU issue rate against single issue (FP32)."""
    import re
    if profile_traffic(path) is None:
        return None
    text = open(path).read()

    def num(pattern):
        m = re.search(pattern, text)
        return float(m.group(1)) if m else None

    out = {"source": "profiles/" + os.path.basename(path),
           "kernel_ms_profiled": num(r"average kernel ([0-9.]+) ms here"),
           "clock_ghz": num(r"clock GRBM_GUI_ACTIVE[^\n]*= ([0-9.]+) GHz"),
           "valu_busy": num(r"VALU busy SQ_ACTIVE_INST_VALU[^\n]*= ([0-9.]+)"),
           "executed_flop_per_pair": num(r"executed FP(?:64|32) flops per [^(\n]*"
                                         r"\([^)]*\): ([0-9.]+)")}
    busy = num(r"FP64 pipe busy ([0-9.]+)")
    if busy is not None:
        out["fp64_pipe_busy"] = busy
    issue = num(r"VALU issue \(rsq at 4 slots\) ([0-9.]+)x")
    if issue is not None:
        out["valu_issue_vs_single"] = issue
    if out["clock_ghz"]:
        out["frac_at_measured_clock"] = frac * NOMINAL_CLOCK_GHZ / out["clock_ghz"]
    if out["executed_flop_per_pair"]:
        out["counter_weighted_frac"] = frac * out["executed_flop_per_pair"] / FLOP_PER_PAIR
    out["note"] = ("clock, busy and executed-flop figures from the summary's "
                   "own run; fractions restate this run's frac with them "
                   "(peak at %.1f GHz nominal)" % NOMINAL_CLOCK_GHZ)
    return out


def profile_traffic(path):
    """traffic_bytes_per_launch of a committed rocprofv3 summary, or None if
    there is none or the kernel's source file (named with its SHA-256 in the
    summary) has changed since it was taken."""
    import hashlib
    if not os.path.exists(path):
        return None
    traffic, ok = None, False
    for line in open(path):
        if line.startswith("traffic_bytes_per_launch:"):
            traffic = float(line.split(":", 1)[1])
        if line.startswith("source_sha256:"):
            digest, name = line.split(":", 1)[1].split()[:2]
            src = os.path.join(ROOT, "paper_1811_05903_amd", "csrc", name.strip("()"))
            ok = (os.path.exists(src) and
                  hashlib.sha256(open(src, "rb").read()).hexdigest() == digest)
    return traffic if ok else None


def li_residual_run(st, dev, ps, nsteps, precision="fp64"):
    """One run of the workload-5 recipe over a log-uniform grid of nsteps
    from ps.a0 to ps.a1; returns |R| / |U_c(a1) - U_c(a0)| for the cosmic
    energy equation in the form d[a (K + W)]/da = -K (K every step, W at the
    two ends)."""
    import numpy as np
    c = ps.cosmo
    cosmo = st.Cosmology(c.H0, c.omega_m, c.omega_l, c.omega_r)
    grid = ps.a0 * (ps.a1 / ps.a0) ** (np.arange(nsteps + 1) / nsteps)
    grid[-1] = ps.a1
    ctx = st.Context(0, precision=precision)
    p, v, m, h = dev(ps.pos), dev(ps.vel), dev(ps.mass), dev(ps.soft)
    acc = st.steps_forces(p, m, h, ctx=ctx)
    e0 = st.steps_energy(p, v, m, h, grid[0], cosmo, ctx=ctx)
    kin, integral = e0["K"], 0.0
    for k in range(nsteps):
        st.steps_step(p, v, m, h, acc, grid[k], grid[k + 1] - grid[k], cosmo, ctx=ctx)
        kn = st.steps_kinetic(v, m, grid[k + 1], ctx=ctx)["K"]
        integral += 0.5 * (kin + kn) * (grid[k + 1] - grid[k])
        kin = kn
    e1 = st.steps_energy(p, v, m, h, grid[-1], cosmo, ctx=ctx)
    ctx.close()
    r = grid[-1] * (e1["K"] + e1["W"]) - grid[0] * (e0["K"] + e0["W"]) + integral
    du = grid[-1] * e1["W"] - grid[0] * e0["W"]
    return abs(r) / abs(du)


def li_adaptive_run(st, dev, ps, eps, dt_max=1e3, precision="fp64"):
    """As li_residual_run, with the step of Eq. 12 (steps_adaptive_dt)
    chosen before every step; returns (|R| / |dU_c|, steps taken)."""
    c = ps.cosmo
    cosmo = st.Cosmology(c.H0, c.omega_m, c.omega_l, c.omega_r)
    ctx = st.Context(0, precision=precision)
    p, v, m, h = dev(ps.pos), dev(ps.vel), dev(ps.mass), dev(ps.soft)
    acc = st.steps_forces(p, m, h, ctx=ctx)
    a, a1 = ps.a0, ps.a1
    e0 = st.steps_energy(p, v, m, h, a, cosmo, ctx=ctx)
    kin, integral, steps = e0["K"], 0.0, 0
    while a < a1:
        _, da = st.steps_adaptive_dt(p, v, h, acc, a, cosmo, eps, dt_max, ctx=ctx)
        an = a1 if a + da >= a1 else a + da
        st.steps_step(p, v, m, h, acc, a, an - a, cosmo, ctx=ctx)
        kn = st.steps_kinetic(v, m, an, ctx=ctx)["K"]
        integral += 0.5 * (kin + kn) * (an - a)
        kin, a, steps = kn, an, steps + 1
    e1 = st.steps_energy(p, v, m, h, a1, cosmo, ctx=ctx)
    ctx.close()
    r = a1 * (e1["K"] + e1["W"]) - ps.a0 * (e0["K"] + e0["W"]) + integral
    du = a1 * e1["W"] - ps.a0 * e0["W"]
    return abs(r) / abs(du), steps


def li_convergence(st, dev, n=131072, steps=(50, 100, 200, 400, 800),
                   eps=(3e-2, 1e-2, 3e-3)):
    """Layzer-Irvine residual of the workload-5 recipe at a smaller N
    against the number of steps: a second-order integrator shows the
    residual falling ~4x per doubling once the steps resolve the dynamics."""
    import synth
    ps = synth.config(5, n=n)
    out = []
    for ns in steps:
        t0 = time.perf_counter()
        rel = li_residual_run(st, dev, ps, ns)
        out.append({"steps": ns, "rel": rel})
        log("Layzer-Irvine study n=%d steps=%d |R|/|dU_c| %.3e (%.1f s)"
            % (n, ns, rel, time.perf_counter() - t0))
    adaptive = []
    for e in eps:
        t0 = time.perf_counter()
        rel, ns = li_adaptive_run(st, dev, ps, e)
        adaptive.append({"eps": e, "steps": ns, "rel": rel})
        log("Layzer-Irvine study n=%d adaptive eps=%g: %d steps, |R|/|dU_c| %.3e (%.1f s)"
            % (n, e, ns, rel, time.perf_counter() - t0))
    return {"n": n, "runs": out,
            "ratios": [out[k]["rel"] / out[k + 1]["rel"] for k in range(len(out) - 1)],
            "adaptive": adaptive}


def workload5(st, dev, args):
    """Workload 5: N = 2^22 (D = 500, r_max = 4000, LCDM 0.3089/0.6911/
    67.74, sigma 1%, Zel'dovich velocities), 50 log steps a 0.1 -> 1.0.
    The mixed-precision run is checked against the FP64 GPU run: force
    error at the start (all particles, plus an oracle spot check on sampled
    rows), Layzer-Irvine energy residual every 25 steps, final positions.
    --steps sets the step count here (default 50, the full run)."""
    import numpy as np
    import torch
    import synth
    study = None if args.no_li_study else li_convergence(st, dev)
    if args.li_study_only:
        return {"layzer_irvine_convergence": study}
    ps = synth.config(5)
    n, grid, c = ps.n, ps.a_grid(), ps.cosmo
    nsteps = min(args.steps if args.steps != 20 else 50, len(grid) - 1)
    cosmo = st.Cosmology(c.H0, c.omega_m, c.omega_l, c.omega_r)
    m, h = dev(ps.mass), dev(ps.soft)
    every = 25   # full energy (an O(N^2) FP64 potential) every this many steps
    log("workload 5: n=%d, %d steps a %.2f -> %.2f" % (n, nsteps, grid[0], grid[nsteps]))
    res = {}
    acc0 = {}
    for prec in ("mixed", "fp64"):
        ctx = st.Context(0, precision=prec, flags=st.STEPS_PROFILE)
        p, v = dev(ps.pos), dev(ps.vel)
        acc = st.steps_forces(p, m, h, ctx=ctx)
        acc0[prec] = acc.cpu().numpy()
        full = {0: st.steps_energy(p, v, m, h, grid[0], cosmo, ctx=ctx)}
        kin = [full[0]["K"]]
        ctx.force_timing(reset=True)
        t_steps = 0.0
        for k in range(nsteps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st.steps_step(p, v, m, h, acc, grid[k], grid[k + 1] - grid[k], cosmo, ctx=ctx)
            torch.cuda.synchronize()
            t_steps += time.perf_counter() - t0
            kin.append(st.steps_kinetic(v, m, grid[k + 1], ctx=ctx)["K"])
            if (k + 1) % every == 0 or k + 1 == nsteps:
                full[k + 1] = st.steps_energy(p, v, m, h, grid[k + 1], cosmo, ctx=ctx)
            log("%s step %d/%d a=%.4f (%.2f s/step)" % (prec, k + 1, nsteps, grid[k + 1], t_steps / (k + 1)))
        kms, cnt = ctx.force_timing(reset=True)
        # cosmic energy equation in the scale factor, d[a (K + W)]/da = -K:
        # R = a (K + W) - a0 (K0 + W0) + int K da, the integral by the
        # trapezoid rule over every step (K is O(N) per step; W, which needs
        # the O(N^2) potential, only at the sampled steps).  Relative to the
        # change of U_c = a W since the start.
        cum = [0.0]
        for k in range(nsteps):
            cum.append(cum[-1] + 0.5 * (kin[k] + kin[k + 1]) * (grid[k + 1] - grid[k]))
        e0 = grid[0] * (full[0]["K"] + full[0]["W"])
        li = []
        for k in sorted(full):
            if k == 0:
                continue
            r = grid[k] * (full[k]["K"] + full[k]["W"]) - e0 + cum[k]
            du = grid[k] * full[k]["W"] - grid[0] * full[0]["W"]
            li.append({"a": grid[k], "residual": r, "delta_U_c": du,
                       "int_K_da": cum[k], "rel": abs(r) / abs(du)})
        pairs = float(n) * n
        res[prec] = {"steps": nsteps, "step_s": t_steps / nsteps,
                     "pairs_per_s": pairs * nsteps / t_steps,
                     "force_kernel_ms": kms / cnt,
                     "force_pairs_per_s": pairs / (kms / cnt * 1e-3),
                     "tflops_20": FLOP_PER_PAIR * pairs / (kms / cnt * 1e-3) / 1e12,
                     "frac_peak": FLOP_PER_PAIR * pairs / (kms / cnt * 1e-3) / 1e12
                     / (FP64_PEAK_TF if prec == "fp64" else FP32_PEAK_TF),
                     "layzer_irvine": li,
                     "energies": {str(k): {"a": grid[k], "K": e["K"], "W": e["W"]}
                                  for k, e in sorted(full.items())},
                     "tile": ctx.get_tile(n)}
        res[prec + "_final_pos"] = p.cpu().numpy()
        ctx.close()
    dpos = np.linalg.norm(res.pop("mixed_final_pos") - res.pop("fp64_final_pos"), axis=0) / ps.soft
    ferr = np.linalg.norm(acc0["mixed"] - acc0["fp64"], axis=0) / np.linalg.norm(acc0["fp64"], axis=0)
    out = {"metric": "pair interactions/s (ordered pairs, whole KDK step)",
           "value": res["mixed"]["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1,
           "steps": nsteps, "warmup": 0, "ms_per_step": 1e3 * res["mixed"]["step_s"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32-pair/f64-acc", "data": "synthetic",
           "config": {"workload": "stereographic sphere N=%d D=500 r_max=4000 LCDM, "
                                  "mixed forces, FP64 kick/drift, a 0.1 -> 1.0" % n,
                      "n": n, "parallelism": "single GPU"},
           "mixed": res["mixed"], "fp64": res["fp64"],
           "layzer_irvine_convergence": study,
           "mixed_vs_fp64_force_rel_err_start": {"median": float(np.median(ferr)),
                                                  "max": float(ferr.max())},
           "mixed_vs_fp64_final_dx_over_h": {"median": float(np.median(dpos)),
                                              "p99": float(np.quantile(dpos, 0.99))}}
    if not args.no_cpu_baseline:
        import oracle
        idx = np.sort(np.random.default_rng(5).choice(n, 4096, replace=False))
        t0 = time.perf_counter()
        ref = oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx)
        tcpu = time.perf_counter() - t0
        for prec in ("mixed", "fp64"):
            e = np.linalg.norm(acc0[prec][:, idx] - ref, axis=0) / np.linalg.norm(ref, axis=0)
            out[prec]["oracle_rel_err"] = {"rows": 4096, "median": float(np.median(e)),
                                           "max": float(e.max())}
        out["cpu_baseline"] = {"value": 4096.0 * n / tcpu, "unit": "pairs/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": "FP64 oracle pair sums for 4096 seeded-sampled "
                                         "i against all %d j (%.1f s)" % (n, tcpu)}
    log("workload 5: mixed %.3e pairs/s, fp64 %.3e; Layzer-Irvine |R|/|dU_c| "
        "at a=1: mixed %.2e fp64 %.2e"
        % (res["mixed"]["pairs_per_s"], res["fp64"]["pairs_per_s"],
           res["mixed"]["layzer_irvine"][-1]["rel"], res["fp64"]["layzer_irvine"][-1]["rel"]))
    return out


def glass_leg(st, dev, n=262144, radius=500.0):
    """Glass relaxation (Sec. 3): an equal-mass Poisson ball of N = 2^18 at
    the mean density, 150 log steps a 0.01 -> 1 with reversed gravity, FP64;
    the nearest-neighbour distance spread (std/mean, inner 80% of the
    radius) before and after."""
    import numpy as np
    import torch
    import synth
    from scipy.spatial import cKDTree
    ps = synth.poisson_ball(n, radius, synth.Cosmo(67.74, 0.3089, 0.6911), seed=31)

    def cv(pos):
        d, _ = cKDTree(pos.T).query(pos.T, k=2)
        keep = np.linalg.norm(pos, axis=0) < 0.8 * radius
        return float(d[keep, 1].std() / d[keep, 1].mean())

    c = ps.cosmo
    cosmo = st.Cosmology(c.H0, c.omega_m, c.omega_l, c.omega_r, reversed_gravity=True)
    grid = ps.a_grid()
    p, v, m, h = dev(ps.pos), dev(ps.vel), dev(ps.mass), dev(ps.soft)
    ctx = st.Context(0, precision="fp64")
    acc = st.steps_forces(p, m, h, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(len(grid) - 1):
        st.steps_step(p, v, m, h, acc, grid[k], grid[k + 1] - grid[k], cosmo, ctx=ctx)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.close()
    out = {"n": n, "steps": len(grid) - 1, "seconds": elapsed,
           "pairs_per_s": float(n) * n * (len(grid) - 1) / elapsed,
           "nn_cv_start": cv(ps.pos), "nn_cv_glass": cv(p.cpu().numpy())}
    log("glass: N=%d, %d steps in %.1f s (%.3e pairs/s); nearest-neighbour "
        "spread %.3f -> %.3f" % (n, out["steps"], elapsed, out["pairs_per_s"],
                                  out["nn_cv_start"], out["nn_cv_glass"]))
    return out


def periodic_leg(st, dev):
    """Periodic box (Eqs. 2 and 5): pair-sum evaluations per image rule on
    uniform particles in a box of side 100 Mpc, FP64, kernel time by HIP
    events (mean of two launches after an untimed one).  The full rule sums every image within
    2.6 L: for uniform particles the expected number of image terms per
    pair is the volume of that sphere in units of L^3, 4/3 pi 2.6^3 = 73.6,
    which prices its roofline (20 flop per image term); the nearest-image
    rule has one term per pair."""
    import math
    import numpy as np
    import torch
    out = {}
    for images, n in ((1, 262144), (2, 65536)):
        rng = np.random.default_rng(40 + images)
        L = 100.0
        p = dev(rng.uniform(0, L, (3, n)))
        m, h = dev(rng.uniform(0.5, 2.0, n)), dev(np.full(n, 0.02 * L / n ** (1 / 3)))
        ctx = st.Context(0, precision="fp64", flags=st.STEPS_PROFILE)
        ctx.set_periodic(L, images)
        acc = st.steps_forces(p, m, h, ctx=ctx)
        torch.cuda.synchronize()
        ctx.force_timing(reset=True)
        for _ in range(2):
            st.steps_forces(p, m, h, acc=acc, ctx=ctx)
        ms, cnt = ctx.force_timing(reset=True)
        ctx.close()
        name = "nearest" if images == 1 else "all_images_2.6L"
        kern_ms = ms / cnt
        terms = 1.0 if images == 1 else 4.0 / 3.0 * math.pi * 2.6 ** 3
        achieved = FLOP_PER_PAIR * terms * float(n) * n / (kern_ms * 1e-3) / 1e12
        kernel = "k_force_periodic<%d>" % images
        prof = os.path.join(ROOT, "profiles", "k_force_periodic_images%d_uniform_box_n%d.md"
                            % (images, n))
        out[name] = {
            "n": n, "kernel_ms": kern_ms, "launches": cnt,
            "pairs_per_s": float(n) * n / (kern_ms * 1e-3),
            "image_terms_per_pair": terms,
            "roofline": {
                "bound": "alu", "pipe": "fp64", "achieved": achieved,
                "peak": FP64_PEAK_TF, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TF,
                "traffic": profile_traffic(prof),
                "counters": counter_roofline(prof, achieved / FP64_PEAK_TF),
                "kernel": kernel,
                "flop_per_pair": FLOP_PER_PAIR,
                "pair_convention": "N^2 ordered pairs per evaluation, times "
                                   "the expected image terms per pair"}}
        log("periodic %s: n=%d, %.2f ms, %.3e pairs/s, %.3f of peak"
            % (name, n, kern_ms, out[name]["pairs_per_s"], achieved / FP64_PEAK_TF))
    return out


def batch_leg(st, dev, nsteps, members=64, n_scale=1.0, sequential=True):
    """Workload 4: 64 members, N_b ~ U{8192..131072}, Omega_m ~ U[0.25,
    0.35] flat, 100 log steps a 0.02 -> 1.0, mixed precision: one
    steps_batch_run (persistent kernel, graph-replayed step, autotuned)
    against the same members run one after another with steps_step.
    members / n_scale give the many-small-runs variant (n_scale shrinks
    every member's N)."""
    import numpy as np
    import torch
    import synth
    members = synth.ensemble(members=members, n_scale=n_scale, nsteps=nsteps)
    offs = np.cumsum([0] + [m.n for m in members])
    cat = lambda key, axis: np.ascontiguousarray(
        np.concatenate([getattr(m, key) for m in members], axis=axis))
    cos = [st.Cosmology(m.cosmo.H0, m.cosmo.omega_m, m.cosmo.omega_l)
           for m in members]
    a0 = [m.a0 for m in members]
    a1 = [m.a1 for m in members]
    pairs = float(sum(m.n * m.n for m in members)) * nsteps
    ctx = st.Context(0, precision="mixed")
    flags = st.STEPS_BATCH_GRAPH | st.STEPS_BATCH_AUTOTUNE
    mass, soft = dev(cat("mass", 0)), dev(cat("soft", 0))
    # warm-up run (allocations, code objects), 2 steps
    p, v = dev(cat("pos", 1)), dev(cat("vel", 1))
    acc = torch.zeros_like(p)
    st.steps_batch_run(p, v, mass, soft, acc, offs, cos, a0, a1, 2,
                       flags=flags, ctx=ctx)
    p, v = dev(cat("pos", 1)), dev(cat("vel", 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status = st.steps_batch_run(p, v, mass, soft, acc, offs, cos, a0, a1,
                                nsteps, flags=flags, ctx=ctx)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    tile = st.steps_batch_tile(ctx)
    log("ensemble: %d members, N=%d, %d steps batched in %.2f s (%.3e pairs/s), tile %s"
        % (len(members), offs[-1], nsteps, t_batch, pairs / t_batch, tile))
    if not sequential:
        ctx.close()
        return {"members": len(members), "n_total": int(offs[-1]),
                "steps": nsteps, "pairs_per_step": pairs / nsteps,
                "batched_s": t_batch, "batched_pairs_per_s": pairs / t_batch,
                "tile": tile}
    # sequential: each member alone through steps_step
    per = [(dev(m.pos), dev(m.vel), dev(m.mass), dev(m.soft)) for m in members]
    grids = [m.a_grid() for m in members]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (pp, vv, mm, hh), g, c in zip(per, grids, cos):
        aa = st.steps_forces(pp, mm, hh, ctx=ctx)
        for k in range(nsteps):
            st.steps_step(pp, vv, mm, hh, aa, g[k], g[k + 1] - g[k], c, ctx=ctx)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    log("ensemble: sequential steps_step runs %.2f s (%.3e pairs/s); batched %.2fx"
        % (t_seq, pairs / t_seq, t_seq / t_batch))
    ctx.close()
    return {"members": len(members), "n_total": int(offs[-1]),
            "steps": nsteps, "pairs_per_step": pairs / nsteps,
            "precision": "mixed_f64acc", "status_ok": status.count(0),
            "batched_s": t_batch, "batched_pairs_per_s": pairs / t_batch,
            "sequential_s": t_seq, "sequential_pairs_per_s": pairs / t_seq,
            "speedup": t_seq / t_batch, "tile": tile,
            "note": "batched time includes the in-library sort and the "
                    "initial force evaluation; the kernel is the one the "
                    "warm-up run's autotune chose (kept in the context)"}


def binned_errors(err, kappa, radius, nbins=3):
    """Median and max relative error in equal-count bins of the oracle's
    condition number kappa (sum of |pair terms| over |S|) and of the
    distance from the centre."""
    import numpy as np
    out = {}
    for name, key in (("kappa", kappa), ("radius", radius)):
        order = np.argsort(key)
        bins = []
        for part in np.array_split(order, min(nbins, max(1, order.size))):
            if part.size == 0:
                continue
            bins.append({"lo": float(key[part[0]]), "hi": float(key[part[-1]]),
                         "median": float(np.median(err[part])),
                         "max": float(err[part].max()), "rows": int(part.size)})
        out[name] = bins
    return out


def _mode_entry(st, ps, rows, dev, reps, prec, tile=None, workload=None):
    """One row of the modes table: mean kernel time of `reps` launches after
    one warm-up in precision prec (optionally a forced launch shape), the
    error against the oracle rows if given, and (FP64 and mixed, with the
    workload named) the counter figures of the kernel's committed profile."""
    import numpy as np
    import torch
    n = ps.n
    pos, mass, soft = dev(ps.pos), dev(ps.mass), dev(ps.soft)
    ctx = st.Context(0, precision=prec, flags=st.STEPS_PROFILE)
    if tile is not None:
        ctx.set_tile(*tile)
    acc = st.steps_forces(pos, mass, soft, ctx=ctx)
    torch.cuda.synchronize()
    ctx.force_timing(reset=True)
    for _ in range(reps):
        st.steps_forces(pos, mass, soft, acc=acc, ctx=ctx)
    ms, cnt = ctx.force_timing(reset=True)
    kms = ms / cnt
    rate = float(n) * n / (kms * 1e-3)
    peak = FP64_PEAK_TF if prec == "fp64" else FP32_PEAK_TF
    entry = {"kernel_ms": kms, "launches": cnt, "pairs_per_s": rate,
             "pairs_distinct_per_s": float(n) * (n - 1) / (kms * 1e-3),
             "tflops_20": FLOP_PER_PAIR * rate / 1e12,
             "frac_peak": FLOP_PER_PAIR * rate / 1e12 / peak,
             "tile": ctx.get_tile(n)}
    if workload is not None and prec in ("fp64", "mixed"):
        entry["counters"] = counter_roofline(
            profile_path(prec, entry["tile"], workload), entry["frac_peak"])
    if rows is not None:
        idx, ref, kap = rows
        got = acc.cpu().numpy()[:, idx]
        err = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
        entry["rel_err_median"] = float(np.median(err))
        entry["rel_err_max"] = float(err.max())
        entry["rel_err_rows"] = int(idx.size)
        entry["rel_err_binned"] = binned_errors(err, kap, np.linalg.norm(ps.pos[:, idx], axis=0))
    ctx.close()
    return entry


def mode_table(st, ps, rows, dev, reps=3, refine=True, workload=None):
    """Force-kernel rate per precision mode at this N (mean of `reps` timed
    launches after one warm-up), and the error against the oracle rows if
    given; with refine, also the default mixed shape with one Newton step on
    the FP32 r^-3."""
    n = ps.n
    res = {}
    for prec in ("fp64", "mixed", "kahan"):
        entry = _mode_entry(st, ps, rows, dev, reps, prec, workload=workload)
        res[prec] = entry
        log("n=%d %s: %.2f ms, %.3e pairs/s%s" % (
            n, prec, entry["kernel_ms"], entry["pairs_per_s"],
            "" if rows is None else ", err median %.2e max %.2e" % (
                entry["rel_err_median"], entry["rel_err_max"])))
    res["mixed_speedup_vs_fp64"] = res["mixed"]["pairs_per_s"] / res["fp64"]["pairs_per_s"]
    if refine:
        # the one-sided FP64 kernel on the vector ALU alone (variant 3, no
        # matrix cores) beside the default
        res["fp64_valu"] = _mode_entry(st, ps, rows, dev, reps, "fp64",
                                       (4, 128, 0, 3), workload=workload)
        log("n=%d fp64 vector-ALU kernel: %.2f ms, %.3e pairs/s, %.3f of peak"
            % (n, res["fp64_valu"]["kernel_ms"], res["fp64_valu"]["pairs_per_s"],
               res["fp64_valu"]["frac_peak"]))
        # the default mixed shape with one Newton step on the FP32 r^-3
        # (variant 26 beside the default's variant 10)
        t = res["mixed"]["tile"]
        if t["variant"] == 10:
            res["mixed_newton"] = _mode_entry(st, ps, rows, dev, reps, "mixed",
                                              (t["r"], t["tj"], t["jsplit"], 26))
            log("n=%d mixed with Newton step: %.2f ms, %.3e pairs/s%s" % (
                n, res["mixed_newton"]["kernel_ms"], res["mixed_newton"]["pairs_per_s"],
                "" if rows is None else ", err median %.2e max %.2e" % (
                    res["mixed_newton"]["rel_err_median"],
                    res["mixed_newton"]["rel_err_max"])))
    return res


if __name__ == "__main__":
    main()
