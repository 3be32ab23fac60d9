"""Benchmark of the StePS direct-summation hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 2]
                    [--no-cpu-baseline] [--no-modes]

A step is one comoving KDK step (kick + drift, one O(N^2) pair sum, kick) of
the whole particle set, with state resident in HBM.  Default workload:
N = 2^18 stereographically projected particles, D = 200 Mpc,
r_max = 2000 Mpc, LCDM (0.3089 / 0.6911 / 67.74), FP64, stepping along its
200-step log-uniform grid from a = 0.02.  The value is ordered pair
interactions per second over the timed steps (N^2 per step).

Also reported on the same JSON line:
  roofline     -- force kernel: 20 flop per ordered pair (convention) over
                  its average launch time (HIP events on its own stream),
                  against the FP64 peak 78.6 TFLOP/s ("bound": "mfma" for the
                  matrix-core kernels, which share that pipe, else "alu");
  cpu_baseline -- the CPU FP64 oracle on a bounded seeded sample of i rows
                  against all N j (rank 0 only);
  modes        -- force-kernel pair rate in FP64 and both mixed modes at the
                  same N and at N = 2^21, with the relative force error
                  against the oracle sample (median, max).

--workload 3 runs the three precision modes at N = 2^21 against the oracle
on 65 536 sampled rows (about a minute of host time); --workload 5 runs
N = 2^22 for 50 steps in mixed precision and in FP64 with the energy checks.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=2, choices=[1, 2, 3, 5])
    ap.add_argument("--no-glass", action="store_true",
                    help="skip the glass-relaxation leg")
    ap.add_argument("--li-study-only", action="store_true",
                    help="workload 5: only the Layzer-Irvine step-convergence "
                         "study at N = 2^17")
    ap.add_argument("--precision", default="fp64",
                    choices=["fp64", "mixed", "kahan"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-modes", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-member ensemble comparison")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample")
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
    if args.workload == 3:
        print(json.dumps(workload3(st, dev, args)), flush=True)
        return

    ps = synth.config(args.workload)
    n = ps.n
    log("workload %d: n=%d precision=%s" % (args.workload, n, args.precision))
    grid = ps.a_grid()
    c = ps.cosmo
    cosmo = st.Cosmology(c.H0, c.omega_m, c.omega_l, c.omega_r)
    stream = torch.cuda.current_stream()
    ctx = st.Context(0, precision=args.precision, flags=st.STEPS_PROFILE,
                     stream=stream)
    if args.tile:
        ctx.set_tile(*(int(x) for x in args.tile.split(",")))
    pos, vel, mass, soft = dev(ps.pos), dev(ps.vel), dev(ps.mass), dev(ps.soft)
    acc = st.steps_forces(pos, mass, soft, ctx=ctx)

    total = args.warmup + args.steps
    if total > len(grid) - 1:
        raise SystemExit("at most %d steps on this grid" % (len(grid) - 1))
    k = 0
    for _ in range(args.warmup):
        st.steps_step(pos, vel, mass, soft, acc, grid[k], grid[k + 1] - grid[k],
                      cosmo, ctx=ctx)
        k += 1
    torch.cuda.synchronize()
    ctx.force_timing(reset=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st.steps_step(pos, vel, mass, soft, acc, grid[k], grid[k + 1] - grid[k],
                      cosmo, ctx=ctx)
        k += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    force_ms, force_cnt = ctx.force_timing(reset=True)
    elapsed = t1 - t0
    ms_step = 1e3 * elapsed / args.steps
    pairs = float(n) * n
    value = pairs * args.steps / elapsed
    kern_ms = force_ms / max(1, force_cnt)
    achieved = FLOP_PER_PAIR * pairs / (kern_ms * 1e-3) / 1e12
    peak = FP64_PEAK_TF if args.precision == "fp64" else FP32_PEAK_TF
    tile = ctx.get_tile(n)
    log("%d steps: %.2f ms/step, %.3e pairs/s; force kernel %.2f ms (%d launches)"
        % (args.steps, ms_step, value, kern_ms, force_cnt))
    assert bool(torch.isfinite(pos).all()) and bool(torch.isfinite(acc).all())

    traffic = profiled_traffic(args.precision, tile, args.workload)
    out = {
        "metric": "pair interactions/s (ordered pairs, whole KDK step)",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-pair/f64-acc",
        "data": "synthetic",
        "config": {"workload": "stereographic sphere N=%d D=%g r_max=%g, %s, "
                               "KDK from a=%.3f" % (n, ps.params["D"],
                                                    ps.params["r_max"],
                                                    args.precision, grid[0]),
                   "n": n, "precision": args.precision, "tile": tile,
                   "parallelism": "single GPU"},
        # the FP64 matrix-core kernel and the vector kernels are both priced
        # at the FP64 peak: on gfx950 dense FP64 MFMA and FP64 VALU share one
        # 78.6 TFLOP/s pipe
        "roofline": {"bound": "mfma" if tile["variant"] & 4
                     and args.precision == "fp64" else "alu",
                     "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": traffic,
                     "kernel": force_kernel_name(args.precision, tile),
                     "kernel_ms": kern_ms,
                     "flop_per_pair": FLOP_PER_PAIR},
    }

    sample_rows = big_rows = None
    big = None if args.no_modes else synth.config(3)
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(12345)
        oracle.forces(ps.pos, ps.mass, ps.soft, idx=rng.choice(n, 16, replace=False))
        probe = rng.choice(n, 512, replace=False)
        t = time.perf_counter()
        oracle.forces(ps.pos, ps.mass, ps.soft, idx=probe)
        rate = 512 * n / (time.perf_counter() - t)
        m = int(min(n, max(64, rate * args.cpu_seconds / n)))
        idx = np.sort(rng.choice(n, m, replace=False))
        log("cpu baseline: oracle on %d sampled rows (%d threads)" % (m, oracle.num_threads()))
        # the same positions the GPU starts from (before stepping)
        t = time.perf_counter()
        ref, kap = oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx, want_kappa=True)
        dt = time.perf_counter() - t
        sample_rows = (idx, ref, kap)
        out["cpu_baseline"] = {
            "value": m * float(n) / dt, "unit": "pairs/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "FP64 oracle pair sums for %d seeded-sampled i of the "
                      "N=%d set against all j (%.1f s)" % (m, n, dt)}
        if not args.no_modes:
            # the oracle's rows of the 2^21 set, the reference of its modes
            # table (not part of the timed sample above)
            bidx = np.sort(np.random.default_rng(3).choice(big.n, 32, replace=False))
            big_rows = (bidx,) + oracle.forces(big.pos, big.mass, big.soft, idx=bidx,
                                               want_kappa=True)

    if not args.no_modes:
        out["modes"] = mode_table(st, ps, sample_rows, dev)
        out["modes_n2e21"] = mode_table(st, big, big_rows, dev)
    if not args.no_batch:
        out["batch"] = batch_leg(st, dev, args.batch_steps)
        # many small members (N_b ~ 256 ... 4096): where one launch per
        # member and step would leave the GPU idle
        out["batch_small"] = batch_leg(st, dev, args.batch_steps, members=256,
                                       n_scale=1.0 / 32)
    if not args.no_glass:
        out["glass"] = glass_leg(st, dev)
        out["periodic"] = periodic_leg(st, dev)
    ctx.close()
    if args.copy_calibration:
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d MiB read + %d MiB written" % (
            args.copy_calibration, args.copy_calibration))
    print(json.dumps(out), flush=True)


def force_kernel_name(precision, tile):
    """Name of the force kernel a launch shape runs (as rocprofv3 lists it)."""
    if precision != "fp64":
        return "k_force_mixed_sym" if tile["variant"] & 8 else "k_force_mixed"
    if tile["variant"] & 8:
        return "k_force_f64_sym"
    return "k_force_f64_mfma" if tile["variant"] & 4 else "k_force_f64"


def profiled_traffic(precision, tile, workload):
    """HBM bytes per force launch from the committed rocprofv3 summary of
    this kernel and launch shape, or None if there is none or the kernel
    source has changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_r%d_tj%d_v%d_workload%d.md"
                        % (force_kernel_name(precision, tile), tile["r"],
                           tile["tj"], tile["variant"], workload))
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
    study = li_convergence(st, dev)
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
    """Periodic box (Eqs. 2 and 5): one pair-sum evaluation per image rule
    on uniform particles in a box of side 100 Mpc, FP64, kernel time by HIP
    events.  The full rule sums every image within 2.6 L (about 74 image
    terms per pair, 179 image tests)."""
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
        st.steps_forces(p, m, h, acc=acc, ctx=ctx)
        ms, cnt = ctx.force_timing(reset=True)
        ctx.close()
        name = "nearest" if images == 1 else "all_images_2.6L"
        out[name] = {"n": n, "kernel_ms": ms / cnt, "pairs_per_s": float(n) * n / (ms / cnt * 1e-3)}
        log("periodic %s: n=%d, %.2f ms, %.3e pairs/s" % (name, n, ms / cnt, out[name]["pairs_per_s"]))
    return out


def batch_leg(st, dev, nsteps, members=64, n_scale=1.0):
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
            "note": "batched time includes the in-library sort, autotune "
                    "and initial force evaluation"}


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


def workload3(st, dev, args, rows=65536):
    """Workload 3: N = 2^21, one force evaluation per precision mode (FP64,
    FP32 pairs with FP64 accumulation, FP32 pairs with Kahan accumulation),
    each against the FP64 oracle on `rows` seeded-sampled i (all j), with
    pair-interactions/s and the mixed-to-FP64 ratio."""
    import numpy as np
    import oracle
    import synth
    ps = synth.config(3)
    n = ps.n
    log("workload 3: n=%d, oracle on %d sampled rows (%d threads)"
        % (n, rows, oracle.num_threads()))
    idx = np.sort(np.random.default_rng(33).choice(n, rows, replace=False))
    refs, kaps = [], []
    t0 = time.perf_counter()
    step = 8192
    for k in range(0, rows, step):
        r, kp = oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx[k:k + step],
                              want_kappa=True)
        refs.append(r)
        kaps.append(kp)
        log("oracle rows %d/%d (%.0f s)" % (min(rows, k + step), rows,
                                            time.perf_counter() - t0))
    odt = time.perf_counter() - t0
    sample = (idx, np.concatenate(refs, axis=1), np.concatenate(kaps))
    modes = mode_table(st, ps, sample, dev)
    return {
        "metric": "pair interactions/s (ordered pairs, one force evaluation)",
        "value": modes["fp64"]["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic",
        "config": {"workload": "stereographic sphere N=%d D=%g r_max=%g, "
                               "three precision modes" % (n, ps.params["D"],
                                                          ps.params["r_max"]),
                   "n": n, "parallelism": "single GPU"},
        "modes": modes,
        "cpu_baseline": {"value": float(rows) * n / odt, "unit": "pairs/s",
                         "cores": oracle.num_threads(), "kind": "oracle",
                         "sample": "FP64 oracle pair sums for %d seeded-sampled "
                                   "i against all %d j (%.1f s)" % (rows, n, odt)},
    }


def mode_table(st, ps, rows, dev):
    """Force-kernel rate per precision mode at this N, one timed launch after
    one warm-up, and the error against the oracle rows if given."""
    import numpy as np
    import torch
    n = ps.n
    pos, mass, soft = dev(ps.pos), dev(ps.mass), dev(ps.soft)
    res = {}
    for prec in ("fp64", "mixed", "kahan"):
        ctx = st.Context(0, precision=prec, flags=st.STEPS_PROFILE)
        acc = st.steps_forces(pos, mass, soft, ctx=ctx)
        torch.cuda.synchronize()
        ctx.force_timing(reset=True)
        reps = 3 if n <= 300000 else 1
        for _ in range(reps):
            st.steps_forces(pos, mass, soft, acc=acc, ctx=ctx)
        ms, cnt = ctx.force_timing(reset=True)
        kms = ms / cnt
        rate = float(n) * n / (kms * 1e-3)
        peak = FP64_PEAK_TF if prec == "fp64" else FP32_PEAK_TF
        entry = {"kernel_ms": kms, "pairs_per_s": rate,
                 "tflops_20": FLOP_PER_PAIR * rate / 1e12,
                 "frac_peak": FLOP_PER_PAIR * rate / 1e12 / peak,
                 "tile": ctx.get_tile(n)}
        if rows is not None:
            idx, ref, kap = rows
            got = acc.cpu().numpy()[:, idx]
            err = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
            entry["rel_err_median"] = float(np.median(err))
            entry["rel_err_max"] = float(err.max())
            entry["rel_err_rows"] = int(idx.size)
            entry["rel_err_binned"] = binned_errors(err, kap, np.linalg.norm(ps.pos[:, idx], axis=0))
        res[prec] = entry
        log("n=%d %s: %.2f ms, %.3e pairs/s%s" % (
            n, prec, kms, rate,
            "" if rows is None else ", err median %.2e max %.2e" % (
                entry["rel_err_median"], entry["rel_err_max"])))
        ctx.close()
    res["mixed_speedup_vs_fp64"] = res["mixed"]["pairs_per_s"] / res["fp64"]["pairs_per_s"]
    return res


if __name__ == "__main__":
    main()
