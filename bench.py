"""Benchmark of the MRSDC time stepper on one MI355X.

Headline workload (default): the batched ensemble of 64 seeded scenarios on
the 7.5 mm machine (stand 54x54x214 + stock 41x41x54 nodes, 714,798 DOF per
scenario, 45,747,072 DOF in all), Gauss-Lobatto M=5, K=4 sweeps, P=5
embedded nodes per interval, dt = 5 s, FP32 inner CG with FP64 iterative
refinement, seeded synthetic inputs.  A "step" is one MRSDC macro-step
(predictor + K sweeps) of every scenario.

Prints ONE JSON line: DOF*steps/s (value), look-ahead factor eta = simulated /
wall time per scenario, p50/p99 macro-step latency, the dominant kernel's
roofline, the CPU oracle timed on a bounded sample of the same workload, and
the other workloads (single machine in FP64 and FP32, irregular meshes,
stationary field, work-precision study, deformation, residual control,
serving replay) as extra keys.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of a timed kernel, from two counter runs (FETCH_SIZE,
# then WRITE_SIZE, KiB per dispatch), each scaled by what the same counter
# read for a 256 MiB device-to-device copy (FETCH_SIZE 131089.0 KiB ->
# x1.99975, WRITE_SIZE 262144.0 KiB -> x1.0).  Each entry holds only for the
# kernel source it was taken on (sha256 of that file).
COUNTER_TRAFFIC = {
    ("machine-310k", 0): {
        "source": "kernels.hip",
        "sha256": "5810bc227099a51e600e65a6166459b275b9e45fe0b3997d8e1d1a8e4f8a7e4e",
        "fetch_kib": 2725.9, "fetch_scale": 1.99974,
        "write_kib": 2454.2, "write_scale": 1.0,
    },
    ("ensemble-64x714798", 1): {
        "source": "batch_kernels.hip",
        "sha256": "397a8c615408062e7cfe64dca8db10423a7aa7863503d8953b3a0c832394f19c",
        "fetch_kib": 162534.8, "fetch_scale": 1.99973,
        "write_kib": 181818.2, "write_scale": 1.0,
    },
    ("ensemble-64x714798", 0): {
        "source": "batch_kernels.hip",
        "sha256": "397a8c615408062e7cfe64dca8db10423a7aa7863503d8953b3a0c832394f19c",
        "fetch_kib": 395314.0, "fetch_scale": 1.99974,
        "write_kib": 361189.8, "write_scale": 1.0,
    },
}


def counter_traffic(workload, precision):
    """Scaled counter bytes per launch, or None if there is no counter run for
    this workload or the kernel source changed since it was taken."""
    import hashlib
    c = COUNTER_TRAFFIC.get((workload, precision))
    if c is None:
        return None
    src = os.path.join(ROOT, "paper_1707_03581_amd", "csrc", c["source"])
    try:
        with open(src, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if digest != c["sha256"]:
        return None
    return (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed macro-steps of the headline")
    ap.add_argument("--warmup", type=int, default=3, help="untimed macro-steps before them")
    ap.add_argument("--config", default="ensemble",
                    choices=["ensemble", "box", "machine", "machine-fp32", "serve"],
                    help="ensemble: the 64-member ensemble headline with every extra key; "
                         "box / machine / machine-fp32: one simulation only; serve: only the "
                         "serving replay")
    ap.add_argument("--headline-only", action="store_true", help="skip the extra keys")
    ap.add_argument("--precision", type=int, default=None,
                    help="0 FP64, 1 FP32+refine (headline form; default FP32+refine for the "
                         "ensemble, the workload's own for the others)")
    ap.add_argument("--serve-requests", type=int, default=16, help="requests replayed (serve)")
    ap.add_argument("--serve-precision", type=int, default=1, choices=[0, 1],
                    help="form of the served simulations: 0 FP64, 1 FP32+refine")
    ap.add_argument("--serve-max-steps", type=int, default=12,
                    help="cap on each request's macro-steps in the bounded replay (serve)")
    ap.add_argument("--serve-budget-gib", type=float, default=0.0,
                    help="HBM budget of the serving replay (0: 90%% of the free device memory)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="finish with a device-to-device copy of this many MiB (counter scale)")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle sample in macro-steps (0: every step the GPU ran)")
    ap.add_argument("--cpu-1thread-steps", type=int, default=2,
                    help="macro-steps of the single-thread oracle figure (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="event timing of kernel classes inside the timed region (adds overhead)")
    ap.add_argument("--op-reps", type=int, default=200, help="operator timing launches")
    ap.add_argument("--machine-steps", type=int, default=40,
                    help="timed macro-steps of the single 310,042-DOF machine (0: skip)")
    ap.add_argument("--deform-reps", type=int, default=5,
                    help="thermo-elastic deformation: timed solves on the 1 cm stand (0: skip)")
    ap.add_argument("--wp-levels", type=int, default=5,
                    help="work-precision study: time-step levels per method (0: skip)")
    ap.add_argument("--ensemble-fp64-steps", type=int, default=6,
                    help="macro-steps of the FP64 ensemble extra key (0: skip)")
    ap.add_argument("--precision-steps", type=int, default=24,
                    help="macro-steps of the FP32+refinement machine (0: skip)")
    return ap.parse_args()


def workload(name, nsteps):
    import mrsdc_inputs as mi
    if name == "box":
        return mi.box_patch_2673()
    if name == "machine-fp32":
        return mi.machine_310k_fp32(nsteps=nsteps)
    return mi.machine_310k(nsteps=nsteps)


METRIC = "look-ahead eta & DOF*steps/s at 1e-7 rel err; p50/p99 macro-step latency"


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the time step of "
              "one simulation is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1707_03581_amd as pkg

    assert torch.cuda.is_available(), "no GPU"
    if args.config == "serve":
        print(json.dumps(serving(pkg, args)), flush=True)
        if args.calibrate_copy:
            calibrate_copy(args.calibrate_copy)
        return
    if args.config != "ensemble":
        out = single(pkg, args, args.config, args.steps, args.warmup, args.precision)
        out.update({"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                    "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                    "data": "synthetic"})
        print(json.dumps(out), flush=True)
        if args.calibrate_copy:
            calibrate_copy(args.calibrate_copy)
        return
    import mrsdc_inputs as mi
    prec = mi.FP32_REFINE if args.precision is None else args.precision
    ens = ensemble(pkg, args, prec, args.steps, args.warmup, headline=True)
    out = {
        "metric": METRIC,
        "value": ens.pop("value"),
        "unit": "DOF*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ens.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ens.pop("dtype"),
        "data": "synthetic",
        "config": ens.pop("config"),
    }
    out.update(ens)
    if not args.headline_only:
        extras(pkg, args, out)
    print(json.dumps(out), flush=True)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)


def extras(pkg, args, out):
    """The other workloads, each as its own key."""
    import mrsdc_inputs as mi
    if args.ensemble_fp64_steps > 0:
        out["ensemble_fp64"] = ensemble(pkg, args, mi.FP64, args.ensemble_fp64_steps, 1)
    if args.machine_steps > 0:
        out["machine_fp64"] = single(pkg, args, "machine", args.machine_steps, 4, None)
    if args.precision_steps > 0:
        out["machine_fp32_refine"] = precision_form(pkg, args)
    out["irregular_machine"] = irregular_form(pkg, args)
    out["graph_capture"] = graph_form(pkg, args)
    out["autotune"] = autotune_form(pkg, args)
    out["stationary"] = stationary_form(pkg, args)
    if args.wp_levels > 0:
        out["work_precision"] = work_precision_form(pkg, args)
    if args.deform_reps > 0:
        out["deformation"] = deformation_form(pkg, args)
    if args.machine_steps > 0:
        out["residual_control"] = residual_control_form(pkg, args,
                                                        out["machine_fp64"]["ms_per_step"] / 1e3)
    if args.serve_requests > 0:
        out["serving"] = serving(pkg, args)


def oracle_baseline(pb, nsteps, gpu_T, label, args, T0=None, **over):
    """The oracle on the host cores over the same steps as the GPU state
    gpu_T: error of that state, DOF*steps/s on every host thread and on one
    thread (a shorter sample), and the split of its time between the CG
    solves and the literal full-vector embedded substeps."""
    import oracle
    oracle.set_threads(os.cpu_count() or 1)
    t = time.perf_counter()
    ref, ost = oracle.run(pb, nsteps=nsteps, T0=T0, **over)
    tc = time.perf_counter() - t
    out = {"value": pb.N * nsteps / tc, "unit": "DOF*steps/s", "cores": int(ost["threads"]),
           "kind": "oracle", "sample": f"{label}, {nsteps} macro-steps", "seconds": tc,
           "pcg_share": ost["t_pcg"] / max(ost["t_total"], 1e-12),
           "embedded_share": ost["t_embedded"] / max(ost["t_total"], 1e-12),
           "note": "literal CPU oracle, not tuned: GPU/CPU ratios overstate the gap to a "
                   "tuned CPU code"}
    n1 = min(args.cpu_1thread_steps, nsteps)
    if n1 > 0:
        oracle.set_threads(1)
        t = time.perf_counter()
        _, o1 = oracle.run(pb, nsteps=n1, T0=T0, **over)
        t1 = time.perf_counter() - t
        oracle.set_threads(os.cpu_count() or 1)
        out["one_thread"] = {"value": pb.N * n1 / t1, "cores": int(o1["threads"]),
                             "sample": f"{label}, {n1} macro-steps", "seconds": t1,
                             "pcg_share": o1["t_pcg"] / max(o1["t_total"], 1e-12)}
    err = float(np.linalg.norm(gpu_T - ref) / np.linalg.norm(ref))
    return out, err


def single(pkg, args, config, steps, warmup, precision):
    """One simulation (no batching): per-step latency, throughput, the CG
    operator's effective bandwidth, and the oracle over every step run."""
    import torch
    pb = workload(config, steps)
    dt = pb.scheme.dt
    N = pb.N
    print(f"[bench] workload {pb.name}: N={N} nnz={pb.nnz}", file=sys.stderr, flush=True)
    if precision is not None:
        pb.scheme.precision = precision
    ctx = pkg.simulation(pb, device=0)
    t_setup = time.perf_counter()
    ctx.advance(warmup * dt)
    t_setup = time.perf_counter() - t_setup
    print(f"[bench] warmup {warmup} steps done ({t_setup:.2f}s incl. setup)", file=sys.stderr,
          flush=True)
    # timed region: one advance call per macro-step (each returns after the
    # device finished the step) -> per-step latency and total wall time
    if args.profile:
        ctx.profile(True)
    torch.cuda.synchronize()
    lat = []
    iters = 0
    redone = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        st = ctx.advance(dt)
        lat.append(time.perf_counter() - s0)
        iters += st["pcg_iters"]
        redone += st["redone_steps"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = ctx.profile_read() if args.profile else None
    print(f"[bench] {pb.name}: timed {steps} steps in {wall:.3f}s", file=sys.stderr, flush=True)
    lat_ms = np.array(lat) * 1e3
    out = {
        "value": N * steps / wall, "unit": "DOF*steps/s", "ms_per_step": wall / steps * 1e3,
        "dtype": "f64" if pb.scheme.precision == 0 else "f32+f64-refine",
        "config": {"workload": pb.name, "dof": N, "nnz": pb.nnz, "M": pb.scheme.M,
                   "nodes": "gauss-lobatto" if pb.scheme.family == 0 else "equidistant",
                   "K": pb.scheme.K, "P": pb.scheme.P, "dt_s": dt, "simulated_s": steps * dt},
        "eta": steps * dt / wall,
        "p50_step_ms": float(np.percentile(lat_ms, 50)),
        "p99_step_ms": float(np.percentile(lat_ms, 99)),
        "cg_iters_per_step": iters / steps,
        "redone_steps": redone,
        "op_form": st["op_form"],
    }
    # the CG operator application, timed with HIP events over back-to-back
    # launches on the library's stream (its own kernel symbol, k_pcg_a<..., 2,
    # ...>, in rocprof summaries).  Its working set fits the 256 MB Infinity
    # Cache, so the figure is an effective (cache-resident) bandwidth.
    us, nbytes = ctx.time_operator(args.op_reps)
    achieved = nbytes / (us * 1e-6) / 1e9
    out["roofline"] = {"bound": "hbm", "kernel": "k_pcg_a (CG operator application)",
                       "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS,
                       "traffic": counter_traffic(pb.name, pb.scheme.precision),
                       "avg_launch_us": us, "launches": args.op_reps, "bytes_per_launch": nbytes,
                       "note": "cache-resident working set: an effective-bandwidth fraction, "
                               "bytes of the form the product reads (op_form)"}
    if kt and kt["iface_launches"]:
        out["iface_avg_us"] = kt["iface_ms"] / kt["iface_launches"] * 1e3
    T = pkg.get_state(ctx, pb)
    ctx.destroy()
    if not args.no_cpu_baseline:
        S = warmup + steps if args.cpu_steps <= 0 else min(args.cpu_steps, warmup + steps)
        ref_pb = workload(config, S)
        if precision is not None:
            ref_pb.scheme.precision = precision
        if S == warmup + steps:
            cb, err = oracle_baseline(ref_pb, S, T, f"{pb.name} (every step run)", args)
        else:
            g = pkg.simulation(ref_pb, device=0)
            g.advance(S * dt)
            Tg = pkg.get_state(g, ref_pb)
            g.destroy()
            cb, err = oracle_baseline(ref_pb, S, Tg, f"first {S} macro-steps of {pb.name}", args)
        out["cpu_baseline"] = cb
        out["rel_l2_vs_oracle"] = err
        out["rel_l2_steps"] = S
    return out


def calibrate_copy(mib):
    """A plain copy of known size: reads and writes mib MiB once each."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"[bench] calibration copy of {mib} MiB done", file=sys.stderr, flush=True)


def residual_control_form(pkg, args, fixed_step_s):
    """The machine with residual-controlled sweeps: the tolerance sits between
    the residuals of iterates 1 and 2 of the first step; eta and sweeps per
    step beside the fixed-K run, and (CPU leg) the error against the oracle
    run with the same rule."""
    import dataclasses
    import mrsdc_inputs as mi
    steps = args.machine_steps
    pb = mi.machine_310k(nsteps=steps)
    probe = pkg.simulation(pb, device=0, final_residual=1)
    r = probe.advance(pb.scheme.dt)["residual"]
    probe.destroy()
    tol = float(np.sqrt(r[1] * r[2]))
    sc = dataclasses.replace(pb.scheme, sweep_tol=tol)
    ctx = pkg.simulation(dataclasses.replace(pb, scheme=sc), device=0)
    ctx.advance(4 * pb.scheme.dt)
    t = time.perf_counter()
    st = ctx.advance(steps * pb.scheme.dt)
    wall = time.perf_counter() - t
    ctx.destroy()
    out = {"sweep_tol": tol, "sweeps_per_step": st["sweeps"] / steps,
           "ms_per_step": wall / steps * 1e3, "eta": pb.scheme.dt * steps / wall,
           "speedup_vs_fixed_K": fixed_step_s / (wall / steps)}
    if not args.no_cpu_baseline:
        import oracle
        S = 4
        g = pkg.simulation(dataclasses.replace(pb, scheme=sc), device=0)
        g.advance(S * pb.scheme.dt)
        Tg = pkg.get_state(g, pb)
        g.destroy()
        Tref, ost = oracle.run(pb, nsteps=S, scheme=sc)
        out["rel_l2_vs_oracle"] = float(np.linalg.norm(Tg - Tref) / np.linalg.norm(Tref))
        out["oracle_sweeps_per_step"] = ost["sweeps"] / S
    return out


def work_precision_form(pkg, args):
    """Time-discretisation error against look-ahead factor for the three
    method classes of the work-precision study (§5): MRSDC (Lobatto M=3, P=2,
    K=0,1,2), single-rate SDC (M=3, coupling implicit, K=0,1,2) and implicit
    Euler, on the benchmark machine from its stationary field (uniform T_env)
    with the study's motion law s(t) = 0.495 sin(2 pi t / 24 s) + 0.505 m over
    10 periods (240 s), at 6, 12, ... steps per period (the study's Delta t =
    2 s is 12).  The error is the max-norm difference at the end time to a
    reference run of MRSDC with Lobatto M=5, P=8, K=7 at a quarter of the
    finest level's dt (its own error estimated against the same run at twice
    that dt); eta = simulated time / wall time of the advance; the observed
    order of each curve is the slope of log error against log dt over its
    two finest levels."""
    import dataclasses
    import mrsdc_inputs as mi
    base = mi.machine_310k(nsteps=1)
    base.motion = mi.Motion(s0=0.505, a=0.495, period=24.0, phase=0.0)
    base.T0 = np.full(base.N, 20.0)
    t_end = 10.0 * base.motion.period
    n0 = 6  # steps per period at the coarsest level
    levels = [n0 * 2**i for i in range(args.wp_levels)]

    def run(sc):
        pb = dataclasses.replace(base, scheme=sc)
        ctx = pkg.simulation(pb, device=0)
        ctx.advance(0.0)  # device state built outside the timed advance
        st = ctx.advance(t_end)
        T = pkg.get_state(ctx, pb)
        ctx.destroy()
        return T, st

    dt_ref = base.motion.period / (4 * levels[-1])
    t = time.perf_counter()
    Tref, _ = run(mi.Scheme(M=5, family=mi.LOBATTO, P=8, K=7, dt=dt_ref))
    print(f"[bench] work-precision reference ({t_end / dt_ref:.0f} steps) "
          f"{time.perf_counter() - t:.1f}s", file=sys.stderr, flush=True)
    rise = float(np.abs(Tref - 20.0).max())
    T2, _ = run(mi.Scheme(M=5, family=mi.LOBATTO, P=8, K=7, dt=2 * dt_ref))
    ref_err = float(np.abs(T2 - Tref).max())
    methods = [(f"MRSDC(3,2) k={k}", dict(M=3, family=mi.LOBATTO, P=2, K=k)) for k in (0, 1, 2)]
    methods += [(f"SDC(3) k={k}", dict(M=3, family=mi.LOBATTO, P=1, K=k, method=mi.SINGLE_RATE))
                for k in (0, 1, 2)]
    methods += [("implicit Euler", dict(M=1, family=mi.EQUI_NOLEFT, P=1, K=0,
                                        method=mi.SINGLE_RATE))]
    curves = []
    for name, kw in methods:
        pts = []
        for n in levels:
            dt = base.motion.period / n
            T, st = run(mi.Scheme(dt=dt, **kw))
            err = float(np.abs(T - Tref).max())
            pts.append({"dt_s": dt, "steps_per_period": n, "steps": st["steps"],
                        "eta": t_end / st["wall_s"], "max_err_K": err, "rel_err": err / rise,
                        "cg_iters": st["pcg_iters"]})
        order = None
        if len(pts) >= 2 and pts[-1]["max_err_K"] > 0 and pts[-2]["max_err_K"] > 0:
            order = float(np.log(pts[-2]["max_err_K"] / pts[-1]["max_err_K"]) /
                          np.log(pts[-2]["dt_s"] / pts[-1]["dt_s"]))
        curves.append({"method": name, "observed_order": order, "points": pts})
        print(f"[bench] work-precision {name}: " +
              " ".join(f"(eta {p['eta']:.0f}, err {p['rel_err']:.1e})" for p in pts) +
              f" order {order}", file=sys.stderr, flush=True)
    return {"workload": base.name + ", motion 0.495 sin(2 pi t / 24 s) + 0.505 m",
            "t_end_s": t_end, "initial": "stationary (uniform T_env)",
            "reference": {"method": "MRSDC Lobatto M=5 P=8 K=7", "dt_s": dt_ref,
                          "max_diff_K_vs_twice_dt": ref_err},
            "max_temperature_rise_K": rise, "curves": curves}


def deformation_form(pkg, args):
    """Thermo-elastic deformation of the benchmark machine's stand (41 x 41 x
    161 nodes, floor clamped, 806,880 displacement DOFs) from its temperature
    after 4 steps: the one-off factorisation, the forward/backward solve per
    output, and the solve's dominant step (the symmetric block product and its
    partial sums) timed per product with HIP events against the HBM peak.  The residual
    ||K_u u - f|| / ||f|| is checked on the host."""
    from mrsdc_inputs.elastic import elastic_box
    import mrsdc_inputs as mi
    pb = mi.machine_310k(nsteps=4)
    el = elastic_box(pb.bodies[0])
    ctx = pkg.simulation(pb, device=0)
    t = time.perf_counter()
    st = ctx.advance(4 * pb.scheme.dt)
    step_ms = (time.perf_counter() - t) / 4 * 1e3
    info = ctx.deform_setup(el)
    solve_us, gemv_us, gemv_bytes = ctx.deform_time(args.deform_reps)
    u = ctx.deform()
    T = ctx.get_temperature(0, pb.bodies[0].n)
    ctx.destroy()
    f = el.gcsr() @ (T - el.T_ref)
    res = float(np.linalg.norm(el.csr() @ u - f) / np.linalg.norm(f))
    gbps = gemv_bytes / (gemv_us * 1e-6) / 1e9
    print(f"[bench] deformation: factor {info['factor_ms']:.0f} ms, solve {solve_us / 1e3:.2f} ms, "
          f"block product {gemv_us:.1f} us = {gbps:.0f} GB/s", file=sys.stderr, flush=True)
    return {"workload": "stand 41x41x161 nodes, clamped floor", "dof": el.n, "nnz": el.nnz,
            "block": info["block"], "padded_block": info["padded_block"],
            "blocks": info["nblocks"], "factor_ms": info["factor_ms"],
            "factor_launches": info["factor_launches"],
            "factor_GiB": info["factor_bytes"] / 2**30, "solve_ms": solve_us / 1e3,
            "solve_per_macro_step": solve_us / 1e3 / step_ms,
            "max_displacement_um": float(np.abs(u).max() * 1e6),
            "relative_residual": res,
            "roofline": {"bound": "hbm",
                         "kernel": "k_symv + k_symv_reduce (symmetric block product, upper-triangle tiles)",
                         "achieved": gbps, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbps / HBM_PEAK_GBS, "avg_launch_us": gemv_us,
                         "bytes_per_launch": gemv_bytes, "traffic": None}}


def stationary_form(pkg, args):
    """The stationary initial field (K + h R) T = g on the benchmark machine:
    one Jacobi-PCG solve on the device, timed; its closed form is T_env."""
    import mrsdc_inputs as mi
    pb = mi.machine_310k(nsteps=1)
    ctx = pkg.simulation(pb, device=0)
    ctx.advance(0.0)  # build the device state outside the timed region
    t = time.perf_counter()
    it = ctx.set_stationary(rtol=1e-12, maxit=200000)
    wall = time.perf_counter() - t
    T = pkg.get_state(ctx, pb)
    ctx.destroy()
    return {"workload": pb.name, "cg_iters": it, "ms": wall * 1e3,
            "max_abs_err_vs_closed_form": float(np.abs(T - 20.0).max())}


def precision_form(pkg, args):
    """Same machine, FP32 inner CG + FP64 refinement: throughput beside the
    FP64 form, and its error against the FP64 oracle over every step run."""
    import torch
    warm = 4
    pb = workload("machine-fp32", args.precision_steps)
    dt = pb.scheme.dt
    ctx = pkg.simulation(pb, device=0)
    ctx.advance(warm * dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.advance(args.precision_steps * dt)
    wall = time.perf_counter() - t0
    us, nbytes = ctx.time_operator(args.op_reps)
    T = pkg.get_state(ctx, pb)
    ctx.destroy()
    print(f"[bench] fp32+refine {args.precision_steps} steps in {wall:.3f}s", file=sys.stderr,
          flush=True)
    out = {"workload": pb.name, "value": pb.N * args.precision_steps / wall,
           "unit": "DOF*steps/s", "ms_per_step": wall / args.precision_steps * 1e3,
           "eta": args.precision_steps * dt / wall,
           "op_avg_us": us, "op_GBps": nbytes / (us * 1e-6) / 1e9,
           "note": "FP32 inner CG dot products summed in FP64"}
    if not args.no_cpu_baseline:
        import oracle
        n = warm + args.precision_steps
        ref, _ = oracle.run(workload("machine", n), nsteps=n)
        out["rel_l2_vs_fp64_oracle"] = float(np.linalg.norm(T - ref) / np.linalg.norm(ref))
        out["rel_l2_steps"] = n
    return out


def serving(pkg, args):
    """Bounded replay of the seeded request trace (Poisson arrivals at 20/s,
    mesh levels 2 cm / 1 cm / 5 mm, per-request parameters): pools sized by
    the levels' footprints within the HBM budget, continuous batching per
    level; each request's steps capped to keep the run short.  The oracle
    reruns one served request of the finest level that was served."""
    import mrsdc_inputs as mi
    from paper_1707_03581_amd.serve import Request, Server, summarize
    trace = mi.serving_trace(args.serve_requests)
    levels = {}
    for name, (stand, stock) in mi.MESH_LEVELS.items():
        levels[name] = mi.machine(stand_nodes=stand, stock_nodes=stock, nsteps=1,
                                  name=f"machine_{name}")
        levels[name].scheme.precision = args.serve_precision
        print(f"[bench] level {name}: N={levels[name].N}", file=sys.stderr, flush=True)
    reqs = []
    for r in trace:
        rng = np.random.default_rng(r["seed"] + 1)
        reqs.append(Request(id=r["id"], arrival=r["arrival"], level=r["level"],
                            nsteps=min(r["nsteps"], args.serve_max_steps), h=r["h"],
                            alpha=r["alpha"], friction_W=r["friction_W"], period=r["period"],
                            T0=20.0 + rng.uniform(-0.5, 0.5, size=levels[r["level"]].N)))
    budget = int(args.serve_budget_gib * 2**30) if args.serve_budget_gib > 0 else None
    srv = Server(levels, slots_per_level=64, hbm_budget_bytes=budget)
    plan = srv.size_pools()
    print(f"[bench] serving pools {plan} within {srv.budget / 2**30:.1f} GiB", file=sys.stderr,
          flush=True)
    done = srv.run(reqs)
    out = summarize(done, 5.0, {k: v.N for k, v in levels.items()})
    out["dtype"] = "f64" if args.serve_precision == 0 else "f32+f64-refine"
    served = [r for r in done if not r.rejected]
    out["eta_per_request"] = {str(r.id): r.nsteps * 5.0 / (r.finished - r.arrival)
                              for r in served}
    if not args.no_cpu_baseline and served:
        import oracle
        big = max({r.level for r in served}, key=lambda k: levels[k].N)
        r = min((q for q in served if q.level == big), key=lambda q: q.nsteps)
        t = time.perf_counter()
        ref, ost = oracle.run(levels[big], nsteps=r.nsteps, T0=r.T0, h=r.h, alpha=r.alpha,
                              friction_W=r.friction_W, period=r.period)
        tc = time.perf_counter() - t
        out["rel_l2_vs_oracle_sample"] = {
            "request": r.id, "level": big, "steps": r.nsteps, "oracle_s": tc,
            "oracle_cores": int(ost["threads"]),
            "value": float(np.linalg.norm(r.result - ref) / np.linalg.norm(ref))}
    out.update({"metric": "serving: p50/p99 macro-step latency, per-request eta, DOF*steps/s",
                "workload": f"first {len(reqs)} requests of the 20 req/s trace, <= "
                            f"{args.serve_max_steps} steps each",
                "levels": {k: v.N for k, v in levels.items()},
                "hbm_budget_GiB": srv.budget / 2**30, "pool_slots": plan,
                "level_bytes": {k: {"shared": v[0], "per_slot": v[1]}
                                for k, v in srv.level_bytes.items()},
                "footprint_bytes": srv.footprint})
    print(f"[bench] serving done in {srv.wall:.2f}s", file=sys.stderr, flush=True)
    return out


def ensemble(pkg, args, precision, steps, warmup, headline=False):
    """64 seeded scenarios on the 7.5 mm machine (714,798 DOF each), one batch:
    per-step latency and throughput, the multi-RHS operator kb_pcg_a_col against
    the HBM roofline, and (headline) the oracle on member 0 over every step."""
    import torch
    import mrsdc_inputs as mi
    S = 64
    pb = mi.ensemble_member(0, nsteps=steps, precision=precision)
    members = []
    for s in range(S):
        h, alpha, pf, period, rng = mi.scenario_params(s)
        members.append(dict(h=h, alpha=alpha, friction_W=pf, period=period,
                            T0=20.0 + rng.uniform(-0.5, 0.5, size=pb.N)))
    dt = pb.scheme.dt
    form = "FP64" if precision == mi.FP64 else "FP32 inner CG + FP64 refinement"
    print(f"[bench] ensemble {S} x {pb.N} DOF, {form}", file=sys.stderr, flush=True)
    t = time.perf_counter()
    ctx = pkg.batch_simulation(pb, members, device=0)
    ctx.advance_steps(warmup)
    torch.cuda.synchronize()
    print(f"[bench] ensemble setup + {warmup} warmup steps {time.perf_counter() - t:.1f}s",
          file=sys.stderr, flush=True)
    lat = []
    iters = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        st = ctx.advance_steps(1)
        lat.append(time.perf_counter() - s0)
        iters += st["pcg_iters"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"[bench] ensemble {steps} steps in {wall:.3f}s", file=sys.stderr, flush=True)
    reps = max(20, args.op_reps // 10)
    us, nbytes = ctx.time_operator(reps)
    footprint = ctx.footprint_bytes()
    T_member0 = ctx.get_scenario_temperature(0, pb.N)
    ctx.destroy()
    lat_ms = np.array(lat) * 1e3
    b = 4 if precision == mi.FP32_REFINE else 8
    # the operator of box bodies runs as the column sweep in both forms
    op_kernel = "kb_pcg_a_col (column-sweep multi-RHS CG operator, 64 scenarios)"
    # algorithmic bytes of one multi-RHS operator launch as the shared operator
    # arrives (CSR): every stored entry once (value + int32 column), the row
    # pointers, and the S right-hand sides read once and written once
    csr_bytes = pb.nnz * (b + 4) + 4 * pb.N + 2 * b * S * pb.N
    achieved = csr_bytes / (us * 1e-6) / 1e9
    out = {
        "value": S * pb.N * steps / wall, "unit": "DOF*steps/s",
        "ms_per_step": wall / steps * 1e3,
        "dtype": "f64" if precision == mi.FP64 else "f32+f64-refine",
        "config": {"workload": f"ensemble-64x{pb.N}-7.5mm", "scenarios": S, "dof": pb.N,
                   "dof_total": S * pb.N, "nnz_shared": pb.nnz, "M": pb.scheme.M,
                   "nodes": "gauss-lobatto", "K": pb.scheme.K, "P": pb.scheme.P, "dt_s": dt,
                   "simulated_s_per_scenario": steps * dt, "form": form},
        "eta_per_scenario": steps * dt / wall,
        "p50_step_ms": float(np.percentile(lat_ms, 50)),
        "p99_step_ms": float(np.percentile(lat_ms, 99)),
        "cg_iters_per_step": iters / steps / S,
        "footprint_GiB": footprint / 2**30,
        "roofline": {"bound": "hbm", "kernel": op_kernel,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": counter_traffic(f"ensemble-64x{pb.N}", precision),
                     "avg_launch_us": us, "launches": reps, "bytes_per_launch": csr_bytes,
                     "bytes_formula": "nnz*(b+4) + 4N + 2*b*S*N (CSR operator, S right-hand "
                                      "sides in and out), b = value bytes",
                     "bytes_kernel_design": nbytes},
    }
    if precision == mi.FP32_REFINE:
        out["note"] = ("FP32 values, vectors and products in the inner CG; its dot products "
                       "are summed in FP64; residual, refinement and node states in FP64")
    if not args.no_cpu_baseline:
        mb = members[0]
        nst = warmup + steps
        cb, err = oracle_baseline(pb, nst, T_member0, "member 0 alone (every step run)", args,
                                  T0=mb["T0"], h=mb["h"], alpha=mb["alpha"],
                                  friction_W=mb["friction_W"], period=mb["period"])
        out["cpu_baseline"] = cb
        out["rel_l2_vs_oracle_member0"] = err
        out["rel_l2_steps"] = nst
        out["meets_1e-7"] = bool(err <= 1e-7)
    return out


def graph_form(pkg, args):
    """Per-step time with the step launched directly and captured once into a
    HIP graph (use_graph), back to back on the same GPU: the 310,042-DOF
    machine (FP64) and the 64-member ensemble (FP32 + refinement)."""
    import torch
    import mrsdc_inputs as mi
    out = {}
    pb = mi.machine_310k(nsteps=1)
    res = {}
    for graph in (0, 1):
        ctx = pkg.simulation(pb, device=0, use_graph=graph)
        ctx.advance(4 * pb.scheme.dt)  # three direct steps learn the budgets, the fourth is captured
        torch.cuda.synchronize()
        n = 40
        t = time.perf_counter()
        for _ in range(n):
            st = ctx.advance(pb.scheme.dt)
        res[graph] = (time.perf_counter() - t) / n * 1e3
        if graph:
            res["launches"] = st["graph_launches"]
        ctx.destroy()
    out["machine_fp64"] = {"ms_per_step_direct": res[0], "ms_per_step_graph": res[1],
                           "speedup": res[0] / res[1]}
    pe = mi.ensemble_member(0, nsteps=1, precision=mi.FP32_REFINE)
    members = []
    for s in range(64):
        h, alpha, pf, period, rng = mi.scenario_params(s)
        members.append(dict(h=h, alpha=alpha, friction_W=pf, period=period,
                            T0=20.0 + rng.uniform(-0.5, 0.5, size=pe.N)))
    for graph in (0, 1):
        ctx = pkg.batch_simulation(pe, members, device=0, use_graph=graph)
        ctx.advance_steps(4)  # three direct steps learn the budgets, the fourth is captured
        torch.cuda.synchronize()
        n = 6
        t = time.perf_counter()
        ctx.advance_steps(n)
        res[graph] = (time.perf_counter() - t) / n * 1e3
        ctx.destroy()
    out["ensemble_fp32_refine"] = {"ms_per_step_direct": res[0], "ms_per_step_graph": res[1],
                                   "speedup": res[0] / res[1]}
    print(f"[bench] graph capture: {out}", file=sys.stderr, flush=True)
    return out


def autotune_form(pkg, args):
    """The 64-member ensemble (FP32 + refinement) with the launch variants of
    its CG kernels chosen by timing (autotune) and with the default ones:
    per-step time, the chosen variant and the operator time of each."""
    import torch
    import mrsdc_inputs as mi
    pe = mi.ensemble_member(0, nsteps=1, precision=mi.FP32_REFINE)
    members = []
    for s in range(64):
        h, alpha, pf, period, rng = mi.scenario_params(s)
        members.append(dict(h=h, alpha=alpha, friction_W=pf, period=period,
                            T0=20.0 + rng.uniform(-0.5, 0.5, size=pe.N)))
    out = {}
    for tune in (0, 1):
        ctx = pkg.batch_simulation(pe, members, device=0, autotune=tune)
        st = ctx.advance_steps(2)
        torch.cuda.synchronize()
        n = 6
        t = time.perf_counter()
        ctx.advance_steps(n)
        ms = (time.perf_counter() - t) / n * 1e3
        us, _ = ctx.time_operator(20)
        ctx.destroy()
        out["tuned" if tune else "default"] = {
            "ms_per_step": ms, "op_avg_us": us, "col_depth": st["col_depth"],
            "groups_b": st["groups_b"], "groups_c": st["groups_c"]}
    out["speedup"] = out["default"]["ms_per_step"] / out["tuned"]["ms_per_step"]
    print(f"[bench] autotune: {out}", file=sys.stderr, flush=True)
    return out


def irregular_form(pkg, args):
    """The 310,042-DOF machine on irregular tensor meshes (no value
    dictionary applies): the CG product reads the plain value array (10 B per
    entry); renumbered, with int32 columns (12 B per entry).  Steps timed, the
    operator's effective bandwidth, and the error against the oracle."""
    import torch
    import mrsdc_inputs as mi
    out = {}
    for renumber in (False, True):
        steps = 8
        pb = mi.machine_310k_irregular(nsteps=steps, renumber=renumber)
        ctx = pkg.simulation(pb, device=0)
        ctx.advance(2 * pb.scheme.dt)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = ctx.advance(steps * pb.scheme.dt)
        wall = time.perf_counter() - t
        us, nbytes = ctx.time_operator(args.op_reps)
        T = pkg.get_state(ctx, pb)
        ctx.destroy()
        gbps = nbytes / (us * 1e-6) / 1e9
        key = "renumbered" if renumber else "ordered"
        r = {"workload": pb.name, "op_form": {1: "values", 2: "dict", 3: "packed",
                                              4: "patterns"}.get(st["op_form"]),
             "col_bytes": st["col_bytes"], "ms_per_step": wall / steps * 1e3,
             "value": pb.N * steps / wall, "unit": "DOF*steps/s",
             "op_avg_us": us, "op_bytes": nbytes, "op_GBps": gbps,
             "op_frac_hbm": gbps / HBM_PEAK_GBS,
             "note": "87.9 MB (ordered) working set: cache-resident, effective bandwidth"}
        if not args.no_cpu_baseline:
            import oracle
            ref, _ = oracle.run(pb, nsteps=steps + 2)
            r["rel_l2_vs_oracle"] = float(np.linalg.norm(T - ref) / np.linalg.norm(ref))
        out[key] = r
        print(f"[bench] irregular {key}: {r['ms_per_step']:.2f} ms/step, operator {us:.1f} us",
              file=sys.stderr, flush=True)
    return out


if __name__ == "__main__":
    main()
