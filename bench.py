"""Benchmark of the MRSDC time stepper on one MI355X.

Workload (default): the two-body machine, stand 41x41x161 + stock 31x31x41
nodes (310,042 DOF, 8,044,322 nonzeros), Gauss-Lobatto M=5, K=4 sweeps, P=5
embedded nodes per interval, dt = 5 s, FP64, seeded synthetic inputs.  A
"step" is one MRSDC macro-step (predictor + K sweeps) of the whole state.

Prints ONE JSON line: DOF*steps/s (value), look-ahead factor eta = simulated /
wall time, p50/p99 macro-step latency, the dominant kernel's roofline and the
CPU oracle timed on a bounded sample of the same workload.
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

# HBM bytes per launch of the timed CG operator kernel on the FP64 machine
# workload, from two counter runs (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch), each scaled by what the same counter read for a 256 MiB
# device-to-device copy (FETCH_SIZE 131088.8 KiB -> x1.99974, WRITE_SIZE
# 262144.0 KiB -> x1.0).  Valid only for the kernel source it was taken on.
COUNTER_TRAFFIC = {
    "kernels_sha256": "990925d289973e22a39614bf0b65626a1f78d032ce857fb9d6dc862edd980adb",
    "workload": "machine-310k", "precision": 0,
    "fetch_kib": 2725.9, "fetch_scale": 1.99974,
    "write_kib": 2454.2, "write_scale": 1.0,
}


def counter_traffic(pb):
    """Scaled counter bytes per launch, or None if the kernel source changed."""
    import hashlib
    src = os.path.join(ROOT, "paper_1707_03581_amd", "csrc", "kernels.hip")
    try:
        with open(src, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    c = COUNTER_TRAFFIC
    if digest != c["kernels_sha256"] or pb.name != c["workload"] or pb.scheme.precision != c["precision"]:
        return None
    return (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=120)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--config", default="machine", choices=["box", "machine", "machine-fp32", "ensemble", "serve"],
                    help="ensemble: only the 64-member ensemble; serve: only the serving replay")
    ap.add_argument("--serve-requests", type=int, default=24, help="requests replayed (serve)")
    ap.add_argument("--serve-precision", type=int, default=1, choices=[0, 1],
                    help="form of the served simulations: 0 FP64, 1 FP32+refine")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="finish with a device-to-device copy of this many MiB (counter scale)")
    ap.add_argument("--serve-max-steps", type=int, default=12,
                    help="cap on each request's macro-steps in the bounded replay (serve)")
    ap.add_argument("--precision", type=int, default=None, help="0 FP64, 1 FP32+refine")
    ap.add_argument("--cpu-steps", type=int, default=4, help="oracle sample (macro-steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="event timing of kernel classes inside the timed region (adds overhead)")
    ap.add_argument("--op-reps", type=int, default=200, help="operator timing launches")
    ap.add_argument("--deform-reps", type=int, default=5,
                    help="thermo-elastic deformation: timed solves on the 1 cm stand (0: skip)")
    ap.add_argument("--wp-levels", type=int, default=5,
                    help="work-precision study: time-step levels per method (0: skip)")
    ap.add_argument("--ensemble-precision", type=int, default=1, choices=[0, 1],
                    help="form of the stand-alone ensemble run: 0 FP64, 1 FP32+refine")
    ap.add_argument("--ensemble-steps", type=int, default=6,
                    help="macro-steps of the 64-member 7.5 mm ensemble (0: skip)")
    ap.add_argument("--precision-steps", type=int, default=24,
                    help="macro-steps of the FP32+refinement form (0: skip)")
    return ap.parse_args()


def workload(name, nsteps):
    import mrsdc_inputs as mi
    if name == "box":
        return mi.box_patch_2673()
    if name == "machine-fp32":
        return mi.machine_310k_fp32(nsteps=nsteps)
    return mi.machine_310k(nsteps=nsteps)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the time step of "
              "one simulation is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1707_03581_amd as pkg

    assert torch.cuda.is_available(), "no GPU"
    if args.config == "ensemble":
        print(json.dumps(ensemble(pkg, args, args.ensemble_precision)), flush=True)
        return
    if args.config == "serve":
        print(json.dumps(serving(pkg, args)), flush=True)
        return
    pb = workload(args.config, args.steps)
    dt = pb.scheme.dt
    N = pb.N
    print(f"[bench] workload {pb.name}: N={N} nnz={pb.nnz}", file=sys.stderr, flush=True)
    over = {} if args.precision is None else {"precision": args.precision}
    ctx = pkg.simulation(pb, device=0, **over)
    t_setup = time.perf_counter()
    ctx.advance(args.warmup * dt)
    t_setup = time.perf_counter() - t_setup
    print(f"[bench] warmup {args.warmup} steps done ({t_setup:.2f}s incl. setup)", file=sys.stderr,
          flush=True)

    # timed region: K macro-steps, one advance call each (the call returns after
    # the device finished the step) -> per-step latency and total wall time
    if args.profile:
        ctx.profile(True)
    torch.cuda.synchronize()
    lat = []
    iters = 0
    redone = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        st = ctx.advance(dt)
        lat.append(time.perf_counter() - s0)
        iters += st["pcg_iters"]
        redone += st["redone_steps"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = ctx.profile_read() if args.profile else None
    print(f"[bench] timed {args.steps} steps in {wall:.3f}s", file=sys.stderr, flush=True)

    dof_steps = N * args.steps / wall
    eta = args.steps * dt / wall
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": "look-ahead eta & DOF*steps/s at 1e-7 rel err; p50/p99 macro-step latency",
        "value": dof_steps,
        "unit": "DOF*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if pb.scheme.precision == 0 else "f32+f64-refine",
        "data": "synthetic",
        "config": {"workload": pb.name, "dof": N, "nnz": pb.nnz, "M": pb.scheme.M,
                   "nodes": "gauss-lobatto" if pb.scheme.family == 0 else "equidistant",
                   "K": pb.scheme.K, "P": pb.scheme.P, "dt_s": dt,
                   "simulated_s": args.steps * dt},
        "eta": eta,
        "p50_step_ms": float(np.percentile(lat_ms, 50)),
        "p99_step_ms": float(np.percentile(lat_ms, 99)),
        "cg_iters_per_step": iters / args.steps,
        "redone_steps": redone,
    }
    # dominant kernel: the CG operator application, timed with HIP events over
    # back-to-back launches on the library's stream (its own kernel symbol,
    # k_pcg_a<..., 2, ...>, in rocprof summaries)
    us, nbytes = ctx.time_operator(args.op_reps)
    achieved = nbytes / (us * 1e-6) / 1e9
    out["roofline"] = {"bound": "hbm", "kernel": "k_pcg_a (CG operator application)",
                       "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(pb),
                       "avg_launch_us": us, "launches": args.op_reps, "bytes_per_launch": nbytes}
    if kt and kt["iface_launches"]:
        out["iface_avg_us"] = kt["iface_ms"] / kt["iface_launches"] * 1e3
    ctx.destroy()

    if not args.no_cpu_baseline and args.cpu_steps > 0:
        import oracle
        S = args.cpu_steps
        ref_pb = workload(args.config, S)
        t = time.perf_counter()
        Tref, ost = oracle.run(ref_pb, nsteps=S)
        tc = time.perf_counter() - t
        out["cpu_baseline"] = {"value": N * S / tc, "unit": "DOF*steps/s",
                               "cores": int(ost["threads"]), "kind": "oracle",
                               "sample": f"first {S} of {args.steps} macro-steps of {pb.name}",
                               "seconds": tc, "pcg_share": ost["t_pcg"] / max(ost["t_total"], 1e-12)}
        g = pkg.simulation(ref_pb, device=0)
        g.advance(S * dt)
        Tg = pkg.get_state(g, ref_pb)
        g.destroy()
        out["rel_l2_vs_oracle"] = float(np.linalg.norm(Tg - Tref) / np.linalg.norm(Tref))
        out["rel_l2_sample_steps"] = S
    if args.precision_steps > 0 and args.config == "machine":
        out["fp32_refine"] = precision_form(pkg, args)
    if args.config == "machine":
        out["stationary"] = stationary_form(pkg, args)
        if args.wp_levels > 0:
            out["work_precision"] = work_precision_form(pkg, args)
        if args.deform_reps > 0:
            out["deformation"] = deformation_form(pkg, args)
        out["residual_control"] = residual_control_form(pkg, args, wall / args.steps)
    if args.ensemble_steps > 0 and args.config == "machine":
        import mrsdc_inputs as mi
        out["ensemble"] = ensemble(pkg, args, mi.FP32_REFINE)
        out["ensemble_fp64"] = ensemble(pkg, args, mi.FP64)
    print(json.dumps(out), flush=True)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)


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
    pb = mi.machine_310k(nsteps=args.steps)
    probe = pkg.simulation(pb, device=0, final_residual=1)
    r = probe.advance(pb.scheme.dt)["residual"]
    probe.destroy()
    tol = float(np.sqrt(r[1] * r[2]))
    sc = dataclasses.replace(pb.scheme, sweep_tol=tol)
    ctx = pkg.simulation(dataclasses.replace(pb, scheme=sc), device=0)
    ctx.advance(args.warmup * pb.scheme.dt)
    t = time.perf_counter()
    st = ctx.advance(args.steps * pb.scheme.dt)
    wall = time.perf_counter() - t
    ctx.destroy()
    out = {"sweep_tol": tol, "sweeps_per_step": st["sweeps"] / args.steps,
           "ms_per_step": wall / args.steps * 1e3, "eta": pb.scheme.dt * args.steps / wall,
           "speedup_vs_fixed_K": fixed_step_s / (wall / args.steps)}
    if not args.no_cpu_baseline:
        import oracle
        S = args.cpu_steps
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
    method classes of the work-precision study: MRSDC (Lobatto M=3, P=2,
    K=0,1,2), single-rate SDC (M=3, coupling implicit, K=0,1,2) and implicit
    Euler, on the benchmark machine from its stationary field (uniform T_env)
    over 10 motion periods.  The error is the max-norm difference at the end
    time to a reference run of MRSDC with Lobatto M=5, P=8, K=7 at a quarter
    of the finest level's dt (its own error estimated against the same run at
    twice that dt); eta = simulated time / wall time of the advance."""
    import dataclasses
    import mrsdc_inputs as mi
    base = mi.machine_310k(nsteps=1)
    base.T0 = np.full(base.N, 20.0)
    t_end = 10.0 * base.motion.period
    n0 = 4  # steps per period at the coarsest level
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
            pts.append({"dt_s": dt, "steps": st["steps"], "eta": t_end / st["wall_s"],
                        "max_err_K": err, "rel_err": err / rise,
                        "cg_iters": st["pcg_iters"]})
        curves.append({"method": name, "points": pts})
        print(f"[bench] work-precision {name}: " +
              " ".join(f"(eta {p['eta']:.0f}, err {p['rel_err']:.1e})" for p in pts),
              file=sys.stderr, flush=True)
    return {"workload": base.name, "t_end_s": t_end, "initial": "stationary (uniform T_env)",
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
    """Same machine, FP32 inner CG + FP64 refinement (error vs the FP64 path)."""
    import torch
    pb = workload("machine-fp32", args.precision_steps)
    dt = pb.scheme.dt
    ctx = pkg.simulation(pb, device=0)
    ctx.advance(args.warmup * dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.advance(args.precision_steps * dt)
    wall = time.perf_counter() - t0
    us, nbytes = ctx.time_operator(args.op_reps)
    ctx.destroy()
    print(f"[bench] fp32+refine {args.precision_steps} steps in {wall:.3f}s", file=sys.stderr,
          flush=True)
    return {"value": pb.N * args.precision_steps / wall, "unit": "DOF*steps/s",
            "ms_per_step": wall / args.precision_steps * 1e3,
            "eta": args.precision_steps * dt / wall,
            "op_avg_us": us, "op_GBps": nbytes / (us * 1e-6) / 1e9}


def serving(pkg, args):
    """Bounded replay of the seeded request trace (Poisson arrivals at 20/s,
    mesh levels 2 cm / 1 cm / 5 mm, per-request parameters), continuous
    batching per level; each request's steps capped to keep the run short."""
    import mrsdc_inputs as mi
    from paper_1707_03581_amd.serve import Request, Server, summarize
    trace = mi.serving_trace(args.serve_requests)
    needed = sorted({r["level"] for r in trace})
    levels = {}
    for name in needed:
        stand, stock = mi.MESH_LEVELS[name]
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
    srv = Server(levels, slots_per_level=64)
    done = srv.run(reqs)
    out = summarize(done, 5.0, {k: v.N for k, v in levels.items()})
    out["dtype"] = "f64" if args.serve_precision == 0 else "f32+f64-refine"
    if not args.no_cpu_baseline:
        # oracle on the smallest level's first request: error of a served result
        import oracle
        small = min(levels, key=lambda k: levels[k].N)
        r = next(q for q in done if q.level == small)
        ref, _ = oracle.run(levels[small], nsteps=r.nsteps, T0=r.T0, h=r.h, alpha=r.alpha,
                            friction_W=r.friction_W, period=r.period)
        out["rel_l2_vs_oracle_sample"] = {
            "request": r.id, "level": small, "steps": r.nsteps,
            "value": float(np.linalg.norm(r.result - ref) / np.linalg.norm(ref))}
    out.update({"metric": "serving: p50/p99 macro-step latency, per-request eta, DOF*steps/s",
                "workload": f"first {len(reqs)} requests of the 20 req/s trace, <= "
                            f"{args.serve_max_steps} steps each",
                "levels": {k: v.N for k, v in levels.items()},
                "footprint_bytes": srv.footprint})
    print(f"[bench] serving done in {srv.wall:.2f}s", file=sys.stderr, flush=True)
    return out


def ensemble(pkg, args, precision=None):
    """64 seeded scenarios on the 7.5 mm machine (714,798 DOF each), one batch."""
    import torch
    import mrsdc_inputs as mi
    S = 64
    if precision is None:
        precision = mi.FP32_REFINE
    pb = mi.ensemble_member(0, nsteps=args.ensemble_steps, precision=precision)
    members = []
    for s in range(S):
        h, alpha, pf, period, rng = mi.scenario_params(s)
        members.append(dict(h=h, alpha=alpha, friction_W=pf, period=period,
                            T0=20.0 + rng.uniform(-0.5, 0.5, size=pb.N)))
    dt = pb.scheme.dt
    ctx = pkg.batch_simulation(pb, members, device=0)
    ctx.advance_steps(1)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.ensemble_steps):
        s0 = time.perf_counter()
        ctx.advance_steps(1)
        lat.append(time.perf_counter() - s0)
    wall = time.perf_counter() - t0
    us, nbytes = ctx.time_operator(max(20, args.op_reps // 10))
    T_member0 = ctx.get_scenario_temperature(0, pb.N)
    ctx.destroy()
    print(f"[bench] ensemble {args.ensemble_steps} steps in {wall:.3f}s", file=sys.stderr,
          flush=True)
    lat_ms = np.array(lat) * 1e3
    form = "FP64" if precision == mi.FP64 else "FP32 inner + FP64 refinement"
    extra = {}
    if not args.no_cpu_baseline:
        # CPU oracle on member 0 over the same steps: error and a per-member baseline
        import oracle
        mb = members[0]
        nst = args.ensemble_steps + 1
        t = time.perf_counter()
        ref, ost = oracle.run(pb, nsteps=nst, T0=mb["T0"], h=mb["h"], alpha=mb["alpha"],
                              friction_W=mb["friction_W"], period=mb["period"])
        tc = time.perf_counter() - t
        extra["rel_l2_vs_oracle_member0"] = float(np.linalg.norm(T_member0 - ref) /
                                                  np.linalg.norm(ref))
        extra["cpu_baseline"] = {"value": pb.N * nst / tc, "unit": "DOF*steps/s",
                                 "cores": int(ost["threads"]), "kind": "oracle",
                                 "sample": f"member 0 alone, {nst} macro-steps", "seconds": tc}
    return {**extra, "workload": f"64 x {pb.N} DOF (7.5 mm machine), {form}", "scenarios": S,
            "dof_total": S * pb.N, "value": S * pb.N * args.ensemble_steps / wall,
            "unit": "DOF*steps/s", "ms_per_step": wall / args.ensemble_steps * 1e3,
            "eta_per_scenario": args.ensemble_steps * dt / wall,
            "p50_step_ms": float(np.percentile(lat_ms, 50)),
            "p99_step_ms": float(np.percentile(lat_ms, 99)),
            "op_kernel": "kb_pcg_a (multi-RHS operator)", "op_avg_us": us,
            "op_GBps": nbytes / (us * 1e-6) / 1e9, "op_frac_hbm": nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS}


if __name__ == "__main__":
    main()
