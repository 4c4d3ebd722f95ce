"""Benchmark of the JFNK hot path on one MI355X.

Workload: the 2D dry thermal in a stably stratified atmosphere, 1024 x 512 grid
over 20 x 10 km, N = 0.01 1/s, +2 K bubble, dt = 1 s, Smagorinsky closure.  One
step = one trapezoidal implicit step solved by inexact Newton (Eisenstat-Walker
forcing) to a relative residual of 1e-8, FGMRES(30).

The physics-based preconditioner of the timed legs applies its field-block
diagonal with --pc-sweeps Jacobi sweeps (default 0): on this workload the GMRES
iteration count is the same for 0 to 8 sweeps (the acoustic coupling between
fields, which no field block holds, sets it), so each sweep only adds time.

The Krylov solve of the timed legs uses the one-reduction Arnoldi step
(--ortho, jfnk_ortho): two passes over the basis per iteration instead of the
three of classical Gram-Schmidt applied twice, equal to it in exact arithmetic.

Legs, all from the same state after the warm-up steps:
  mixed     FP32 Krylov / Jv, physics-based preconditioner, FP64 Newton   (timed leg)
  plain     FP64 everywhere, physics-based preconditioner
  mixed_pc_sweeps2  the mixed leg with two preconditioner sweeps (the source of
            roofline_pc, whose kernels the timed legs launch without sweeps)
  mixed_cgs2  the mixed leg with the CGS2 Arnoldi step
  ensemble  one mixed step of the 64-instance heat-island ensemble (3.93 M points,
            uneven grids), reported in config.ensemble_64_heat_island
  learned   FP32 Krylov / Jv, learned BF16-MFMA right preconditioner, FP64 Newton;
            the network is trained first on pairs the solver generates on this
            workload (training time reported, not timed with the steps)
  mixed_p3  the mixed leg with the 9-point (p = 3) derivative
  mixed_deardorff  the mixed leg with the anisotropic exchange coefficients (Eq. 7)
  mixed_3d_256x256x128  the mixed leg on the 3D neutral thermal (20 x 20 x 10 km, dt = 2 s)
Each context is autotuned (tile or row-marching launch shapes) before its steps.
A second learned comparison runs on the same thermal at 256 x 128, where the
acoustic CFL number is a quarter of the full grid's.

Printed JSON line:
  value          whole-job Jv throughput of the timed leg: grid points x Jv
                 evaluations / wall time of the timed steps [Gpoint-residuals/s]
  ms_per_step    wall time per implicit step of the timed leg
  roofline       the dominant kernel class of the timed leg (algorithmic bytes over
                 the summed HIP-event time of its launches) against 8 TB/s HBM;
                 roofline_jv for the Jv kernel, roofline_pc for the preconditioner
                 (from mixed_pc_sweeps2), roofline_net for the network.
                 Each leg runs its steps twice from the same state: the wall time
                 above comes from the run without instrumentation, the per-class
                 HIP events from the second run (their packets add ~20% to a step)
  cpu_baseline   the FP64 oracle on a bounded sample of the same workload

kernel_micro   the residual, Jv and physics-preconditioner kernels alone on grids
               whose vectors exceed the 256 MB Infinity Cache (2D 8192 x 8192, p = 2
               and 3, 3D 256 x 256 x 128), FP32 and FP64: per-launch HIP-event time,
               algorithmic bytes (residual and Jv: read u and v or f, write the
               result, 3 n_f w per point; preconditioner: the library's per-launch
               count of its diagonal start and sweeps) and the HBM fraction

--copy-probe GIB runs only a device-to-device copy of GIB GiB (the calibration
kernel for the hardware byte counters) and prints its size and time.
--micro-only runs only the kernel micro-benchmark.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--learned-steps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--legs", default="mixed,plain,sweeps2,cgs2,learned,p3,deardorff,3d,ensemble")
    ap.add_argument("--ortho", default="one_reduction", choices=["one_reduction", "cgs2"],
                    help="Gram-Schmidt form of the Arnoldi step in the timed legs (the cgs2 leg repeats the timed "
                         "configuration with CGS2)")
    ap.add_argument("--pc-sweeps", type=int, default=0,
                    help="Jacobi sweeps of the physics preconditioner in the timed legs (0: its field-block "
                         "diagonal alone; the sweeps2 leg repeats the timed configuration with 2)")
    ap.add_argument("--train-iters", type=int, default=1500)
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--nz", type=int, default=512)
    ap.add_argument("--copy-probe", type=float, default=0.0)
    ap.add_argument("--micro-only", action="store_true")
    ap.add_argument("--pin", default="", help="launch shapes pinned over the autotuner on the timed "
                    "context, e.g. 'f32_jv=8,f32_pc_sweep=4' (rows per workgroup)")
    ap.add_argument("--micro-pin", default="", help="the same for the 2D micro-benchmark contexts")
    ap.add_argument("--no-micro", action="store_true")
    ap.add_argument("--micro-reps", type=int, default=20)
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_steps(ctx, u, k, torch, **opts):
    """Advance u by k implicit steps; returns per-step info."""
    infos = []
    nxt = torch.empty_like(u)
    for _ in range(k):
        nxt.copy_(u)
        r = ctx.newton_step(u, nxt, **opts)
        if not r.converged:
            raise RuntimeError(f"Newton did not converge: {r}")
        infos.append(r)
        u.copy_(nxt)
    return infos


def timed_leg(ctx, u0, k, torch, L, classes, **opts):
    """k steps from u0, twice: the wall time comes from a run without
    instrumentation; a second run of the same steps from the same state records
    HIP events around every launch of the given kernel classes (the event
    packets themselves cost about a fifth of the step time at 1024 x 512)."""
    u = u0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = run_steps(ctx, u, k, torch, **opts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mask = 0
    for c in classes.values():
        mask |= 1 << c
    ui = u0.clone()
    torch.cuda.synchronize()
    ctx.timing(mask)
    t0 = time.perf_counter()
    run_steps(ctx, ui, k, torch, **opts)
    torch.cuda.synchronize()
    wall_i = time.perf_counter() - t0
    tm = {name: ctx.timing_read(c) for name, c in classes.items()}    # (ms, launches, bytes or flops)
    ctx.timing(0)
    del ui
    return {"wall": wall, "wall_instrumented": wall_i, "infos": infos, "tm": tm, "u": u}


def per_step(leg):
    k = len(leg["infos"])
    return {"ms_per_step": leg["wall"] / k * 1e3,
            "newton_iters_per_step": sum(r.newton_iters for r in leg["infos"]) / k,
            "gmres_iters_per_step": sum(r.gmres_iters_total for r in leg["infos"]) / k,
            "fallbacks": sum(r.fallbacks for r in leg["infos"]),
            "ms_per_step_instrumented": leg["wall_instrumented"] / k * 1e3,
            "kernel_ms_per_step": {c: v[0] / k for c, v in leg["tm"].items()}}


def cpu_baseline(prob, U0, seconds, sweeps):
    """Oracle (FP64 numpy) on a bounded sample of the same workload: GMRES
    iterations of the first Newton iteration of the first step (physics
    preconditioner, stable-FD Jv, CGS2 Arnoldi), stopped after `seconds`."""
    from threadpoolctl import threadpool_limits

    from oracle import krylov as K
    from oracle import model as M
    from oracle import precond as PC

    with threadpool_limits(limits=1):
        f = M.rhs(prob, U0)
        R = M.residual(prob, U0, f)
        fr = PC.frozen_coefficients(prob, U0)
        calls = [0]
        t0 = time.perf_counter()

        class Stop(Exception):
            pass

        def mv(v):
            if time.perf_counter() - t0 > seconds:
                raise Stop
            calls[0] += 1
            return M.jv(prob, U0, v, M.fd_eps(prob, U0, v, 2.0 ** -52))

        pc = lambda r: PC.physics_pc(prob, U0, r, sweeps, fr)
        try:
            K.fgmres(mv, pc, -R, m=30, tol=1e-12, max_iters=10 ** 6, true_residual=False)
        except Stop:
            pass
        el = time.perf_counter() - t0
    gpts = prob.npts * calls[0] / el / 1e9
    return {"value": gpts, "unit": "Gpoint-residuals/s", "cores": 1, "kind": "oracle",
            "sample": f"{calls[0]} FP64 GMRES iterations (PC with {sweeps} sweeps + Jv + CGS2) of the first Newton "
                      f"iteration of step 1 on the same {prob.nx}x{prob.nz} grid, {el:.1f} s, 1 thread"}


def sources_sha256(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic(name, shapes=None):
    """HBM bytes per launch of a kernel class from the committed hardware-counter
    summary profiles/<name>.md (FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel
    factor), or None if there is none, the kernel sources changed since, or the
    launch shapes it was measured with differ from this run's."""
    path = os.path.join(ROOT, "profiles", name + ".md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"^sources: (.+)$", text, re.M)
    m_sha = re.search(r"^sources_sha256: ([0-9a-f]{64})$", text, re.M)
    m_val = re.search(r"^hbm_bytes_per_launch: ([0-9.eE+]+)$", text, re.M)
    if not (m_src and m_sha and m_val):
        return None
    if sources_sha256(m_src.group(1).split()) != m_sha.group(1):
        return None
    m_shape = re.search(r"^launch_shapes: (.+)$", text, re.M)
    if m_shape:
        want = parse_shapes(m_shape.group(1))
        if shapes is None or any(shapes.get(k) != v for k, v in want.items()):
            return None
    return float(m_val.group(1))


# rows per workgroup of a launch shape -> jfnk_set_variant variant
SHAPE_VARIANT = {4: 0, 8: 1, 16: 2, 32: 3, 64: 4, 256: 5}


def parse_shapes(text):
    """'f32_jv=8,f32_pc_sweep=4' -> {'f32_jv': 8, 'f32_pc_sweep': 4}"""
    out = {}
    for item in filter(None, (x.strip() for x in text.split(","))):
        k, v = item.split("=")
        out[k.strip()] = int(v)
    return out


def pin_shapes(ctx, shapes, pins):
    """Pin launch shapes (rows per workgroup) over the autotuner's choices."""
    for key, rows in pins.items():
        dtype, stage = key.split("_", 1)
        ctx.set_variant(stage, dtype, SHAPE_VARIANT[rows])
        shapes[key] = rows
    return shapes


def copy_probe(gib):
    import torch
    n = int(gib * 2 ** 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e)
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "ms": ms,
                      "GBps_read_plus_write": 8 * n / ms / 1e6}), flush=True)


def synth_state(torch, prob, seed=0):
    """Timing input on the device: smooth velocities (a few sine modes of a
    streamfunction in x-z, scaled to 10 m/s), the +2 K bubble and Gaussian
    pressure noise of standard deviation 0.01."""
    dev = "cuda"
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    nf, nz, ny, nx = prob.shape
    x = (torch.arange(nx, device=dev, dtype=torch.float64) + 0.5) * (prob.lx / nx)
    y = (torch.arange(ny, device=dev, dtype=torch.float64) + 0.5) * (prob.ly / ny)
    z = (torch.arange(nz, device=dev, dtype=torch.float64) + 0.5) * (prob.lz / nz)
    Z, Y, X = torch.meshgrid(z, y, x, indexing="ij")
    U = torch.zeros(prob.shape, dtype=torch.float64, device=dev)
    amp = torch.randn((4, 4), generator=g, device=dev, dtype=torch.float64)
    for m in range(1, 5):
        for n in range(1, 5):
            a = float(amp[m - 1, n - 1]) / (m * m + n * n)
            ax, az = m * math.pi / prob.lx, n * math.pi / prob.lz
            U[0] += -a * az * torch.sin(ax * X) * torch.cos(az * Z)
            U[prob.dim - 1] += a * ax * torch.cos(ax * X) * torch.sin(az * Z)
    if prob.dim == 3:
        U[1] = 0.5 * U[0] * torch.cos(math.pi * Y / prob.ly)
    vmax = U[:prob.dim].abs().max()
    U[:prob.dim] *= 10.0 / vmax
    r = torch.sqrt((X - prob.lx / 2) ** 2 + (Z - 2000.0) ** 2 + ((Y - prob.ly / 2) ** 2 if prob.dim == 3 else 0.0))
    U[-1] = torch.where(r <= 2000.0, 2.0 * torch.cos(math.pi * r / 4000.0) ** 2, torch.zeros_like(r))
    U[prob.dim] = 0.01 * torch.randn(U[prob.dim].shape, generator=g, device=dev, dtype=torch.float64)
    return U.reshape(-1)


def jv_kernel_name(rows):
    """Name of the FP32 Jv kernel of an autotuned launch shape (rows per workgroup)."""
    if rows >= 32:
        return f"k_march_2d<float, W, true> ({rows}-row chunks of 64-column strips)"
    return f"k_jv_2d<float, 64, {rows}>"


def kernel_micro(torch, I, L, Context, reps, pins=None):
    """Residual, Jv and physics-preconditioner kernels alone at sizes beyond the
    Infinity Cache."""
    out = {}
    cases = [("2d_8192x8192", I.thermal_stable_2d(8192, 8192)), ("3d_256x256x128", I.thermal_neutral_3d()),
             ("2d_8192x8192_p3", I.thermal_stable_2d(8192, 8192).replace(dd_p=3))]
    for name, prob in cases:
        ctx = Context(prob, max_m=1)
        shapes = ctx.tune()
        if prob.dim == 2 and pins:
            shapes = pin_shapes(ctx, shapes, pins)
        u64 = synth_state(torch, prob)
        g = torch.Generator(device="cuda")
        g.manual_seed(1)
        v64 = torch.randn(prob.n, generator=g, device="cuda", dtype=torch.float64)
        v64 /= v64.norm()
        res = {}
        for dt in ("f32", "f64"):
            u = u64 if dt == "f64" else u64.float()
            v = v64 if dt == "f64" else v64.float()
            f = torch.zeros_like(u)
            o = torch.empty_like(u)
            w = u.element_size()
            z = torch.empty_like(u)
            for _ in range(3):
                ctx.jv(u, v, o, mode="stable", eps=1e-3)
                ctx.apply_F(u, o, what=2, f=f)
                ctx.precond_apply(u, v, z, pc="physics", sweeps=2)
            torch.cuda.synchronize()
            # pc: one launch = the diagonal start or one Jacobi sweep (3 per application);
            # its algorithmic bytes are the library's own per-launch accounting
            for kname, call, cls in [("jv", lambda: ctx.jv(u, v, o, mode="stable", eps=1e-3), L.KC_JV),
                                     ("residual", lambda: ctx.apply_F(u, o, what=2, f=f), L.KC_RESIDUAL),
                                     ("pc", lambda: ctx.precond_apply(u, v, z, pc="physics", sweeps=2), L.KC_PC)]:
                ctx.timing(1 << cls)
                for _ in range(reps):
                    call()
                torch.cuda.synchronize()
                ms, launches, amount = ctx.timing_read(cls)
                ctx.timing(0)
                per = ms / launches * 1e3
                by = amount / launches if kname == "pc" else 3.0 * prob.n * w
                gbs = by / (per * 1e-6) / 1e9
                res[f"{kname}_{dt}"] = {"avg_launch_us": per, "bytes_per_launch": by, "GBps": gbs,
                                        "frac": gbs / HBM_PEAK_GBS,
                                        "gpts": prob.npts / (per * 1e-6) / 1e9}
        res["launch_shapes"] = shapes
        out[name] = res
        del ctx, u64, v64
        torch.cuda.empty_cache()
    return out


def learned_small(torch, I, LRN, Context, train_iters, sweeps, ortho):
    """Trained network vs the physics preconditioner (with the timed legs' sweep
    count and with two sweeps; and the plain FP64 solve with it) vs the untrained
    form on the stable thermal at 256 x 128 (two steps each from the same state)."""
    import numpy as np
    prob = I.thermal_stable_2d(256, 128)
    ctx = Context(prob, max_m=30)
    u = torch.from_numpy(I.bubble_state(prob)).cuda()
    R, DU, u_end = LRN.collect_pairs(ctx, u, steps=4, cap=256)
    t0 = time.perf_counter()
    theta, losses = LRN.train_mixed(ctx, R, DU, u_end, iters=train_iters, lr=2e-3, batch=8)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    out = {"grid": [256, 128], "train_s": train_s, "pairs": int(R.shape[0])}
    for name, pc, params, sw, inner in [("physics", "physics", None, sweeps, "f32"),
                                        ("physics_sweeps2", "physics", None, 2, "f32"),
                                        ("plain_f64_physics", "physics", None, sweeps, "f64"),
                                        ("learned", "learned", theta, 0, "f32"),
                                        ("untrained_form", "learned", np.zeros(ctx.n_params, np.float32), 0, "f32")]:
        if params is not None:
            ctx.net_set_params(params)
        extra = dict(eta_floor=1e-4) if inner == "f32" else {}
        leg = timed_leg(ctx, u_end, 2, torch, None, {}, rtol=1e-8, m=30, max_restarts=20, inner=inner,
                        pc=pc, sweeps=sw, ortho=ortho, **extra)
        out[name] = per_step(leg)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the solver would shard).", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return
    if args.micro_only:
        import torch

        from paper_2007_10411_amd import _lib as L
        from paper_2007_10411_amd import inputs as I
        from paper_2007_10411_amd.jfnk import Context
        torch.cuda.set_device(0)
        print(json.dumps({"kernel_micro": kernel_micro(torch, I, L, Context, args.micro_reps,
                                                       parse_shapes(args.micro_pin))}), flush=True)
        return
    import numpy as np
    import torch

    from paper_2007_10411_amd import _lib as L
    from paper_2007_10411_amd import inputs as I
    from paper_2007_10411_amd import learned as LRN
    from paper_2007_10411_amd.jfnk import Context

    legs_wanted = [x for x in args.legs.split(",") if x]
    if args.no_learned and "learned" in legs_wanted:
        legs_wanted.remove("learned")
    if "mixed" not in legs_wanted:
        legs_wanted.insert(0, "mixed")
    torch.cuda.set_device(0)
    prob = I.thermal_stable_2d(args.nx, args.nz)
    U0 = I.bubble_state(prob)
    ctx = Context(prob, max_m=30)
    shapes = ctx.tune()                 # launch shapes of the stencil stages (setup, untimed)
    shapes = pin_shapes(ctx, shapes, parse_shapes(args.pin))
    log(f"launch shapes (rows per workgroup): {shapes}")
    common = dict(rtol=1e-8, m=30, max_restarts=20, ortho=args.ortho)
    opts = {"mixed": dict(common, inner="f32", eta_floor=1e-4, pc="physics", sweeps=args.pc_sweeps),
            "plain": dict(common, inner="f64", pc="physics", sweeps=args.pc_sweeps),
            "learned": dict(common, inner="f32", eta_floor=1e-4, pc="learned")}
    steps = {"mixed": args.steps, "plain": args.plain_steps, "learned": args.learned_steps}
    classes = {"mixed": {"jv": L.KC_JV, "pc": L.KC_PC, "arnoldi": L.KC_ARNOLDI},
               "plain": {"jv": L.KC_JV, "pc": L.KC_PC, "arnoldi": L.KC_ARNOLDI},
               "learned": {"jv": L.KC_JV, "arnoldi": L.KC_ARNOLDI, "net": L.KC_NET}}

    u = torch.from_numpy(U0).cuda()
    log(f"warmup {args.warmup} mixed steps")
    run_steps(ctx, u, args.warmup, torch, **opts["mixed"])
    legs = {}
    log(f"timing {steps['mixed']} mixed steps")
    legs["mixed"] = timed_leg(ctx, u, steps["mixed"], torch, L, classes["mixed"], **opts["mixed"])
    if "plain" in legs_wanted:
        log(f"timing {steps['plain']} plain FP64 steps")
        legs["plain"] = timed_leg(ctx, u, steps["plain"], torch, L, classes["plain"], **opts["plain"])
    if "sweeps2" in legs_wanted:
        # the timed configuration with two Jacobi sweeps in the physics preconditioner
        log(f"timing {steps['plain']} mixed steps with two preconditioner sweeps")
        legs["mixed_pc_sweeps2"] = timed_leg(ctx, u, steps["plain"], torch, L, classes["mixed"],
                                             **dict(opts["mixed"], sweeps=2))
    if "cgs2" in legs_wanted and args.ortho != "cgs2":
        # the timed configuration with classical Gram-Schmidt applied twice
        log(f"timing {steps['plain']} mixed steps with the CGS2 Arnoldi step")
        legs["mixed_cgs2"] = timed_leg(ctx, u, steps["plain"], torch, L, classes["mixed"],
                                       **dict(opts["mixed"], ortho="cgs2"))
    train_info = None
    small = None
    if "learned" in legs_wanted:
        log("recording solver pairs and training the learned preconditioner")
        t0 = time.perf_counter()
        R, DU, u_tr = LRN.collect_pairs(ctx, u, steps=2, cap=96)
        t1 = time.perf_counter()
        theta, losses = LRN.train_mixed(ctx, R, DU, u_tr, iters=args.train_iters, lr=2e-3, batch=8)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        train_info = {"pairs": int(R.shape[0]), "collect_s": t1 - t0, "train_s": t2 - t1,
                      "adam_steps": args.train_iters, "dilations": list(LRN.DILATIONS),
                      "loss_first": losses[0], "loss_last": float(np.mean(losses[-20:]))}
        del R, DU
        torch.cuda.empty_cache()
        log(f"timing {steps['learned']} learned steps")
        legs["learned"] = timed_leg(ctx, u, steps["learned"], torch, L, classes["learned"], **opts["learned"])
        log("learned vs physics preconditioner at 256 x 128")
        small = learned_small(torch, I, LRN, Context, args.train_iters, args.pc_sweeps, args.ortho)
    if "p3" in legs_wanted:
        # the same workload with the 9-point (p = 3) derivative
        prob3 = prob.replace(dd_p=3)
        ctx3 = Context(prob3, max_m=30)
        ctx3.tune()
        u3 = torch.from_numpy(U0).cuda()
        log("mixed steps with the 9-point stencil")
        run_steps(ctx3, u3, args.warmup, torch, **opts["mixed"])
        legs["mixed_p3"] = timed_leg(ctx3, u3, args.plain_steps, torch, L, classes["mixed"], **opts["mixed"])
        del ctx3
    if "deardorff" in legs_wanted:
        # the same workload with the anisotropic exchange coefficients of Eq. 7
        probd = prob.replace(closure=I.CLOSURE_DEARDORFF)
        ctxd = Context(probd, max_m=30)
        ctxd.tune()
        ud = torch.from_numpy(U0).cuda()
        log("mixed steps with the anisotropic (Eq. 7) closure")
        run_steps(ctxd, ud, args.warmup, torch, **opts["mixed"])
        legs["mixed_deardorff"] = timed_leg(ctxd, ud, args.plain_steps, torch, L, classes["mixed"],
                                            **opts["mixed"])
        del ctxd
    if "3d" in legs_wanted:
        # the 3D neutral thermal at 256 x 256 x 128 (20 x 20 x 10 km, dt = 2 s), mixed precision
        prob3d = I.thermal_neutral_3d()
        ctx3d = Context(prob3d, max_m=30)
        u3d = torch.from_numpy(I.bubble_state(prob3d)).cuda()
        log("mixed steps of the 3D thermal 256x256x128")
        run_steps(ctx3d, u3d, 1, torch, **opts["mixed"])
        legs["mixed_3d_256x256x128"] = timed_leg(ctx3d, u3d, args.plain_steps, torch, L, classes["mixed"],
                                                 **opts["mixed"])
        del ctx3d, u3d
        torch.cuda.empty_cache()

    ensemble = None
    if "ensemble" in legs_wanted:
        # the 64-instance heat-island ensemble (uneven 2D grids, one launch per stage)
        from paper_2007_10411_amd.jfnk import Batch
        log("one mixed step of the 64-instance heat-island ensemble")
        eprobs = I.heat_island_ensemble(64, seed=0)
        bt = Batch(eprobs, max_m=30)
        erows = bt.tune()
        un_e = bt.pack([I.rest_state(p) for p in eprobs])
        ue = un_e.clone()
        bt.newton_step(un_e, ue, sweeps=args.pc_sweeps, ortho=args.ortho)   # untimed: first launches
        ue = un_e.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eres = bt.newton_step(un_e, ue, sweeps=args.pc_sweeps, ortho=args.ortho)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        its = [r.gmres_iters_total for r in eres]
        ensemble = {"instances": len(eprobs), "points": int(sum(p.npts for p in eprobs)),
                    "ms_per_step": el * 1e3, "converged": all(r.converged for r in eres),
                    "gmres_iters_per_instance": [min(its), max(its)], "gmres_iters_total": sum(its),
                    "pc_sweeps": args.pc_sweeps, "ortho": args.ortho, "launch_shapes": erows}
        del bt, un_e, ue
        torch.cuda.empty_cache()

    T = legs["mixed"]
    tm = T["tm"]
    npts = prob.npts

    def roof(leg, name, kernel, bound="hbm", traffic=None):
        ms, launches, amount = legs[leg]["tm"][name]
        rate = amount / (ms / 1e3) if ms > 0 else 0.0
        per = amount / max(launches, 1)
        if bound == "mfma":
            achieved = rate / 1e12
            return {"kernel": kernel, "bound": "mfma", "achieved": achieved, "peak": BF16_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved / BF16_PEAK_TFLOPS, "traffic": None,
                    "flops_per_launch": per, "avg_launch_us": ms / max(launches, 1) * 1e3, "launches": launches}
        achieved = rate / 1e9
        return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "bytes_per_launch": per, "avg_launch_us": ms / max(launches, 1) * 1e3, "launches": launches}

    kernels = {"arnoldi": ("k_dg_dot<float> + k_dg_finish + k_dg_update<float> (one-reduction Arnoldi step and "
                           "Givens step of one GMRES iteration)" if args.ortho == "one_reduction" else
                           "k_cgs_reg<float> x3 + k_cgs_finish x3 (CGS2 passes and Givens step of one GMRES "
                           "iteration)"),
               "pc": "k_pc_diag_2d<float> + 2 x k_pc_sweep_2d<float> (physics preconditioner with two sweeps, "
                     "mixed_pc_sweeps2 leg)" if "mixed_pc_sweeps2" in legs else
                     f"k_pc_diag_2d<float> + {args.pc_sweeps} x k_pc_sweep_2d<float> (physics preconditioner)",
               "jv": f"{jv_kernel_name(shapes['f32_jv'])} (stable finite-difference Jv)"}
    traffic_name = {"arnoldi": ("arnoldi_f32_counters_thermal_stable_1024x512" if args.ortho == "one_reduction"
                                else "arnoldi_cgs2_f32_counters_thermal_stable_1024x512"),
                    "pc": "pc_f32_counters_thermal_stable_1024x512",
                    "jv": "jv_f32_counters_thermal_stable_1024x512"}
    dominant = max(kernels, key=lambda k: tm[k][0])
    full = (prob.nx, prob.nz) == (1024, 512)

    def traffic_of(k):
        return counter_traffic(traffic_name[k], shapes) if full else None

    jv_ms, jv_launches, _ = tm["jv"]
    value = npts * jv_launches / T["wall"] / 1e9
    out = {
        "metric": "Gpoint-residuals/s (Jv) and ms per implicit step at 1e-8 Newton tol, plain vs learned",
        "value": value,
        "unit": "Gpoint-residuals/s",
        "n_gpus": 1,
        "steps": steps["mixed"],
        "warmup": args.warmup,
        "ms_per_step": T["wall"] / steps["mixed"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 Krylov/Jv, f64 Newton",
        "data": "synthetic",
        "config": {
            "workload": f"stable 2D dry thermal {prob.nx}x{prob.nz} (20x10 km, N=0.01/s, +2 K bubble, "
                        f"dt={prob.dt} s, Smagorinsky), mixed-precision JFNK with the physics-based "
                        f"preconditioner (field-block diagonal, {args.pc_sweeps} Jacobi sweeps): FGMRES(30) "
                        f"with the {args.ortho} Arnoldi step, Newton rtol 1e-8",
            "grid": [prob.nx, prob.nz],
            "pc_sweeps": args.pc_sweeps,
            "ortho": args.ortho,
            "timed_leg": "mixed",
            "legs": {k: per_step(v) for k, v in legs.items()},
            "plain_over_mixed_time": (per_step(legs["plain"])["ms_per_step"] / per_step(T)["ms_per_step"]
                                      if "plain" in legs else None),
            "training": train_info,
            "learned_256x128": small,
            "ensemble_64_heat_island": ensemble,
            "jv_kernel_gpts": npts * jv_launches / (jv_ms / 1e3) / 1e9 if jv_ms > 0 else 0.0,
            "kernel_ms_per_step": {k: v[0] / steps["mixed"] for k, v in tm.items()},
            "launch_shapes": shapes,
        },
        "roofline": roof("mixed", dominant, kernels[dominant], traffic=traffic_of(dominant)),
        "roofline_jv": roof("mixed", "jv", kernels["jv"], traffic=traffic_of("jv")),
        "roofline_pc": roof("mixed_pc_sweeps2" if "mixed_pc_sweeps2" in legs else "mixed", "pc", kernels["pc"],
                            traffic=traffic_of("pc")),
    }
    if "learned" in legs and legs["learned"]["tm"]["net"][1] > 0:
        out["roofline_net"] = roof("learned", "net", "k_conv_mfma x4 (BF16 3x3 conv layers of the learned PC)",
                                   "mfma")
    if not args.no_micro:
        del legs
        torch.cuda.empty_cache()
        log("kernel micro-benchmark (2D 8192x8192, 3D 256x256x128)")
        micro = kernel_micro(torch, I, L, Context, args.micro_reps, parse_shapes(args.micro_pin))
        out["kernel_micro"] = micro
        best = micro["2d_8192x8192"]["jv_f32"]
        jk = jv_kernel_name(micro["2d_8192x8192"]["launch_shapes"]["f32_jv"])
        out["roofline_jv_micro"] = {"kernel": f"{jk} at 8192x8192 (vectors beyond the Infinity Cache)",
                                    "bound": "hbm", "achieved": best["GBps"], "peak": HBM_PEAK_GBS,
                                    "unit": "GB/s", "frac": best["frac"],
                                    "traffic": counter_traffic("jv_f32_counters_8192x8192",
                                                               micro["2d_8192x8192"]["launch_shapes"]),
                                    "bytes_per_launch": best["bytes_per_launch"],
                                    "avg_launch_us": best["avg_launch_us"]}
    if not args.no_cpu:
        log(f"cpu baseline ({args.cpu_seconds} s)")
        out["cpu_baseline"] = cpu_baseline(prob, U0, args.cpu_seconds, args.pc_sweeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
