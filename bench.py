"""Benchmark of the JFNK hot path on one MI355X.

Headline workload: the 3D neutral dry thermal, 256 x 256 x 128 points over
20 x 20 x 10 km (78.125 m spacing), +2 K cosine-squared bubble of radius 2 km
at (10, 10, 2) km, dt = 2 s, Smagorinsky closure, free-slip walls.  One step =
one trapezoidal implicit step solved by inexact Newton (Eisenstat-Walker
forcing) to a relative residual of 1e-8 with FGMRES(30).

Legs at that size, each from the same state after the warm-up steps:
  mixed     FP32 Krylov / Jv, physics-based preconditioner, FP64 Newton   (timed leg)
  plain     FP64 everywhere, physics-based preconditioner
  learned   FP32 Krylov / Jv, learned BF16-MFMA 3x3x3 right preconditioner judged
            by the physics-based one, FP64 Newton; the network is trained first on
            crops of solver pairs from this workload and from the 2D thermal at the
            same spacing and time step (training reported, not timed with the steps)
The physics-based preconditioner applies its field-block diagonal with
--pc-sweeps Jacobi sweeps (default 0: on these workloads the sweeps leave the
GMRES iteration count unchanged).  The Krylov solves use the one-reduction
Arnoldi step (--ortho).

config.mixed_vs_fp64: the mixed steps' error per field against the plain FP64
steps after the plain leg's step count (relative to the FP64 steps' change and to
the field), the FP64 path being the one that matches the oracle to 1e-11.

Further legs (config.legs_2d, config.learned_256x128, config.ensemble_64_heat_island):
the 2D stable thermal at 1024 x 512 (mixed and plain), the trained 2D network
against the physics preconditioner at 256 x 128, and one mixed step of the
64-instance heat-island ensemble.

Printed JSON line:
  value          Jv throughput of the timed leg: grid points x Jv evaluations /
                 summed Jv kernel time (HIP events on the context stream around
                 every Jv launch of the steps) [Gpoint-residuals/s]
  ms_per_step    wall time per implicit step of the timed leg
  roofline       the dominant kernel class of the timed leg (algorithmic bytes over
                 the summed HIP-event time of its launches) against 8 TB/s HBM;
                 roofline_jv for the Jv kernel, roofline_pc for the preconditioner,
                 roofline_net for the network.  Each leg runs its steps twice from
                 the same state: the wall time comes from the run without events,
                 the kernel-class times from the second run.
  cpu_baseline   the FP64 oracle's Jv on a bounded sample of the same workload (the
                 lowest planes of the grid), on all host cores (one process per
                 core) and on one core (value_1core), with nproc and the CPU model
  kernel_micro   the residual, Jv and physics-preconditioner kernels alone (3D
                 256 x 256 x 128 and 2D 8192 x 8192, vectors beyond the Infinity
                 Cache), FP32 and FP64: per-launch HIP-event time, algorithmic bytes
                 and the HBM fraction

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
# FP32 vector issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one lane operation per
# lane and cycle without packed FP32; FP32 FMA counts as one operation here)
VALU_PEAK_TLANEOPS = 256 * 4 * 16 * 2.4e9 / 1e12
ALL_LEGS = "mixed,plain,learned,2d,learned2d,ensemble"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--learned-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--legs", default=ALL_LEGS)
    ap.add_argument("--ortho", default="one_reduction", choices=["one_reduction", "cgs2"],
                    help="Gram-Schmidt form of the Arnoldi step in the timed legs")
    ap.add_argument("--pc-sweeps", type=int, default=0,
                    help="Jacobi sweeps of the physics preconditioner in the timed legs (0: its field-block "
                         "diagonal alone)")
    ap.add_argument("--train-iters", type=int, default=600)
    ap.add_argument("--train-iters-2d", type=int, default=3000)
    ap.add_argument("--train-lr-2d", type=float, default=4e-3)
    ap.add_argument("--copy-probe", type=float, default=0.0)
    ap.add_argument("--micro-only", action="store_true")
    ap.add_argument("--pin", default="", help="launch shapes pinned over the autotuner on the 2D "
                    "contexts, e.g. 'f32_jv=8,f32_pc_sweep=4' (rows per workgroup)")
    ap.add_argument("--micro-pin", default="", help="the same for the 2D micro-benchmark contexts")
    ap.add_argument("--no-micro", action="store_true")
    ap.add_argument("--micro-reps", type=int, default=20)
    ap.add_argument("--micro-cases", default="3d_256x256x128,2d_8192x8192,2d_8192x8192_p3",
                    help="kernel micro-benchmark cases to run")
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
    HIP events around every launch of the given kernel classes."""
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
    infos_i = run_steps(ctx, ui, k, torch, **opts)
    torch.cuda.synchronize()
    wall_i = time.perf_counter() - t0
    tm = {name: ctx.timing_read(c) for name, c in classes.items()}    # (ms, launches, bytes or flops)
    ctx.timing(0)
    del ui
    return {"wall": wall, "wall_instrumented": wall_i, "infos": infos, "infos_instrumented": infos_i, "tm": tm,
            "u": u}


def per_step(leg, npts=None):
    k = len(leg["infos"])
    nn = sum(r.newton_iters for r in leg["infos"])
    ng = sum(r.gmres_iters_total for r in leg["infos"])
    out = {"ms_per_step": leg["wall"] / k * 1e3,
           "newton_iters_per_step": nn / k,
           "gmres_iters_per_step": ng / k,
           "gmres_iters_per_newton_iter": ng / max(nn, 1),
           "fallbacks": sum(r.fallbacks for r in leg["infos"]),
           "ms_per_step_instrumented": leg["wall_instrumented"] / k * 1e3,
           "kernel_ms_per_step": {c: v[0] / k for c, v in leg["tm"].items()}}
    if npts is not None and "jv" in leg["tm"] and leg["tm"]["jv"][0] > 0:
        ms, launches, _ = leg["tm"]["jv"]
        out["jv_kernel_gpts"] = npts * launches / (ms / 1e3) / 1e9
    return out


def field_differences(torch, ctx, u0, u_ref, k, opts, names):
    """The mixed-precision steps' error per field against the plain FP64 steps
    (whose FP64 kernels match the oracle to 1e-11): k mixed steps from u0 (not
    timed), then ||u_mixed - u_fp64|| relative to the FP64 steps' change
    ||u_fp64 - u0|| and to ||u_fp64||, per field."""
    u = u0.clone()
    run_steps(ctx, u, k, torch, **opts)
    nf = len(names)
    d = (u - u_ref).reshape(nf, -1).norm(dim=1)
    ch = (u_ref - u0).reshape(nf, -1).norm(dim=1)
    nr = u_ref.reshape(nf, -1).norm(dim=1)
    out = {"steps": k}
    for i, name in enumerate(names):
        out[name] = {"rel_to_change": float(d[i] / ch[i]) if ch[i] > 0 else None,
                     "rel_to_field": float(d[i] / nr[i]) if nr[i] > 0 else None}
    del u
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_jv_worker(args):
    """One process: the oracle's FP64 stable-FD Jv on the sample, repeated until
    `seconds` have passed, with one BLAS / OpenMP thread.  Returns (calls, points
    per call, seconds)."""
    nz_s, seconds = args
    from threadpoolctl import threadpool_limits

    import numpy as np

    from oracle import model as M
    from paper_2007_10411_amd import inputs as I
    full = I.thermal_neutral_3d()
    prob = full.replace(nz=nz_s, lz=full.lz * nz_s / full.nz)
    U = I.bubble_state(prob, center=(full.lx / 2, full.ly / 2, 2000.0))
    V = I.random_vector(prob, seed=1)
    calls = 0
    with threadpool_limits(limits=1):
        eps = M.fd_eps(prob, U, V, 2.0 ** -52)
        t0 = time.perf_counter()
        while True:
            M.jv(prob, U, V, eps)
            calls += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                break
    return calls, prob.npts, el


def cpu_baseline(seconds, nz_s=16):
    """FP64 oracle on a bounded sample of the workload: its Jv on the lowest
    nz_s planes of the 256 x 256 x 128 grid (same spacing, bubble state, unit
    random direction), on one core and then on every core of the host's share
    (one single-threaded process per core, all at once)."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    c1, npts, el1 = _oracle_jv_worker((nz_s, seconds))
    one = npts * c1 / el1 / 1e9
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_jv_worker, [(nz_s, seconds)] * cores)
    wall = time.perf_counter() - t0
    pts = sum(c * n for c, n, _ in res)
    span = max(e for _, _, e in res)
    allv = pts / span / 1e9
    return {"value": allv, "unit": "Gpoint-residuals/s", "cores": cores, "kind": "oracle",
            "sample": f"the FP64 oracle's stable-FD Jv on the lowest {nz_s} planes of the 256x256x128 grid "
                      f"({npts} points, bubble state, unit random direction): {cores} single-threaded "
                      f"processes at once, {sum(c for c, _, _ in res)} evaluations in {span:.1f} s "
                      f"(pool wall {wall:.1f} s); one process alone: {c1} evaluations in {el1:.1f} s",
            "value_1core": one, "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "affinity_cores": len(os.sched_getaffinity(0))}


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


def counter_value(name, key):
    """A per-launch figure (line '<key>: <value>') of the committed counter summary
    profiles/<name>.md, or None if there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", name + ".md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"^sources: (.+)$", text, re.M)
    m_sha = re.search(r"^sources_sha256: ([0-9a-f]{64})$", text, re.M)
    m_val = re.search(r"^" + re.escape(key) + r": ([0-9.eE+]+)$", text, re.M)
    if not (m_src and m_sha and m_val) or sources_sha256(m_src.group(1).split()) != m_sha.group(1):
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


# kernels of the 3D operators (256 x 256 x 128)
JV3_KERNEL = "k3f_jv<16> (single z-marching launch, 32 x 16 columns, ring columns on waves of their own)"
RES3_KERNEL = "k3m_derived<double, false> + k3m_point<double, 0, 8>"


def jv_kernel_name(rows):
    """Name of the FP32 Jv kernel of an autotuned launch shape (rows per workgroup)."""
    if rows >= 32:
        return f"k_march_2d<float, W, true> ({rows}-row chunks of 64-column strips)"
    return f"k_jv_2d<float, 64, {rows}>"


def kernel_micro(torch, I, L, Context, reps, pins=None, names=None):
    """Residual, Jv and physics-preconditioner kernels alone at sizes beyond the
    Infinity Cache."""
    out = {}
    cases = [("3d_256x256x128", I.thermal_neutral_3d()), ("2d_8192x8192", I.thermal_stable_2d(8192, 8192)),
             ("2d_8192x8192_p3", I.thermal_stable_2d(8192, 8192).replace(dd_p=3))]
    if names:
        cases = [c for c in cases if c[0] in names]
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


def learned_small(torch, I, LRN, Context, train_iters, sweeps, ortho, lr=4e-3):
    """Trained network vs the physics preconditioner (with the timed legs' sweep
    count and with two sweeps; and the plain FP64 solve with it) vs the untrained
    form on the stable thermal at 256 x 128 (two steps each from the same state)."""
    import numpy as np
    prob = I.thermal_stable_2d(256, 128)
    ctx = Context(prob, max_m=30)
    u = torch.from_numpy(I.bubble_state(prob)).cuda()
    R, DU, u_end = LRN.collect_pairs(ctx, u, steps=4, cap=256)
    t0 = time.perf_counter()
    theta, losses = LRN.train_mixed(ctx, R, DU, u_end, iters=train_iters, lr=lr, batch=8)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    out = {"grid": [256, 128], "train_s": train_s, "pairs": int(R.shape[0]), "adam_steps": train_iters, "lr": lr,
           "loss_last": float(np.mean(losses[-50:]))}
    zero = np.zeros(ctx.n_params, np.float32)
    # learned: judged by the physics-based preconditioner (the library's behaviour);
    # *_unjudged: the network's own iteration counts
    for name, pc, params, sw, inner, judge in [("physics", "physics", None, sweeps, "f32", True),
                                               ("physics_sweeps2", "physics", None, 2, "f32", True),
                                               ("plain_f64_physics", "physics", None, sweeps, "f64", True),
                                               ("learned", "learned", theta, 0, "f32", True),
                                               ("learned_unjudged", "learned", theta, 0, "f32", False),
                                               ("untrained_form_unjudged", "learned", zero, 0, "f32", False)]:
        if params is not None:
            ctx.net_set_params(params)
        extra = dict(eta_floor=1e-4) if inner == "f32" else {}
        leg = timed_leg(ctx, u_end, 2, torch, None, {}, rtol=1e-8, m=30, max_restarts=20, inner=inner,
                        pc=pc, sweeps=sw, ortho=ortho, judge=judge, **extra)
        out[name] = per_step(leg)
    return out


def train_learned_3d(torch, I, LRN, Context, ctx, u, iters, sweeps):
    """Train the 3x3x3 network of the 256 x 256 x 128 context on crops of solver
    pairs: Krylov directions and their images from one physics-preconditioned
    step of this workload (64 x 64 x 32 crops), the same from the 2D neutral
    thermal at the same spacing and time step (256 x 128, embedded as y-invariant
    3D fields, 128 x 16 x 64 crops), and noise directions through this
    context's Jv (64 x 64 x 32 crops)."""
    t0 = time.perf_counter()
    p3 = ctx.prob
    R3, DU3, _ = LRN.collect_pairs(ctx, u, steps=1, cap=24, sweeps=sweeps)
    p2 = I.thermal_neutral_2d(256, 128)
    ctx2 = Context(p2, max_m=30)
    u2 = torch.from_numpy(I.bubble_state(p2)).cuda()
    R2, DU2, _ = LRN.collect_pairs(ctx2, u2, steps=3, cap=64, sweeps=sweeps)
    ny2 = 16
    R2e, DU2e = LRN.embed_2d(R2, p2.nx, p2.nz, ny2), LRN.embed_2d(DU2, p2.nx, p2.nz, ny2)
    del ctx2, R2, DU2
    t1 = time.perf_counter()
    crop3 = (64, 64, 32)
    sources = [(R3, DU3, (p3.nf, p3.nz, p3.ny, p3.nx), crop3),
               (R2e, DU2e, (5, p2.nz, ny2, p2.nx), (128, ny2, 64))]
    noise = (LRN.NoisePairs(ctx, u, LRN.field_rms(DU3, p3.nf), seed=1), crop3)
    theta, losses = LRN.train_3d_crops(ctx, sources, iters=iters, lr=2e-3, batch=4, noise=noise)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = {"pairs_3d": int(R3.shape[0]), "pairs_2d": int(R2e.shape[0]), "crop_3d": list(crop3),
            "crop_2d_embedded": [128, ny2, 64], "collect_s": t1 - t0, "train_s": t2 - t1, "adam_steps": iters,
            "loss_first": float(losses[0]), "loss_last": float(sum(losses[-30:]) / min(30, len(losses))),
            "loss_every_100": [float(x) for x in losses[::100]]}
    del R3, DU3, R2e, DU2e
    torch.cuda.empty_cache()
    return theta, info


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path (one GPU per "
              "process; --gpus must be 1).", file=sys.stderr)
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
                                                       parse_shapes(args.micro_pin),
                                                       args.micro_cases.split(","))}), flush=True)
        return
    import numpy as np
    import torch

    from paper_2007_10411_amd import _lib as L
    from paper_2007_10411_amd import inputs as I
    from paper_2007_10411_amd import learned as LRN
    from paper_2007_10411_amd.jfnk import Context

    legs_wanted = [x for x in args.legs.split(",") if x]
    if args.no_learned:
        legs_wanted = [x for x in legs_wanted if x not in ("learned", "learned2d")]
    if "mixed" not in legs_wanted:
        legs_wanted.insert(0, "mixed")
    torch.cuda.set_device(0)
    prob = I.thermal_neutral_3d()
    npts = prob.npts
    ctx = Context(prob, max_m=30)
    shapes = ctx.tune()
    common = dict(rtol=1e-8, m=30, max_restarts=20, ortho=args.ortho)
    opts = {"mixed": dict(common, inner="f32", eta_floor=1e-4, pc="physics", sweeps=args.pc_sweeps),
            "plain": dict(common, inner="f64", pc="physics", sweeps=args.pc_sweeps),
            "learned": dict(common, inner="f32", eta_floor=1e-4, pc="learned", sweeps=args.pc_sweeps)}
    steps = {"mixed": args.steps, "plain": args.plain_steps, "learned": args.learned_steps}
    cls = {"jv": L.KC_JV, "pc": L.KC_PC, "arnoldi": L.KC_ARNOLDI, "residual": L.KC_RESIDUAL}
    classes = {"mixed": cls, "plain": cls, "learned": dict(cls, net=L.KC_NET)}

    u = torch.from_numpy(I.bubble_state(prob)).cuda()
    log(f"3D thermal 256x256x128: warmup {args.warmup} mixed steps")
    run_steps(ctx, u, args.warmup, torch, **opts["mixed"])
    legs = {}
    log(f"timing {steps['mixed']} mixed steps")
    legs["mixed"] = timed_leg(ctx, u, steps["mixed"], torch, L, classes["mixed"], **opts["mixed"])
    mixed_vs_fp64 = None
    if "plain" in legs_wanted:
        log(f"timing {steps['plain']} plain FP64 steps")
        legs["plain"] = timed_leg(ctx, u, steps["plain"], torch, L, classes["plain"], **opts["plain"])
        mixed_vs_fp64 = field_differences(torch, ctx, u, legs["plain"]["u"], steps["plain"], opts["mixed"],
                                          ("u", "v", "w", "p", "theta"))
    train_info = None
    learned_error = None
    if "learned" in legs_wanted:
        log("recording solver pairs and training the 3D network")
        theta, train_info = train_learned_3d(torch, I, LRN, Context, ctx, u, args.train_iters, args.pc_sweeps)
        # the judge's record: one physics-preconditioned step of the timed configuration
        run_steps(ctx, u.clone(), 1, torch, **opts["mixed"])
        log(f"timing {steps['learned']} learned steps")
        try:
            legs["learned"] = timed_leg(ctx, u, steps["learned"], torch, L, classes["learned"], **opts["learned"])
        except RuntimeError as ex:            # reported in the line, not hidden
            learned_error = str(ex)
            log(f"learned leg failed: {ex}")
    del ctx
    torch.cuda.empty_cache()

    legs_2d = None
    if "2d" in legs_wanted:
        # the 2D stable thermal at 1024 x 512 (N = 0.01 1/s, dt = 1 s), mixed and plain
        p2 = I.thermal_stable_2d(1024, 512)
        c2 = Context(p2, max_m=30)
        sh2 = pin_shapes(c2, c2.tune(), parse_shapes(args.pin))
        u2 = torch.from_numpy(I.bubble_state(p2)).cuda()
        log("2D stable thermal 1024x512: mixed and plain legs")
        run_steps(c2, u2, args.warmup, torch, **opts["mixed"])
        legs_2d = {"workload": "stable 2D dry thermal 1024x512 (20x10 km, N=0.01/s, dt=1 s)", "launch_shapes": sh2}
        for name in ("mixed", "plain"):
            k = steps["mixed"] if name == "mixed" else steps["plain"]
            legs_2d[name] = per_step(timed_leg(c2, u2, k, torch, L, cls, **opts[name]), p2.npts)
        del c2, u2
        torch.cuda.empty_cache()
    small = None
    if "learned2d" in legs_wanted:
        log("learned vs physics preconditioner, 2D stable thermal 256 x 128")
        small = learned_small(torch, I, LRN, Context, args.train_iters_2d, args.pc_sweeps, args.ortho,
                              args.train_lr_2d)
    ensemble = None
    if "ensemble" in legs_wanted:
        from paper_2007_10411_amd.jfnk import Batch
        log("one mixed step of the 64-instance heat-island ensemble")
        eprobs = I.heat_island_ensemble(64, seed=0)
        bt = Batch(eprobs, max_m=30)
        erows = bt.tune()
        un_e = bt.pack([I.rest_state(p) for p in eprobs])
        eopts = dict(sweeps=args.pc_sweeps, ortho=args.ortho)
        ens_ms = {}
        for mode, graph in (("graph", True), ("host", False)):
            ue = un_e.clone()
            bt.newton_step(un_e, ue, use_graph=graph, **eopts)   # untimed: first launches, graph capture
            ue = un_e.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eres = bt.newton_step(un_e, ue, use_graph=graph, **eopts)
            torch.cuda.synchronize()
            ens_ms[mode] = (time.perf_counter() - t0) * 1e3
        its = [r.gmres_iters_total for r in eres]
        ensemble = {"instances": len(eprobs), "points": int(sum(p.npts for p in eprobs)),
                    "ms_per_step": ens_ms["graph"], "ms_per_step_host_decided": ens_ms["host"],
                    "converged": all(r.converged for r in eres),
                    "gmres_iters_per_instance": [min(its), max(its)], "gmres_iters_total": sum(its),
                    "pc_sweeps": args.pc_sweeps, "ortho": args.ortho, "launch_shapes": erows,
                    "cycle": "one captured HIP graph per restart cycle, decisions on the device"}
        del bt, un_e, ue
        torch.cuda.empty_cache()

    T = legs["mixed"]
    tm = T["tm"]

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
               "pc": f"k3_pc_diag<float> + {args.pc_sweeps} x k3m_pc_sweep<float> (physics preconditioner)",
               "jv": JV3_KERNEL + " (stable finite-difference Jv, FP32)",
               "residual": RES3_KERNEL + " (FP64 residual)"}
    traffic_name = {"arnoldi": "arnoldi_f32_counters_thermal_3d_256x256x128",
                    "pc": "pc_f32_counters_thermal_3d_256x256x128",
                    "jv": "jv_f32_counters_thermal_3d_256x256x128",
                    "residual": "residual_f64_counters_thermal_3d_256x256x128"}
    dominant = max(("arnoldi", "jv", "pc"), key=lambda k: tm[k][0])
    jv_ms, jv_launches, _ = tm["jv"]
    value = npts * jv_launches / (jv_ms / 1e3) / 1e9 if jv_ms > 0 else 0.0
    leg_summary = {k: per_step(v, npts) for k, v in legs.items()}
    mixed_ms = leg_summary["mixed"]["ms_per_step"]
    out = {
        "metric": "Gpoint-residuals/s (Jv) and ms per implicit step at 1e-8 Newton tol, plain vs learned",
        "value": value,
        "unit": "Gpoint-residuals/s",
        "n_gpus": 1,
        "steps": steps["mixed"],
        "warmup": args.warmup,
        "ms_per_step": mixed_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 Krylov/Jv, f64 Newton",
        "data": "synthetic",
        "config": {
            "workload": f"3D neutral dry thermal 256x256x128 (20x20x10 km, +2 K bubble r=2 km at (10,10,2) km, "
                        f"dt={prob.dt} s, Smagorinsky, free-slip), mixed-precision JFNK with the physics-based "
                        f"preconditioner (field-block diagonal, {args.pc_sweeps} Jacobi sweeps): FGMRES(30) "
                        f"with the {args.ortho} Arnoldi step, Newton rtol 1e-8",
            "grid": [prob.nx, prob.ny, prob.nz],
            "pc_sweeps": args.pc_sweeps,
            "ortho": args.ortho,
            "timed_leg": "mixed",
            "value_definition": "grid points x Jv evaluations / summed Jv kernel time (HIP events) of the timed leg",
            "jv_wall_gpts": npts * jv_launches / T["wall"] / 1e9 * len(T["infos"]) / len(T["infos_instrumented"]),
            "legs": leg_summary,
            "plain_ms_over_mixed_ms": (leg_summary["plain"]["ms_per_step"] / mixed_ms if "plain" in legs else None),
            "plain_ms_over_learned_ms": (leg_summary["plain"]["ms_per_step"] / leg_summary["learned"]["ms_per_step"]
                                         if "plain" in legs and "learned" in legs else None),
            "mixed_vs_fp64": mixed_vs_fp64,
            "training_3d": train_info,
            "learned_error": learned_error,
            "legs_2d": legs_2d,
            "learned_256x128": small,
            "ensemble_64_heat_island": ensemble,
            "kernel_ms_per_step": {k: v[0] / steps["mixed"] for k, v in tm.items()},
            "launch_shapes": shapes,
        },
        "roofline": roof("mixed", dominant, kernels[dominant], traffic=counter_traffic(traffic_name[dominant])),
        "roofline_jv": roof("mixed", "jv", kernels["jv"], traffic=counter_traffic(traffic_name["jv"])),
        "roofline_pc": roof("mixed", "pc", kernels["pc"], traffic=counter_traffic(traffic_name["pc"])),
    }
    # the 3D Jv against the vector-ALU issue rate: VALU lane operations per launch from
    # the committed SQ_INSTS_VALU counter summary (wave instructions x 64 lanes)
    ops = counter_value("jv3d_f32_sq_counters_256x256x128", "valu_lane_ops_per_launch")
    if ops is not None:
        rj = out["roofline_jv"]
        alu = ops / (rj["avg_launch_us"] * 1e-6) / 1e12
        rj["valu"] = {"bound": "alu", "achieved": alu, "peak": VALU_PEAK_TLANEOPS, "unit": "T lane-ops/s",
                      "frac": alu / VALU_PEAK_TLANEOPS, "lane_ops_per_launch": ops}
    if "learned" in legs and legs["learned"]["tm"]["net"][1] > 0:
        out["roofline_net"] = roof("learned", "net", "k3_conv_march x4 (BF16 3x3x3 conv layers of the learned PC, z-marching)",
                                   "mfma")
    if not args.no_micro:
        del legs
        torch.cuda.empty_cache()
        log("kernel micro-benchmark (3D 256x256x128, 2D 8192x8192)")
        micro = kernel_micro(torch, I, L, Context, args.micro_reps, parse_shapes(args.micro_pin),
                             args.micro_cases.split(","))
        out["kernel_micro"] = micro
    if not args.no_cpu:
        log(f"cpu baseline ({args.cpu_seconds} s per process)")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
