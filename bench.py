"""Benchmark of the JFNK hot path on one MI355X.

Workload (default): the 2D dry thermal in a stably stratified atmosphere,
1024 x 512 grid over 20 x 10 km, N = 0.01 1/s, +2 K bubble, dt = 1 s,
Smagorinsky closure.  One step = one trapezoidal implicit step solved by inexact
Newton to a relative residual of 1e-8 (FP64 outer residual / update / norms),
with GMRES(30) right-preconditioned by the physics-based field-block
preconditioner.  The timed leg runs the mixed form (FP32 Krylov and Jv inside the
FP64 Newton); the plain FP64 form is timed beside it for the ms/step comparison.

Printed JSON line:
  value          whole-job Jv throughput: grid points x Jv evaluations during the
                 timed steps / wall time of those steps [Gpoint-residuals/s]
  ms_per_step    wall time per implicit step of the timed (mixed) leg
  roofline       the Jv kernel: algorithmic bytes 3 n_f w per point and launch
                 over its average HIP-event duration, against 8 TB/s HBM
  cpu_baseline   the FP64 oracle on a bounded sample of the same workload
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

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--nz", type=int, default=512)
    return ap.parse_args()


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


def cpu_baseline(prob, U0, seconds):
    """Oracle (FP64 numpy) on a bounded sample of the same workload: GMRES
    iterations of the first Newton iteration of the first step (physics
    preconditioner, stable-FD Jv, CGS2 Arnoldi), stopped after `seconds`."""
    import numpy as np
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

        pc = lambda r: PC.physics_pc(prob, U0, r, 2, fr)
        try:
            K.fgmres(mv, pc, -R, m=30, tol=1e-12, max_iters=10 ** 6, true_residual=False)
        except Stop:
            pass
        el = time.perf_counter() - t0
    gpts = prob.npts * calls[0] / el / 1e9
    return {"value": gpts, "unit": "Gpoint-residuals/s", "cores": 1, "kind": "oracle",
            "sample": f"{calls[0]} FP64 GMRES iterations (PC + Jv + CGS2) of the first Newton "
                      f"iteration of step 1 on the same {prob.nx}x{prob.nz} grid, {el:.1f} s, 1 thread"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the solver would shard).", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2007_10411_amd import _lib as L
    from paper_2007_10411_amd import inputs as I
    from paper_2007_10411_amd.jfnk import Context

    torch.cuda.set_device(0)
    prob = I.thermal_stable_2d(args.nx, args.nz)
    U0 = I.bubble_state(prob)
    ctx = Context(prob, max_m=30)
    mixed = dict(rtol=1e-8, inner="f32", eta_floor=1e-4, m=30, max_restarts=20, pc="physics")
    plain = dict(rtol=1e-8, inner="f64", m=30, max_restarts=20, pc="physics")

    u = torch.from_numpy(U0).cuda()
    print(f"[bench] warmup {args.warmup} mixed steps", file=sys.stderr, flush=True)
    run_steps(ctx, u, args.warmup, torch, **mixed)
    torch.cuda.synchronize()
    ctx.timing(True)
    print(f"[bench] timing {args.steps} mixed steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = run_steps(ctx, u, args.steps, torch, **mixed)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cls = {"jv": L.KC_JV, "pc": L.KC_PC, "arnoldi": L.KC_ARNOLDI, "residual": L.KC_RESIDUAL}
    tm = {k: ctx.timing_read(v) for k, v in cls.items()}      # (ms, launches, algorithmic bytes)
    ctx.timing(False)

    # plain FP64 leg from the same state, for the ms/step comparison
    print(f"[bench] timing {args.plain_steps} plain FP64 steps", file=sys.stderr, flush=True)
    u64 = u.clone()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pinfos = run_steps(ctx, u64, args.plain_steps, torch, **plain)
    torch.cuda.synchronize()
    plain_wall = time.perf_counter() - t1

    npts = prob.npts
    gm_total = sum(r.gmres_iters_total for r in infos)
    jv_ms, jv_launches, jv_bytes_total = tm["jv"]
    # Jv evaluations: one per GMRES iteration plus one per restart (true residual)
    value = npts * jv_launches / wall / 1e9

    def roof(name, kernel):
        ms, launches, nbytes = tm[name]
        achieved = nbytes / (ms / 1e3) / 1e9 if ms > 0 else 0.0
        return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "bytes_per_launch": nbytes / max(launches, 1), "avg_launch_us": ms / max(launches, 1) * 1e3,
                "launches": launches}

    kernels = {"arnoldi": "k_cgs<float> x3 + k_cgs_finish x3 (CGS2 passes of one GMRES iteration)",
               "pc": "k_pc_diag_2d<float> + k_pc_sweep_2d<float,64,8> (physics preconditioner)",
               "jv": "k_jv_2d<float,64,8> (stable finite-difference Jv)"}
    dominant = max(kernels, key=lambda k: tm[k][0])
    out = {
        "metric": "Gpoint-residuals/s (Jv) and ms per implicit step at 1e-8 Newton tol, plain vs learned",
        "value": value,
        "unit": "Gpoint-residuals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 Krylov/Jv, f64 Newton",
        "data": "synthetic",
        "config": {
            "workload": f"stable 2D dry thermal {prob.nx}x{prob.nz} (20x10 km, N=0.01/s, +2 K bubble, "
                        f"dt={prob.dt} s, Smagorinsky), mixed FP32-inner/FP64-outer JFNK, physics PC, "
                        f"GMRES(30), Newton rtol 1e-8",
            "grid": [prob.nx, prob.nz],
            "newton_iters_per_step": sum(r.newton_iters for r in infos) / len(infos),
            "gmres_iters_per_step": gm_total / len(infos),
            "plain_f64_ms_per_step": plain_wall / args.plain_steps * 1e3,
            "plain_f64_gmres_iters_per_step": sum(r.gmres_iters_total for r in pinfos) / len(pinfos),
            "jv_kernel_gpts": npts * jv_launches / (jv_ms / 1e3) / 1e9 if jv_ms > 0 else 0.0,
            "kernel_ms_per_step": {k: v[0] / args.steps for k, v in tm.items()},
        },
        "roofline": roof(dominant, kernels[dominant]),
        "roofline_jv": roof("jv", kernels["jv"]),
    }
    if not args.no_cpu:
        print(f"[bench] cpu baseline ({args.cpu_seconds} s)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, U0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
