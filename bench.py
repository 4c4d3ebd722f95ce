"""Benchmark of the JFNK hot path on one MI355X.

Workload: the 2D dry thermal in a stably stratified atmosphere, 1024 x 512 grid
over 20 x 10 km, N = 0.01 1/s, +2 K bubble, dt = 1 s, Smagorinsky closure.  One
step = one trapezoidal implicit step solved by inexact Newton (Eisenstat-Walker
forcing) to a relative residual of 1e-8, FGMRES(30).

Legs, all from the same state after the warm-up steps:
  learned   FP32 Krylov / Jv, learned BF16-MFMA right preconditioner, FP64 Newton
            (the network is trained first on pairs the solver generates on this
            workload; training time is reported, not timed with the steps)
  mixed     FP32 Krylov / Jv, physics-based preconditioner, FP64 Newton
  plain     FP64 everywhere, physics-based preconditioner

Printed JSON line (the timed leg is `learned`, or `mixed` with --no-learned):
  value          whole-job Jv throughput: grid points x Jv evaluations during the
                 timed steps / wall time of those steps [Gpoint-residuals/s]
  ms_per_step    wall time per implicit step of the timed leg
  roofline       dominant kernel class of the timed leg (algorithmic bytes over
                 summed HIP-event time) against 8 TB/s HBM; roofline_jv and
                 roofline_net for the Jv kernel and the network (vs 2.5 PFLOP/s BF16)
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
BF16_PEAK_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--train-iters", type=int, default=1500)
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--nz", type=int, default=512)
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


def timed_leg(ctx, u0, k, torch, L, **opts):
    u = u0.clone()
    torch.cuda.synchronize()
    ctx.timing(True)
    t0 = time.perf_counter()
    infos = run_steps(ctx, u, k, torch, **opts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cls = {"jv": L.KC_JV, "pc": L.KC_PC, "arnoldi": L.KC_ARNOLDI, "residual": L.KC_RESIDUAL, "net": L.KC_NET}
    tm = {name: ctx.timing_read(c) for name, c in cls.items()}    # (ms, launches, bytes or flops)
    ctx.timing(False)
    return {"wall": wall, "infos": infos, "tm": tm, "u": u}


def cpu_baseline(prob, U0, seconds):
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
    import numpy as np
    import torch

    from paper_2007_10411_amd import _lib as L
    from paper_2007_10411_amd import inputs as I
    from paper_2007_10411_amd import learned as LRN
    from paper_2007_10411_amd.jfnk import Context

    torch.cuda.set_device(0)
    prob = I.thermal_stable_2d(args.nx, args.nz)
    U0 = I.bubble_state(prob)
    ctx = Context(prob, max_m=30)
    common = dict(rtol=1e-8, m=30, max_restarts=20)
    mixed = dict(common, inner="f32", eta_floor=1e-4, pc="physics")
    plain = dict(common, inner="f64", pc="physics")
    learned = dict(common, inner="f32", eta_floor=1e-4, pc="learned")

    u = torch.from_numpy(U0).cuda()
    log(f"warmup {args.warmup} mixed steps")
    run_steps(ctx, u, args.warmup, torch, **mixed)
    train_info = None
    if not args.no_learned:
        log("recording solver pairs and training the learned preconditioner")
        t0 = time.perf_counter()
        R, DU, u = LRN.collect_pairs(ctx, u, steps=2, cap=96)
        t1 = time.perf_counter()
        theta, losses = LRN.train_mixed(ctx, R, DU, u, iters=args.train_iters, lr=2e-3, batch=8)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        train_info = {"pairs": int(R.shape[0]), "collect_s": t1 - t0, "train_s": t2 - t1,
                      "adam_steps": args.train_iters, "loss_first": losses[0],
                      "loss_last": float(np.mean(losses[-20:]))}
        del R, DU
        torch.cuda.empty_cache()
    legs = {}
    if not args.no_learned:
        log(f"timing {args.steps} learned steps")
        legs["learned"] = timed_leg(ctx, u, args.steps, torch, L, **learned)
    log(f"timing {args.steps} mixed steps")
    legs["mixed"] = timed_leg(ctx, u, args.steps, torch, L, **mixed)
    log(f"timing {args.plain_steps} plain FP64 steps")
    legs["plain"] = timed_leg(ctx, u, args.plain_steps, torch, L, **plain)
    main_leg = "learned" if "learned" in legs else "mixed"
    T = legs[main_leg]
    tm = T["tm"]
    npts = prob.npts

    def per_step(leg):
        k = len(legs[leg]["infos"])
        return {"ms_per_step": legs[leg]["wall"] / k * 1e3,
                "newton_iters_per_step": sum(r.newton_iters for r in legs[leg]["infos"]) / k,
                "gmres_iters_per_step": sum(r.gmres_iters_total for r in legs[leg]["infos"]) / k,
                "fallbacks": sum(r.fallbacks for r in legs[leg]["infos"])}

    def roof(name, kernel, bound="hbm"):
        ms, launches, amount = tm[name]
        rate = amount / (ms / 1e3) if ms > 0 else 0.0
        if bound == "mfma":
            achieved = rate / 1e12
            return {"kernel": kernel, "bound": "mfma", "achieved": achieved, "peak": BF16_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved / BF16_PEAK_TFLOPS, "traffic": None,
                    "flops_per_launch": amount / max(launches, 1), "avg_launch_us": ms / max(launches, 1) * 1e3,
                    "launches": launches}
        achieved = rate / 1e9
        return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "bytes_per_launch": amount / max(launches, 1), "avg_launch_us": ms / max(launches, 1) * 1e3,
                "launches": launches}

    kernels = {"arnoldi": "k_cgs<float> x3 + k_cgs_finish x3 (CGS2 passes of one GMRES iteration)",
               "pc": "k_pc_diag_2d<float> + k_pc_sweep_2d<float,64,8> (physics preconditioner)",
               "jv": "k_jv_2d<float,64,8> (stable finite-difference Jv)"}
    dominant = max(kernels, key=lambda k: tm[k][0])
    jv_ms, jv_launches, _ = tm["jv"]
    value = npts * jv_launches / T["wall"] / 1e9
    out = {
        "metric": "Gpoint-residuals/s (Jv) and ms per implicit step at 1e-8 Newton tol, plain vs learned",
        "value": value,
        "unit": "Gpoint-residuals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32 Krylov/Jv, bf16 MFMA learned PC, f64 Newton" if main_leg == "learned"
                  else "f32 Krylov/Jv, f64 Newton"),
        "data": "synthetic",
        "config": {
            "workload": f"stable 2D dry thermal {prob.nx}x{prob.nz} (20x10 km, N=0.01/s, +2 K bubble, "
                        f"dt={prob.dt} s, Smagorinsky), {main_leg} JFNK: FGMRES(30), Newton rtol 1e-8",
            "grid": [prob.nx, prob.nz],
            "timed_leg": main_leg,
            "legs": {k: per_step(k) for k in legs},
            "training": train_info,
            "jv_kernel_gpts": npts * jv_launches / (jv_ms / 1e3) / 1e9 if jv_ms > 0 else 0.0,
            "kernel_ms_per_step": {k: v[0] / args.steps for k, v in tm.items()},
        },
        "roofline": roof(dominant, kernels[dominant]),
        "roofline_jv": roof("jv", kernels["jv"]),
    }
    if tm["net"][1] > 0:
        out["roofline_net"] = roof("net", "k_conv_mfma x4 (BF16 3x3 conv layers of the learned PC)", "mfma")
    if not args.no_cpu:
        log(f"cpu baseline ({args.cpu_seconds} s)")
        out["cpu_baseline"] = cpu_baseline(prob, U0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
