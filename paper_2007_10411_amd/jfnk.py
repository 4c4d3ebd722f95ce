"""Python view of the JFNK C ABI with the same entry-point names.

Arrays are torch CUDA (HIP) tensors of shape ``(n_f, nz, ny, nx)`` (or any shape
with that many contiguous elements); torch supplies device memory and the
stream.  Argument marshalling only: every step runs in ``libjfnk.so``.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib as L

DTYPES = {"f64": L.F64, "f32": L.F32}
PCS = {"none": L.PC_NONE, "physics": L.PC_PHYSICS, "learned": L.PC_LEARNED}
JVS = {"stable": L.JV_STABLE, "literal": L.JV_LITERAL, "analytic": L.JV_ANALYTIC}
ORTHO = {"cgs2": L.ORTHO_CGS2, "one_reduction": L.ORTHO_ONE_REDUCTION}


def _torch():
    import torch
    return torch


def _dcode(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return L.F64
    if t.dtype == torch.float32:
        return L.F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("arrays must be contiguous device tensors")
    return C.c_void_p(t.data_ptr())


@dataclass
class GmresResult:
    iters: int
    restarts: int
    converged: bool
    res0: float
    res_est: float
    H: np.ndarray = None
    fallback: bool = False
    res_true: float = -1.0


@dataclass
class NewtonResult:
    newton_iters: int
    gmres_iters_total: int
    converged: bool
    res0: float
    res_final: float
    fallbacks: int = 0


def jv_noalloc(prob, u, v, out, mode="stable", eps=0.0, stream=None):
    """``jfnk_jv_noalloc``: Jv of ``prob`` without a context; no device memory is
    allocated (the library's fixed per-GPU scratch array holds the background
    profiles and reductions)."""
    torch = _torch()
    lib = L.load()
    n = prob.n
    for t in (u, v, out):
        if t.numel() != n:
            raise ValueError(f"expected {n} elements, got {t.numel()}")
    s = stream if stream is not None else torch.cuda.current_stream()
    ps = L.problem_struct(prob)
    L.check(lib.jfnk_jv_noalloc(C.byref(ps), _dcode(u), JVS[mode], _ptr(u), _ptr(v), float(eps), _ptr(out),
                                C.c_void_p(s.cuda_stream)), "jfnk_jv_noalloc", soft_ok=False)
    return out


class Context:
    """One problem on the current device (``jfnk_create`` / ``jfnk_destroy``)."""

    def __init__(self, prob, max_m: int = 30, stream=None):
        torch = _torch()
        self.lib = L.load()
        self.prob = prob
        self.n = prob.n
        s = stream if stream is not None else torch.cuda.current_stream()
        self._stream = s
        h = C.c_void_p()
        ps = L.problem_struct(prob)
        L.check(self.lib.jfnk_create(C.byref(ps), int(max_m), C.c_void_p(s.cuda_stream), C.byref(h)),
                "jfnk_create", soft_ok=False)
        self.h = h
        self.max_m = max_m

    def close(self):
        if getattr(self, "h", None):
            self.lib.jfnk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_size(self, *ts):
        for t in ts:
            if t is not None and t.numel() != self.n:
                raise ValueError(f"expected {self.n} elements, got {t.numel()}")

    # -- operators ------------------------------------------------------------
    def rhs(self, u_n, f):
        self._check_size(u_n, f)
        L.check(self.lib.jfnk_rhs(self.h, _ptr(u_n), _ptr(f)), "jfnk_rhs", soft_ok=False)
        return f

    def residual(self, u, f, R):
        self._check_size(u, f, R)
        L.check(self.lib.jfnk_residual(self.h, _ptr(u), _ptr(f), _ptr(R)), "jfnk_residual", soft_ok=False)
        return R

    def apply_F(self, u, out, what=0, f=None):
        self._check_size(u, f, out)
        L.check(self.lib.jfnk_apply_F(self.h, _dcode(u), int(what), _ptr(u), _ptr(f), _ptr(out)),
                "jfnk_apply_F", soft_ok=False)
        return out

    def jv(self, u, v, out, mode="stable", eps=0.0):
        self._check_size(u, v, out)
        L.check(self.lib.jfnk_jv(self.h, _dcode(u), JVS[mode], _ptr(u), _ptr(v), float(eps), _ptr(out)),
                "jfnk_jv", soft_ok=False)
        return out

    def precond_apply(self, u, r, z, pc="physics", sweeps=2):
        self._check_size(u, r, z)
        L.check(self.lib.jfnk_precond_apply(self.h, PCS[pc], _dcode(u), _ptr(u), _ptr(r), _ptr(z), int(sweeps)),
                "jfnk_precond_apply", soft_ok=False)
        return z

    def gmres(self, u, b, x, m=30, max_restarts=20, tol=1e-6, pc="physics", jv="stable", sweeps=2,
              max_iters=0, want_H=False, ortho="cgs2", judge=True, fallback=True):
        """judge=False runs a learned-preconditioner solve without the physics-based
        preconditioner's judgement (jfnk_gmres_opts.no_judge = 1); with
        fallback=False as well, its result is returned even when it has not
        converged (no_judge = 2)."""
        self._check_size(u, b, x)
        nj = 0 if judge else (1 if fallback else 2)
        o = L.GmresOpts(m=m, max_restarts=max_restarts, tol=tol, pc=PCS[pc], jv=JVS[jv], sweeps=sweeps,
                        max_iters=max_iters, ortho=ORTHO[ortho], no_judge=nj)
        info = L.GmresInfo()
        Hbuf = None
        if want_H:
            Hbuf = (C.c_double * ((m + 1) * m))()
            info.h_out = C.cast(Hbuf, C.POINTER(C.c_double))
        L.check(self.lib.jfnk_gmres(self.h, _dcode(u), _ptr(u), _ptr(b), _ptr(x), C.byref(o), C.byref(info)),
                "jfnk_gmres")
        H = np.ctypeslib.as_array(Hbuf).reshape(m + 1, m).copy() if want_H else None
        return GmresResult(info.iters, info.restarts, bool(info.converged), info.res0, info.res_est, H,
                           bool(info.fallback), info.res_true)

    def newton_step(self, u_n, u_np1, rtol=1e-8, atol_factor=1e-13, max_newton=20, inner="f64",
                    m=30, max_restarts=20, pc="physics", jv="stable", sweeps=2, forcing="ew", eta=1e-2,
                    eta_floor=0.0, record=None, record_krylov=False, ortho="cgs2", judge=True):
        """record: optional (R, DU, count) with R, DU float32 device tensors of
        shape (cap, n) receiving the Newton linear systems; count is a one-element
        list updated in place.  ortho: "cgs2" or "one_reduction" (jfnk_ortho).
        judge=False: learned-preconditioner solves run unjudged (no_judge)."""
        self._check_size(u_n, u_np1)
        gm = L.GmresOpts(m=m, max_restarts=max_restarts, tol=0.0, pc=PCS[pc], jv=JVS[jv], sweeps=sweeps,
                         max_iters=0, ortho=ORTHO[ortho], no_judge=0 if judge else 1)
        o = L.NewtonOpts(rtol=rtol, atol_factor=atol_factor, max_newton=max_newton, inner=DTYPES[inner],
                         gm=gm, forcing=0 if forcing == "ew" else 1, eta=eta, eta_floor=eta_floor)
        cnt = C.c_int32(0)
        if record is not None:
            Rr, Dr, count = record
            cnt.value = count[0]
            o.rec_r = Rr.data_ptr()
            o.rec_du = Dr.data_ptr()
            o.rec_cap = Rr.shape[0]
            o.rec_count = C.pointer(cnt)
            o.rec_krylov = 1 if record_krylov else 0
        info = L.NewtonInfo()
        L.check(self.lib.jfnk_newton_step(self.h, _ptr(u_n), _ptr(u_np1), C.byref(o), C.byref(info)),
                "jfnk_newton_step")
        if record is not None:
            record[2][0] = cnt.value
        return NewtonResult(info.newton_iters, info.gmres_iters_total, bool(info.converged), info.res0,
                            info.res_final, info.fallbacks)

    def nlpc_residual(self, u, f, out, sweeps=2):
        """out = R~(u) = P^{-1}(u) R(u) (FP64)."""
        self._check_size(u, f, out)
        L.check(self.lib.jfnk_nlpc_residual(self.h, _ptr(u), _ptr(f), _ptr(out), int(sweeps)),
                "jfnk_nlpc_residual", soft_ok=False)
        return out

    def nlpc_step(self, u_n, u_np1, method="newton", rtol=1e-8, atol_factor=1e-13, max_iter=20, m=30,
                  max_restarts=20, sweeps=2, forcing="ew", eta=1e-2, eta_floor=0.0):
        """One step on the nonlinearly preconditioned system: method "newton"
        (Newton-Krylov on R~) or "fixed_point" (u <- u - R~(u))."""
        self._check_size(u_n, u_np1)
        gm = L.GmresOpts(m=m, max_restarts=max_restarts, tol=0.0, pc=PCS["none"], jv=L.JV_STABLE,
                         sweeps=sweeps, max_iters=0)
        o = L.NewtonOpts(rtol=rtol, atol_factor=atol_factor, max_newton=max_iter, inner=L.F64, gm=gm,
                         forcing=0 if forcing == "ew" else 1, eta=eta, eta_floor=eta_floor)
        info = L.NewtonInfo()
        code = {"fixed_point": 0, "newton": 1}[method]
        L.check(self.lib.jfnk_nlpc_step(self.h, _ptr(u_n), _ptr(u_np1), C.byref(o), code, C.byref(info)),
                "jfnk_nlpc_step")
        return NewtonResult(info.newton_iters, info.gmres_iters_total, bool(info.converged), info.res0,
                            info.res_final, info.fallbacks)

    def norm(self, x):
        out = C.c_double()
        L.check(self.lib.jfnk_norm(self.h, _dcode(x), _ptr(x), x.numel(), C.byref(out)), "jfnk_norm",
                soft_ok=False)
        return out.value

    # -- learned preconditioner -----------------------------------------------
    def net_init(self, dilations=(1, 1, 1, 1)):
        n = C.c_int64()
        d = (C.c_int32 * 4)(*[int(x) for x in dilations])
        L.check(self.lib.jfnk_net_init(self.h, d, C.byref(n)), "jfnk_net_init", soft_ok=False)
        self.n_params = n.value
        self.dilations = tuple(int(x) for x in dilations)
        return n.value

    def net_set_loss(self, kind):
        """kind: "solution" (||z - du||^2 / ||du||^2) or "rest_jacobian"
        (||J0 (z - du)||^2 / ||J0 du||^2, J0 the Jacobian at rest)."""
        code = {"solution": L.NET_LOSS_SOLUTION, "rest_jacobian": L.NET_LOSS_REST_JACOBIAN}[kind]
        L.check(self.lib.jfnk_net_set_loss(self.h, code), "jfnk_net_set_loss", soft_ok=False)

    def net_set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        L.check(self.lib.jfnk_net_set_params(self.h, th.ctypes.data_as(C.c_void_p), th.size),
                "jfnk_net_set_params", soft_ok=False)

    def net_get_params(self):
        th = np.empty(self.n_params, dtype=np.float32)
        L.check(self.lib.jfnk_net_get_params(self.h, th.ctypes.data_as(C.c_void_p), th.size),
                "jfnk_net_get_params", soft_ok=False)
        return th

    def net_apply(self, r, z, bf16=True):
        self._check_size(r, z)
        L.check(self.lib.jfnk_net_apply(self.h, 1 if bf16 else 0, _ptr(r), _ptr(z)), "jfnk_net_apply",
                soft_ok=False)
        return z

    def net_loss_grad(self, R, DU, want_grad=True):
        """R, DU: float32 device tensors holding `batch` state vectors back to back."""
        batch = R.numel() // self.n
        loss = C.c_double()
        g = np.empty(self.n_params, dtype=np.float32) if want_grad else None
        L.check(self.lib.jfnk_net_loss_grad(self.h, _ptr(R), _ptr(DU), batch, C.byref(loss),
                                            g.ctypes.data_as(C.c_void_p) if want_grad else None),
                "jfnk_net_loss_grad", soft_ok=False)
        return loss.value, g

    def net_train_step(self, R, DU, lr, crop=None):
        """One Adam step on the pairs (R, DU); crop = (nx, ny, nz) when they are
        crops of that size rather than vectors of the context's grid."""
        nvec = self.n if crop is None else self.prob.nf * int(crop[0]) * int(crop[1]) * int(crop[2])
        batch = R.numel() // nvec
        loss = C.c_double()
        cd = None if crop is None else (C.c_int32 * 3)(*[int(x) for x in crop])
        L.check(self.lib.jfnk_net_train_step(self.h, _ptr(R), _ptr(DU), batch, cd, float(lr), C.byref(loss)),
                "jfnk_net_train_step", soft_ok=False)
        return loss.value

    def tune(self):
        """Autotune the stencil tile shapes; returns the chosen tile heights."""
        rows = (C.c_int32 * 6)()
        L.check(self.lib.jfnk_tune(self.h, rows), "jfnk_tune", soft_ok=False)
        keys = ["f64_residual", "f32_residual", "f64_jv", "f32_jv", "f64_pc_sweep", "f32_pc_sweep"]
        return dict(zip(keys, list(rows)))

    def set_variant(self, stage, dtype, variant):
        """Pin a stencil launch shape: stage "residual" / "jv" / "pc_sweep",
        dtype "f64" / "f32", variant 0-2 (tiles 64 x 4/8/16) or 3-5 (row marching
        over 32/64/256 rows; residual and Jv); for 3D contexts the FP32 Jv only,
        variant 7 (one z-marching launch) or 6 (two launches)."""
        st = {"residual": 0, "jv": 1, "pc_sweep": 2}[stage]
        dt = {"f64": L.F64, "f32": L.F32}[dtype]
        L.check(self.lib.jfnk_set_variant(self.h, st, dt, int(variant)), "jfnk_set_variant", soft_ok=False)

    # -- timing ----------------------------------------------------------------
    def timing(self, on):
        """Start (clearing the counters) or stop HIP-event timing: True records
        every kernel class, an int is a bit mask of classes (bit k: class k)."""
        mask = -1 if on is True else (0 if on is False else int(on))
        L.check(self.lib.jfnk_timing_enable(self.h, mask), "jfnk_timing_enable", soft_ok=False)

    def timing_read(self, cls):
        """(total ms, launches, algorithmic bytes) of one kernel class."""
        ms = C.c_double()
        cnt = C.c_int64()
        by = C.c_double()
        L.check(self.lib.jfnk_timing_read(self.h, int(cls), C.byref(ms), C.byref(cnt), C.byref(by)),
                "jfnk_timing_read", soft_ok=False)
        return ms.value, cnt.value, by.value


class Batch:
    """Ensemble of independent 2D problems solved together (``jfnk_batch_*``).
    Batch vectors are the instances' state vectors back to back."""

    def __init__(self, probs, max_m: int = 30, stream=None):
        torch = _torch()
        self.lib = L.load()
        self.probs = list(probs)
        arr = (L.Problem * len(self.probs))(*[L.problem_struct(p) for p in self.probs])
        s = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        L.check(self.lib.jfnk_batch_create(arr, len(self.probs), int(max_m), C.c_void_p(s.cuda_stream), C.byref(h)),
                "jfnk_batch_create", soft_ok=False)
        self.h = h
        tot = C.c_int64()
        offs = (C.c_int64 * (len(self.probs) + 1))()
        L.check(self.lib.jfnk_batch_size(self.h, C.byref(tot), offs), "jfnk_batch_size", soft_ok=False)
        self.n = tot.value
        self.offsets = list(offs)

    def close(self):
        if getattr(self, "h", None):
            self.lib.jfnk_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, states):
        """List of (n_f, nz, 1, nx) numpy states -> one FP64 device vector."""
        torch = _torch()
        flat = np.concatenate([np.ascontiguousarray(s, dtype=np.float64).ravel() for s in states])
        return torch.from_numpy(flat).cuda()

    def unpack(self, t):
        h = t.detach().double().cpu().numpy()
        return [h[self.offsets[i]:self.offsets[i + 1]].reshape(p.shape) for i, p in enumerate(self.probs)]

    def apply_F(self, u, out, what=0, f=None):
        L.check(self.lib.jfnk_batch_apply_F(self.h, int(what), _ptr(u), _ptr(f), _ptr(out)), "jfnk_batch_apply_F",
                soft_ok=False)
        return out

    def tune(self):
        rows = (C.c_int32 * 3)()
        L.check(self.lib.jfnk_batch_tune(self.h, rows), "jfnk_batch_tune", soft_ok=False)
        return dict(zip(["f64_residual", "f32_jv", "f32_pc_sweep"], list(rows)))

    def newton_step(self, u_n, u_np1, rtol=1e-8, atol_factor=1e-13, max_newton=20, m=30, max_restarts=20,
                    pc="physics", sweeps=2, forcing="ew", eta=1e-2, eta_floor=1e-4, ortho="cgs2", use_graph=False):
        """use_graph: each restart cycle as one captured HIP graph with the
        per-instance decisions on the device (jfnk_batch_newton_step)."""
        gm = L.GmresOpts(m=m, max_restarts=max_restarts, tol=0.0, pc=PCS[pc], jv=L.JV_STABLE, sweeps=sweeps,
                         max_iters=0, ortho=ORTHO[ortho])
        o = L.NewtonOpts(rtol=rtol, atol_factor=atol_factor, max_newton=max_newton, inner=L.F32, gm=gm,
                         forcing=0 if forcing == "ew" else 1, eta=eta, eta_floor=eta_floor)
        infos = (L.NewtonInfo * len(self.probs))()
        L.check(self.lib.jfnk_batch_newton_step(self.h, _ptr(u_n), _ptr(u_np1), C.byref(o), infos,
                                                1 if use_graph else 0), "jfnk_batch_newton_step")
        return [NewtonResult(i.newton_iters, i.gmres_iters_total, bool(i.converged), i.res0, i.res_final,
                             i.fallbacks) for i in infos]
