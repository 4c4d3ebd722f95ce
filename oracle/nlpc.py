"""Physics-based nonlinear preconditioning (section 2.5.2).

ORACLE - test infrastructure only.  Plain FP64 numpy on top of the model, the
physics-based preconditioner and the GMRES of this package.

The paper's preconditioned nonlinear system

    R~(u) = u - P^{-1}(u) [ f(u^n) - L(u) + P(u) u ]

(reading: the preconditioning operator P(u) acts on u inside the bracket) is
P^{-1}(u) (L(u) - f) = P^{-1}(u) R(u), with P^{-1}(u) the field-block
preconditioner with coefficients frozen at u, applied by Jacobi sweeps.  Its
roots are the roots of R.  Two solvers:

* fixed point      u <- u - R~(u)          (the iteration whose convergence the
                                             paper ties to the eigenvalues of J~)
* Newton-Krylov    J~ du = -R~(u) by GMRES without further preconditioning,
                   J~ v = [R~(u + eps v) - R~(u)] / eps with the usual eps;
                   Eisenstat-Walker forcing on the sequence ||R~(u_k)|| with the
                   safeguard tolerance rtol ||R~(u^0)||.

Both stop on the unpreconditioned residual, ||R(u)|| <= max(rtol ||R(u^n)||,
atol_factor ||2 u^n / dt||), like the plain Newton step.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import krylov as K
from . import model as M
from . import precond as PC


def rtilde(prob, U, f, sweeps=2):
    """R~(u) = P^{-1}(u) R(u)."""
    return PC.physics_pc(prob, U, M.residual(prob, U, f), sweeps)


@dataclass
class NlpcInfo:
    iters: int = 0
    gmres_iters: List[int] = field(default_factory=list)
    res: List[float] = field(default_factory=list)
    converged: bool = False


def _tolerance(prob, Un, f, U, rtol, atol_factor):
    r0 = K._nrm(M.residual(prob, U, f))
    return r0, max(rtol * r0, atol_factor * K._nrm(2.0 * Un / prob.dt))


def fixed_point_step(prob, Un, rtol=1e-8, atol_factor=1e-13, max_iter=200, sweeps=2):
    """One trapezoidal step by the fixed-point iteration u <- u - R~(u)."""
    f = M.rhs(prob, Un)
    U = Un.copy()
    rn, tol = _tolerance(prob, Un, f, U, rtol, atol_factor)
    info = NlpcInfo(res=[rn])
    for k in range(max_iter + 1):
        if rn <= tol:
            info.converged = True
            break
        if k == max_iter or not np.isfinite(rn):
            break
        U = U - rtilde(prob, U, f, sweeps)
        rn = K._nrm(M.residual(prob, U, f))
        info.res.append(rn)
        info.iters = k + 1
    return U, info


def newton_krylov_step(prob, Un, opts: K.NewtonOpts = K.NewtonOpts()):
    """One trapezoidal step by inexact Newton-GMRES on R~ (opts.sweeps Jacobi
    sweeps in P^{-1}; opts.pc is not used: the system is already preconditioned)."""
    f = M.rhs(prob, Un)
    U = Un.copy()
    rn, tol = _tolerance(prob, Un, f, U, opts.rtol, opts.atol_factor)
    info = NlpcInfo(res=[rn])
    Rt = rtilde(prob, U, f, opts.sweeps)
    rt = K._nrm(Rt)
    tol_t = opts.rtol * rt
    rt_prev, eta = rt, 0.5
    for k in range(opts.max_newton + 1):
        if rn <= tol:
            info.converged = True
            break
        if k == opts.max_newton:
            break
        if opts.forcing == "ew":
            eta = K.ew_forcing(k, rt, rt_prev, eta, tol_t)
        else:
            eta = opts.eta
        eta = max(eta, opts.eta_floor)
        Uk, Rtk = U, Rt

        def matvec(v, Uk=Uk, Rtk=Rtk):
            eps = M.fd_eps(prob, Uk, v, opts.eps_mach)
            return (rtilde(prob, Uk + eps * v, f, opts.sweeps) - Rtk) / eps

        du, gi = K.fgmres(matvec, lambda r: r, -Rt, m=opts.m, tol=eta,
                          max_iters=opts.m * opts.max_restarts, ortho=opts.ortho, true_residual=False)
        info.gmres_iters.append(gi.iters)
        U = U + du
        rn = K._nrm(M.residual(prob, U, f))
        info.res.append(rn)
        info.iters = k + 1
        Rt = rtilde(prob, U, f, opts.sweeps)
        rt_prev, rt = rt, K._nrm(Rt)
    return U, info
