"""Restarted (flexible) GMRES with right preconditioning and the inexact
Newton iteration around it (section 2.5.1, equation 8; GMRES of Saad and
Schultz 1986).

ORACLE - test infrastructure only.  Plain FP64 numpy.

* GMRES(m): x0 = 0; Arnoldi by modified Gram-Schmidt or by classical
  Gram-Schmidt applied twice (CGS2); the preconditioned vectors z_j = M^-1 v_j
  are kept (flexible form), x = x0 + Z y.  Givens rotations with
  r = hypot(a, b), c = a/r, s = b/r; y by back substitution.  Stop when the
  least-squares residual |g_{j+1}| <= tol ||b|| or after max_iters iterations;
  restarts continue from the current x with the true residual b - A x.
* Newton: u_0 = u^n (or a given guess); J(u_k) du = -R(u_k) solved to a relative
  tolerance eta_k; full step u_{k+1} = u_k + du; stop when
  ||R(u_k)|| <= max(rtol ||R(u_0)||, atol).  eta_k is the Eisenstat-Walker
  choice 2 (gamma = 0.9, alpha = 2, eta_max = 0.9, eta_0 = 0.5) with the usual
  safeguards: eta_k >= gamma eta_{k-1}^alpha whenever that exceeds 0.1, and
  eta_k >= 0.5 tol / ||R(u_k)|| so the last solve is not over-solved; or a fixed
  eta.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from . import model as M
from . import precond as PC


def _dot(a, b):
    return float(np.dot(a.ravel(), b.ravel()))


def _nrm(a):
    return math.sqrt(_dot(a, a))


@dataclass
class GmresInfo:
    iters: int = 0
    restarts: int = 0
    res0: float = 0.0
    res_est: float = 0.0
    res_true: float = float("nan")
    converged: bool = False
    H: Optional[np.ndarray] = None          # Hessenberg of the last cycle (before rotations)
    history: List[float] = field(default_factory=list)


def fgmres(matvec: Callable, precond: Callable, b: np.ndarray, m: int = 30,
           tol: float = 1e-6, max_iters: int = 600, ortho: str = "cgs2",
           x0: Optional[np.ndarray] = None, true_residual: bool = True):
    x = np.zeros_like(b) if x0 is None else x0.copy()
    info = GmresInfo()
    bnorm = _nrm(b)
    r = b - matvec(x) if x0 is not None else b.copy()
    beta = _nrm(r)
    info.res0 = beta
    info.res_est = beta
    info.history.append(beta)
    if bnorm == 0.0 or beta == 0.0:
        info.converged = True
        info.res_true = beta
        return x, info
    total = 0
    while True:
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        Hraw = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        done = False
        for j in range(m):
            z = precond(V[j])
            Z.append(z)
            w = matvec(z)
            if ortho == "mgs":
                for i in range(j + 1):
                    H[i, j] = _dot(V[i], w)
                    w = w - H[i, j] * V[i]
            else:                                   # classical Gram-Schmidt, twice
                for _ in range(2):
                    h = np.array([_dot(V[i], w) for i in range(j + 1)])
                    for i in range(j + 1):
                        w = w - h[i] * V[i]
                    H[: j + 1, j] += h
            H[j + 1, j] = _nrm(w)
            Hraw[:, j] = H[:, j]
            breakdown = H[j + 1, j] == 0.0
            V.append(w / H[j + 1, j] if not breakdown else w)
            for i in range(j):                      # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            rr = math.hypot(a, bb)
            cs[j], sn[j] = (a / rr, bb / rr) if rr > 0 else (1.0, 0.0)
            H[j, j] = rr
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            total += 1
            info.res_est = abs(g[j + 1])
            info.history.append(info.res_est)
            if info.res_est <= tol * bnorm or breakdown or total >= max_iters:
                done = True
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):              # back substitution
            y[i] = (g[i] - float(np.dot(H[i, i + 1:k], y[i + 1:k]))) / H[i, i]
        for i in range(k):
            x = x + y[i] * Z[i]
        info.H = Hraw[: k + 1, :k]
        info.iters = total
        if done:
            info.converged = info.res_est <= tol * bnorm
            break
        info.restarts += 1
        r = b - matvec(x)
        beta = _nrm(r)
        if beta == 0.0:
            info.converged = True
            break
    if true_residual:
        info.res_true = _nrm(b - matvec(x))
    return x, info


# --------------------------------------------------------------------------- #
# dense reference for tiny grids
# --------------------------------------------------------------------------- #
def dense_jacobian(prob, U, eps=0.0):
    """Columns J e_k of the analytic (eps = 0) Jacobian of R at U."""
    n = U.size
    J = np.zeros((n, n))
    e = np.zeros(n)
    for k in range(n):
        e[:] = 0.0
        e[k] = 1.0
        J[:, k] = M.jv(prob, U, e.reshape(U.shape), eps).ravel()
    return J


# --------------------------------------------------------------------------- #
# Newton
# --------------------------------------------------------------------------- #
@dataclass
class NewtonOpts:
    rtol: float = 1e-8
    atol_factor: float = 1e-13          # atol = atol_factor * ||2 u^n / dt||
    max_newton: int = 20
    m: int = 30
    max_restarts: int = 20
    forcing: str = "ew"                 # "ew" or "fixed"
    eta: float = 1e-2                   # fixed forcing term
    eta_floor: float = 0.0
    pc: str = "physics"                 # "physics" or "none"
    sweeps: int = 2
    jv: str = "stable"                  # "stable", "literal" or "analytic"
    eps_mach: float = 2.0 ** -52
    ortho: str = "cgs2"


@dataclass
class NewtonInfo:
    newton_iters: int = 0
    gmres_iters: List[int] = field(default_factory=list)
    res: List[float] = field(default_factory=list)
    converged: bool = False


def ew_forcing(k, rn, rprev, eta_prev, tol, gamma=0.9, alpha=2.0, eta_max=0.9, eta0=0.5):
    if k == 0:
        eta = eta0
    else:
        eta = gamma * (rn / rprev) ** alpha
        sg = gamma * eta_prev ** alpha
        if sg > 0.1:
            eta = max(eta, sg)
        eta = min(eta, eta_max)
    eta = max(eta, 0.5 * tol / rn)
    return min(eta, eta_max)


def newton_step(prob, Un, opts: NewtonOpts = NewtonOpts(), guess=None):
    """One trapezoidal step: solve L(u) = f(u^n) by inexact Newton-GMRES."""
    f = M.rhs(prob, Un)
    U = Un.copy() if guess is None else guess.copy()
    R = M.residual(prob, U, f)
    r0 = _nrm(R)
    tol = max(opts.rtol * r0, opts.atol_factor * _nrm(2.0 * Un / prob.dt))
    info = NewtonInfo()
    info.res.append(r0)
    rn, rprev, eta = r0, r0, 0.5
    for k in range(opts.max_newton + 1):
        if rn <= tol:
            info.converged = True
            break
        if k == opts.max_newton:
            break
        if opts.forcing == "ew":
            eta = ew_forcing(k, rn, rprev, eta, tol)
        else:
            eta = opts.eta
        eta = max(eta, opts.eta_floor)
        Uk = U

        def matvec(v, Uk=Uk):
            if opts.jv == "analytic":
                return M.jv(prob, Uk, v, 0.0)
            eps = M.fd_eps(prob, Uk, v, opts.eps_mach)
            if opts.jv == "literal":
                return M.jv_literal(prob, Uk, v, eps)
            return M.jv(prob, Uk, v, eps)

        if opts.pc == "physics":
            fr = PC.frozen_coefficients(prob, Uk)
            pc = lambda r, fr=fr, Uk=Uk: PC.physics_pc(prob, Uk, r, opts.sweeps, fr)
        else:
            pc = lambda r: r
        du, gi = fgmres(matvec, pc, -R, m=opts.m, tol=eta,
                        max_iters=opts.m * opts.max_restarts, ortho=opts.ortho,
                        true_residual=False)
        info.gmres_iters.append(gi.iters)
        U = U + du
        R = M.residual(prob, U, f)
        rprev, rn = rn, _nrm(R)
        info.res.append(rn)
        info.newton_iters = k + 1
    return U, info
