"""Constant-coefficient dry thermal runs (section 3.1.1, Table 1).

A +2 K thermal of radius 2 km rises in a neutral environment over 20 x 10 km
with constant momentum and heat exchange coefficients K_M, K_H (Case A: fixed
Prandtl number 0.71; Case B: K_H = 5 with varying K_M).  ``run_case`` advances
the implicit solver to t_end and returns the extreme values of theta', u, w and
the vorticity omega = du/dz - dw/dx at t_end (the quantities of Tables 2 and 3)
with the time series of the kinetic and potential energies of section 3.1.3,
E_k = 1/2 int (u^2 + w^2) dV and E_p = int (z_max - z) theta' dV.  The exchange
between them runs through the buoyancy g theta'/theta0, so the energy budget
adds (g/theta0) E_p to E_k (``total_energy``).

The steps run in the HIP library; the diagnostics here are plain torch
reductions over the state between steps (the vorticity with the same 5-point
derivative, mirror-reflected at the walls) and are not part of the timed path.
The paper does not state its grid or time step: the default 256 x 128 grid
(78.125 m) and dt = 2 s are this driver's choice.
"""
from __future__ import annotations

import time

from . import inputs as I

CASE_A = [(10.0, 14.1), (5.0, 7.04), (2.5, 3.52), (1.0, 1.41)]   # (K_M, K_H), Pr = 0.71
CASE_B = [(10.0, 5.0), (5.0, 5.0), (2.5, 5.0)]                   # K_H = 5


def case_problem(km, kh, nx=256, nz=128, dt=2.0, n_bv=0.0):
    return I.thermal_neutral_2d(nx, nz).replace(closure=I.CLOSURE_CONST_K, k_m=float(km), k_h=float(kh),
                                                dt=float(dt), n_bv=float(n_bv))


def _d5(a, axis, h, parity):
    """5-point derivative (2/3, -1/12)/h along axis with a mirror ghost of the
    given parity (+1 even, -1 odd) at both walls."""
    import torch
    n = a.shape[axis]
    lo = a.narrow(axis, 0, 2).flip(axis) * parity
    hi = a.narrow(axis, n - 2, 2).flip(axis) * parity
    e = torch.cat([lo, a, hi], dim=axis)
    s = lambda k: e.narrow(axis, 2 + k, n)
    return ((2.0 / 3.0) * (s(1) - s(-1)) - (1.0 / 12.0) * (s(2) - s(-2))) / h


def diagnostics(prob, u):
    """Extremes of theta', u, w, omega and the energies of a 2D state (device
    tensor) with free-slip walls (u even across the bottom and top, w even across
    the sides)."""
    U = u.reshape(prob.shape)[:, :, 0, :]           # (4, nz, nx)
    uu, ww, th = U[0], U[1], U[3]
    dx, dz = prob.lx / prob.nx, prob.lz / prob.nz
    om = _d5(uu, 0, dz, 1.0) - _d5(ww, 1, dx, 1.0)
    import torch
    z = (torch.arange(prob.nz, device=u.device, dtype=u.dtype) + 0.5) * dz
    dA = dx * dz
    ek = 0.5 * float(((uu * uu + ww * ww).sum()) * dA)
    ep = float((((prob.lz - z)[:, None]) * th).sum() * dA)
    ext = {}
    for name, f in (("theta", th), ("u", uu), ("w", ww), ("omega", om)):
        ext[name + "_min"] = float(f.min())
        ext[name + "_max"] = float(f.max())
    return ext, ek, ep


def total_energy(prob, ek, ep):
    """E_k + (g/theta0) E_p, the sum that the buoyancy exchange conserves."""
    return ek + prob.g / prob.theta0 * ep


def run_case(ctx, prob, t_end=1000.0, inner="f32", rtol=1e-8, every=10, pc="physics"):
    """Advance the thermal from rest to t_end; returns (extremes at t_end,
    [(t, E_k, E_p)], totals)."""
    import torch
    u = torch.from_numpy(I.bubble_state(prob)).cuda()
    nxt = torch.empty_like(u)
    nsteps = int(round(t_end / prob.dt))
    series = []
    _, ek, ep = diagnostics(prob, u)
    series.append((0.0, ek, ep))
    newton = gmres = 0
    t0 = time.perf_counter()
    for k in range(1, nsteps + 1):
        nxt.copy_(u)
        r = ctx.newton_step(u, nxt, rtol=rtol, inner=inner, pc=pc, eta_floor=1e-4 if inner == "f32" else 0.0)
        if not r.converged:
            raise RuntimeError(f"step {k}: Newton did not converge: {r}")
        newton += r.newton_iters
        gmres += r.gmres_iters_total
        u.copy_(nxt)
        if k % every == 0 or k == nsteps:
            _, ek, ep = diagnostics(prob, u)
            series.append((k * prob.dt, ek, ep))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ext, _, _ = diagnostics(prob, u)
    return ext, series, {"steps": nsteps, "newton_iters": newton, "gmres_iters": gmres, "wall_s": wall, "u": u}
