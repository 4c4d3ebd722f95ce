"""Physics-based preconditioner (section 2.5.2): keep each field's own diagonal
block of L(u) = 2u/dt - F(u) and drop the coupling between fields.

ORACLE - test infrastructure only.

Reading used (the paper names the idea, not the operator): with the state u frozen
at the current Newton iterate, the block of field phi is

    P_phi z = (2/dt) z + C(a(u); z) - sum_j D_j( K_phi D_j z ),

the skew convection of z by the frozen velocity plus a frozen-coefficient
diffusion, K = nu(u) for velocity components, nu(u)/Pr_t for theta and 0 for the
pressure.  It is applied approximately by Jacobi sweeps with the diagonal
d_phi = 2/dt + (sum_m c_m^2) K_phi sum_j 1/h_j^2 (c_m the derivative stencil,
the skew convection contributes nothing to the diagonal):

    z_0 = r / d,   z_{s+1} = z_s + (r - P z_s) / d,   s = 0 .. sweeps-1.

For a fixed number of sweeps this is a fixed linear map, so it is a valid right
preconditioner for GMRES.
"""
from __future__ import annotations

import numpy as np

from . import model as M
from .stencil import stencil


def frozen_coefficients(prob, U):
    """Extended frozen velocity and the (horizontal, vertical) momentum and heat
    coefficients of the state U (one array both ways for isotropic closures)."""
    ops = M._Ops(prob)
    vel, p, th = M._ext_state(prob, U)
    S = M.strain(ops, vel)
    Kmom, Kheat = M.exchange_coefficients(prob, S, p.shape)
    return vel, Kmom, Kheat


def _block_coeff(prob, name, Kmom, Kheat):
    if name == "p":
        z = np.zeros(Kmom[0].shape)
        return z, z
    if name == "theta":
        return Kheat
    return Kmom


def apply_blocks(prob, U, Z, frozen=None):
    """P(u) z for all fields (block-diagonal operator)."""
    vel, Kmom, Kheat = frozen if frozen is not None else frozen_coefficients(prob, U)
    ops = M._Ops(prob)
    names = M.field_names(prob)
    out = np.zeros(Z.shape)
    for k, name in enumerate(names):
        z = M.extend(prob, Z[k], name)
        K = _block_coeff(prob, name, Kmom, Kheat)
        t = 0.0
        for j in range(prob.dim):
            t = t - ops.D((K[1] if j == prob.dim - 1 else K[0]) * ops.D(z, j), j)
        if prob.convection:
            t = t + M.convection(ops, vel, z)
        out[k] = 2.0 * Z[k] / prob.dt + M.interior(prob, t)
    return out


def diagonal(prob, U, frozen=None):
    vel, Kmom, Kheat = frozen if frozen is not None else frozen_coefficients(prob, U)
    _, c = stencil(prob.dd_p)
    cD = float(np.sum(c * c))
    dx, dy, dz = M.spacings(prob)
    inv_hh = 1.0 / dx ** 2 + (1.0 / dy ** 2 if prob.dim == 3 else 0.0)
    inv_h2 = 1.0 / dx ** 2 + 1.0 / dz ** 2 + (1.0 / dy ** 2 if prob.dim == 3 else 0.0)
    names = M.field_names(prob)
    d = np.zeros((prob.nf,) + (prob.nz, prob.ny, prob.nx))
    for k, name in enumerate(names):
        Kh, Kv = _block_coeff(prob, name, Kmom, Kheat)
        if Kh is Kv:                      # isotropic: K sum_j 1/h_j^2
            d[k] = 2.0 / prob.dt + cD * M.interior(prob, Kh) * inv_h2
        else:                             # sum_j K_j / h_j^2
            d[k] = 2.0 / prob.dt + cD * (M.interior(prob, Kh) * inv_hh + M.interior(prob, Kv) / dz ** 2)
    return d


def physics_pc(prob, U, R, sweeps=2, frozen=None):
    """z ~ P(u)^{-1} r by ``sweeps`` Jacobi sweeps after the diagonal start."""
    fr = frozen if frozen is not None else frozen_coefficients(prob, U)
    d = diagonal(prob, U, fr)
    z = R / d
    for _ in range(sweeps):
        z = z + (R - apply_blocks(prob, U, z, fr)) / d
    return z
