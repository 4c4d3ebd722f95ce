"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds problem *parameters* and *initial states* only.  It contains none
of the solver's arithmetic (no background profiles, no derivative stencils, no
residual terms, no heat-flux conversion): both the CPU oracle and the HIP library
derive everything else from these numbers on their own.

Physical constants are the ones the paper lists with the governing equations
(section 2.1: p0 = 1000 hPa, R = 287, c_p = 1004, c_v = 717); g = 9.81 m/s^2 and
theta0 = 300 K are the values used by the paper's test cases (section 3.1).

Workloads (synthetic stand-ins for the paper's dry-thermal and urban-heat-island
experiments, sections 3.1-3.2):

* ``thermal_neutral_2d``   128 x 64 over 20 x 10 km, free-slip, +2 K bubble.
* ``thermal_stable_2d``    1024 x 512 over 20 x 10 km, N = 0.01 1/s, Smagorinsky.
* ``heat_island_2d``       2048 x 256 over 40 x 4 km, N = 0.01 1/s, 250 W/m^2 strip.
* ``heat_island_ensemble`` 64 uneven 2D heat-island instances drawn from a seed.
* ``thermal_neutral_3d``   256 x 256 x 128 over 20 x 20 x 10 km.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

# closure kinds
CLOSURE_CONST_K = 0
CLOSURE_SMAGORINSKY = 1
CLOSURE_NONE = 2
CLOSURE_DEARDORFF = 3              # anisotropic coefficients of Eq. 7
# boundary kinds
BC_FREE_SLIP = 0
BC_NO_SLIP_BOTTOM = 1
BC_PERIODIC = 2
# surface strip shapes
STRIP_TOPHAT = 0
STRIP_TANH = 1


@dataclass
class Problem:
    """Parameters of one implicit-step problem.  Field layout of every state
    vector is ``[n_f][nz][ny][nx]`` (x fastest); 2D problems have ``ny == 1`` and
    fields (u, w, p, theta), 3D problems fields (u, v, w, p, theta)."""

    dim: int = 2
    nx: int = 128
    ny: int = 1
    nz: int = 64
    lx: float = 20000.0
    ly: float = 1.0
    lz: float = 10000.0
    dt: float = 2.0
    theta0: float = 300.0
    g: float = 9.81
    cp: float = 1004.0
    cv: float = 717.0
    rgas: float = 287.0
    p_ref: float = 100000.0          # Pa, reference pressure p0
    kappa_div: float = 0.0           # <= 0 selects the default reading R/c_v
    n_bv: float = 0.0                # Brunt-Vaisala frequency [1/s]
    closure: int = CLOSURE_SMAGORINSKY
    cs: float = 0.18
    pr_t: float = 0.71
    k_m: float = 10.0
    k_h: float = 14.1
    bc_lateral: int = BC_FREE_SLIP
    bc_vertical: int = BC_FREE_SLIP
    h0: float = 0.0                  # surface heat flux over the strip [W/m^2]
    strip_width: float = 0.0         # [m]
    strip_center: float = 0.0        # [m], x position of the strip centre
    strip_shape: int = STRIP_TOPHAT
    strip_xi: float = 0.1
    convection: int = 1              # 0 drops the convective terms (linear test operator)
    energy_test: int = 0             # 1: frozen Exner coefficient, no background-gradient term
    dd_p: int = 2                    # Deslauriers-Dubuc order parameter

    @property
    def nf(self) -> int:
        return 4 if self.dim == 2 else 5

    @property
    def npts(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n(self) -> int:
        return self.nf * self.npts

    @property
    def shape(self):
        return (self.nf, self.nz, self.ny, self.nx)

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------- #
# named workloads
# --------------------------------------------------------------------------- #
def thermal_neutral_2d(nx=128, nz=64) -> Problem:
    return Problem(dim=2, nx=nx, nz=nz, lx=20000.0, lz=10000.0, dt=2.0, n_bv=0.0)


def thermal_stable_2d(nx=1024, nz=512) -> Problem:
    return Problem(dim=2, nx=nx, nz=nz, lx=20000.0, lz=10000.0, dt=1.0, n_bv=0.01)


def heat_island_2d(nx=2048, nz=256, h0=250.0, width=4000.0, n_bv=0.01) -> Problem:
    return Problem(dim=2, nx=nx, nz=nz, lx=40000.0, lz=4000.0, dt=2.0, n_bv=n_bv,
                   bc_vertical=BC_NO_SLIP_BOTTOM, h0=h0, strip_width=width,
                   strip_center=20000.0)


def thermal_neutral_3d(nx=256, ny=256, nz=128) -> Problem:
    return Problem(dim=3, nx=nx, ny=ny, nz=nz, lx=20000.0, ly=20000.0, lz=10000.0,
                   dt=2.0, n_bv=0.0)


ENSEMBLE_GRIDS = [(256, 64), (512, 64), (512, 128), (1024, 128)]


def heat_island_ensemble(n_inst=64, seed=0) -> List[Problem]:
    """Draws, per instance and in this order: grid (uniform over four sizes),
    H0 log-uniform in [25, 930] W/m^2, strip width uniform in [1, 8] km and
    N uniform in [0.005, 0.02] 1/s.  Domain 40 x 4 km as the single heat island."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n_inst):
        gi = int(rng.integers(0, len(ENSEMBLE_GRIDS)))
        h0 = float(np.exp(rng.uniform(np.log(25.0), np.log(930.0))))
        width = float(rng.uniform(1000.0, 8000.0))
        nbv = float(rng.uniform(0.005, 0.02))
        nx, nz = ENSEMBLE_GRIDS[gi]
        out.append(heat_island_2d(nx=nx, nz=nz, h0=h0, width=width, n_bv=nbv))
    return out


# --------------------------------------------------------------------------- #
# initial states
# --------------------------------------------------------------------------- #
def _coords(prob: Problem):
    """Cell-centre coordinates x_i = (i + 1/2) dx (and y, z alike)."""
    x = (np.arange(prob.nx) + 0.5) * (prob.lx / prob.nx)
    y = (np.arange(prob.ny) + 0.5) * (prob.ly / prob.ny)
    z = (np.arange(prob.nz) + 0.5) * (prob.lz / prob.nz)
    return x, y, z


def bubble_state(prob: Problem, center=None, radius=2000.0, amp=2.0) -> np.ndarray:
    """Rest state plus a cosine-squared potential-temperature bubble,
    theta' = amp cos^2(pi r / (2 R)) for r <= R, zero elsewhere."""
    x, y, z = _coords(prob)
    if center is None:
        center = (prob.lx / 2, prob.ly / 2, 2000.0)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    r2 = (X - center[0]) ** 2 + (Z - center[2]) ** 2
    if prob.dim == 3:
        r2 = r2 + (Y - center[1]) ** 2
    r = np.sqrt(r2)
    th = np.where(r <= radius, amp * np.cos(np.pi * r / (2 * radius)) ** 2, 0.0)
    U = np.zeros(prob.shape)
    U[-1] = th
    return U


def rest_state(prob: Problem) -> np.ndarray:
    return np.zeros(prob.shape)


def smooth_flow_state(prob: Problem, seed=0, kmax=16, umax=10.0, p_std=0.01,
                      with_bubble=True) -> np.ndarray:
    """Random smooth divergence-free velocity from a sine-series streamfunction
    (modes 1..kmax per direction), scaled to max |velocity| = umax, plus the
    +2 K bubble and Gaussian pressure noise of standard deviation p_std.

    The series is differentiated analytically, so the velocity vanishes in the
    wall-normal component at free-slip walls; it is an input, not a discrete
    divergence-free field of any particular stencil."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y, z = _coords(prob)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    U = np.zeros(prob.shape)
    km = min(kmax, max(1, prob.nx // 4)), min(kmax, max(1, prob.nz // 4))
    if prob.dim == 2:
        u = np.zeros(X.shape)
        w = np.zeros(X.shape)
        for m in range(1, km[0] + 1):
            for n in range(1, km[1] + 1):
                a = rng.normal() / (m * m + n * n)
                ax, az = m * np.pi / prob.lx, n * np.pi / prob.lz
                # psi = a sin(ax x) sin(az z); u = -dpsi/dz, w = dpsi/dx
                u += -a * az * np.sin(ax * X) * np.cos(az * Z)
                w += a * ax * np.cos(ax * X) * np.sin(az * Z)
        s = umax / max(np.abs(u).max(), np.abs(w).max(), 1e-300)
        U[0], U[1] = u * s, w * s
    else:
        # two streamfunction components: psi_x, psi_y give u = curl(psi)
        u = np.zeros(X.shape); v = np.zeros(X.shape); w = np.zeros(X.shape)
        kmy = min(kmax, max(1, prob.ny // 4))
        kk = min(km[0], kmy, km[1], 6)
        for m in range(1, kk + 1):
            for l in range(1, kk + 1):
                for n in range(1, kk + 1):
                    a, b = rng.normal(size=2) / (m * m + l * l + n * n)
                    ax, ay, az = m * np.pi / prob.lx, l * np.pi / prob.ly, n * np.pi / prob.lz
                    # A = (0, a s_x c_y s_z? ...): use u = -d(psi1)/dz, w = d(psi1)/dx and
                    # v = -d(psi2)/dz, w += d(psi2)/dy with psi1 = a s(ax x) c(ay y) s(az z),
                    # psi2 = b c(ax x) s(ay y) s(az z); each pair is divergence free.
                    u += -a * az * np.sin(ax * X) * np.cos(ay * Y) * np.cos(az * Z)
                    w += a * ax * np.cos(ax * X) * np.cos(ay * Y) * np.sin(az * Z)
                    v += -b * az * np.cos(ax * X) * np.sin(ay * Y) * np.cos(az * Z)
                    w += b * ay * np.cos(ax * X) * np.cos(ay * Y) * np.sin(az * Z)
        s = umax / max(np.abs(u).max(), np.abs(v).max(), np.abs(w).max(), 1e-300)
        U[0], U[1], U[2] = u * s, v * s, w * s
    U[-2] = rng.normal(scale=p_std, size=X.shape)
    if with_bubble:
        U[-1] = bubble_state(prob)[-1]
    return U


def random_vector(prob: Problem, seed=1, normalize=True) -> np.ndarray:
    """Standard-normal direction vector (optionally unit 2-norm)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.normal(size=prob.shape)
    if normalize:
        v /= np.sqrt(np.sum(v * v))
    return v


def random_smooth_vector(prob: Problem, seed=2) -> np.ndarray:
    """Smooth random direction (used where a rough direction would hide bugs in
    the derivative terms behind grid-scale noise)."""
    V = smooth_flow_state(prob, seed=seed, umax=1.0, p_std=0.0, with_bubble=False)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    x, y, z = _coords(prob)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    for f in (-2, -1):
        a, b = rng.normal(size=2)
        V[f] = a * np.cos(2 * np.pi * X / prob.lx) * np.cos(np.pi * Z / prob.lz) + \
            b * np.cos(np.pi * X / prob.lx) * np.cos(2 * np.pi * Z / prob.lz)
    return V


# --------------------------------------------------------------------------- #
# learned-preconditioner parameters
# --------------------------------------------------------------------------- #
NET_HIDDEN = 16


def net_layer_shapes(nf: int, dim: int = 2):
    """(W shape, b shape) per layer of the 4-layer network nf->16->16->16->nf
    (3 x 3 kernels in 2D, 3 x 3 x 3 in 3D)."""
    ch = [nf, NET_HIDDEN, NET_HIDDEN, NET_HIDDEN, nf]
    return [((ch[l + 1], ch[l]) + (3,) * dim, (ch[l + 1],)) for l in range(4)]


def net_init_params(nf: int, seed: int = 0, out_scale: float = 0.1, dim: int = 2) -> np.ndarray:
    """Seeded He-normal initial weights, zero biases, last layer scaled by
    out_scale; one flat float64 vector (per layer W[co][ci][taps], then b)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    shapes = net_layer_shapes(nf, dim)
    for l, (ws, bs) in enumerate(shapes):
        W = rng.normal(scale=math.sqrt(2.0 / (ws[1] * 3 ** dim)), size=ws)
        if l == len(shapes) - 1:
            W = W * out_scale
        parts += [W.ravel(), np.zeros(bs)]
    return np.concatenate(parts)
