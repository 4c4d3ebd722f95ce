"""Pins of three oracle parts that the symmetry and conservation tests do not
reach: the background terms of the Exner equation (section 2.1, Eq. 1 read for
the total p_bar + p'), the tanh surface-flux strip (section 3.2 boundary
condition) and the filter width Delta_LES of the eddy viscosity (section 2.4)
on a grid with dx != dz.  Each expected value is built from something other
than the oracle's own formula: a rigid translation of the hydrostatic column,
the closed-form action of the derivative on sinusoids with a background
integrated by quadrature, the closed-form integral of the tanh strip, and the
exact strain of a linear shear.  Each test also checks that the mistake it
guards against (named in the test) would move the result far outside its
tolerance.  No GPU."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import model as M
from paper_2007_10411_amd import inputs as I


def _grid(prob):
    x = (np.arange(prob.nx) + 0.5) * (prob.lx / prob.nx)
    z = (np.arange(prob.nz) + 0.5) * (prob.lz / prob.nz)
    return np.meshgrid(z, np.zeros(1), x, indexing="ij")


def _hydrostatic_column(prob, z):
    """Exner background from the hydrostatic balance dP/dz = -g / theta_bar(z),
    P(0) = c_p, integrated by adaptive quadrature, theta_bar = theta0 + beta z with
    beta fixed by the Brunt-Vaisala frequency (N^2 = g beta / theta0)."""
    b = prob.n_bv ** 2 * prob.theta0 / prob.g
    integrand = lambda s: prob.g / (prob.theta0 + b * s)
    return np.array([prob.cp - integrate.quad(integrand, 0.0, float(zz), epsabs=0.0, epsrel=1e-13)[0]
                     for zz in np.ravel(z)]).reshape(np.shape(z))


def _column_slope(prob, z, h=0.25):
    """dP/dz of the quadrature column by a fourth-order central difference."""
    P = lambda s: _hydrostatic_column(prob, s)
    return (8.0 * (P(z + h) - P(z - h)) - (P(z + 2 * h) - P(z - 2 * h))) / (12.0 * h)


def _kmod(k, h):
    """Modified wavenumber of the 5-point DD derivative (coefficients 2/3, -1/12,
    pinned by the stencil tests): D sin(kx) = kmod cos(kx) on samples."""
    return ((4.0 / 3.0) * math.sin(k * h) - (1.0 / 6.0) * math.sin(2.0 * k * h)) / h


# --------------------------------------------------------------------------- #
# Exner equation: -w dp_bar/dz and kappa (p_bar + p') div u
# --------------------------------------------------------------------------- #
def test_uniform_lift_moves_the_background_column():
    """A uniform vertical velocity w0 with no perturbations carries the hydrostatic
    column rigidly: at a fixed point the total Exner pressure changes as
    -w0 dP/dz and the potential temperature as -w0 dtheta_bar/dz, while nothing
    else moves.  Doubly periodic grid (test boundary kind) so that a uniform w is
    admissible; the background terms are pointwise.  Guards a sign slip in
    -w dp_bar/dz (the tendency would point the other way) and in -beta w."""
    prob = I.Problem(dim=2, nx=8, nz=16, lx=20000.0, lz=10000.0, dt=2.0, n_bv=0.012,
                     bc_lateral=I.BC_PERIODIC, bc_vertical=I.BC_PERIODIC)
    w0 = 3.0
    U = np.zeros(prob.shape)
    U[1] = w0
    Fv = M.F(prob, U)
    Z = _grid(prob)[0]
    dPdz = _column_slope(prob, Z)
    beta = prob.n_bv ** 2 * prob.theta0 / prob.g
    want_p = -w0 * dPdz
    assert np.abs(Fv[2] - want_p).max() <= 1e-10 * np.abs(want_p).max()
    assert np.abs(Fv[3] + w0 * beta).max() <= 1e-13 * w0 * beta
    assert np.abs(Fv[0]).max() == 0.0 and np.abs(Fv[1]).max() == 0.0
    # upward motion raises the pressure at a fixed point (it decreases with height)
    assert (Fv[2] > 0).all()
    # a flipped background advection would be off by twice the term
    assert np.abs(-want_p - want_p).max() > 1e6 * 1e-10 * np.abs(want_p).max()


def _exner_state(prob, A, B, C, P0, mx, mz):
    X = _grid(prob)[2]
    Z = _grid(prob)[0]
    kx, kz = 2 * math.pi * mx / prob.lx, math.pi * mz / prob.lz
    U = np.zeros(prob.shape)
    U[0] = A * np.sin(kx * X) * np.cos(kz * Z)
    U[1] = B * np.cos(kx * X) * np.sin(kz * Z)
    U[2] = C * np.cos(kx * X) * np.cos(kz * Z) + P0
    div = (A * _kmod(kx, prob.lx / prob.nx) + B * _kmod(kz, prob.lz / prob.nz)) * np.cos(kx * X) * np.cos(kz * Z)
    return U, div, Z


@pytest.mark.parametrize("n_bv", [0.0, 0.01])
def test_exner_tendency_closed_form_with_lift_and_perturbation(n_bv):
    """F_p for u = A sin(kx x) cos(kz z), w = B cos(kx x) sin(kz z),
    p' = C cos(kx x) cos(kz z) + P0 on a grid periodic in x with free-slip walls
    in z (the sinusoids carry the walls' parities, so their ghost values are
    their own continuation), convection and closure off:
        F_p = -w dP/dz - kappa (P + p') div u,
    P the hydrostatic column by quadrature, div u = (A kmod_x + B kmod_z) cos cos
    from the derivative's closed form on sinusoids, kappa = R / c_v (Exner
    pressure of an adiabatic, mass-conserving parcel).  Guards a sign flip of
    -w dp_bar/dz, a dropped kappa p' div u, and the printed c_p / c_v."""
    prob = I.Problem(dim=2, nx=32, nz=24, lx=20000.0, lz=10000.0, dt=2.0, n_bv=n_bv,
                     bc_lateral=I.BC_PERIODIC, bc_vertical=I.BC_FREE_SLIP,
                     closure=I.CLOSURE_NONE, convection=0)
    U, div, Z = _exner_state(prob, A=1.5, B=-2.0, C=40.0, P0=15.0, mx=2, mz=3)
    Fv = M.F(prob, U)
    P = _hydrostatic_column(prob, Z)
    dPdz = _column_slope(prob, Z)
    kap = prob.rgas / prob.cv
    want = -U[1] * dPdz - kap * (P + U[2]) * div
    tol = 1e-11 * np.abs(want).max()
    assert np.abs(Fv[2] - want).max() <= tol
    # the mistakes this pins would each move F_p far beyond the tolerance
    mutants = {"flipped background advection": +U[1] * dPdz - kap * (P + U[2]) * div,
               "dropped kappa p' div u": -U[1] * dPdz - kap * P * div,
               "printed c_p / c_v": -U[1] * dPdz - (prob.cp / prob.cv) * (P + U[2]) * div}
    for name, bad in mutants.items():
        assert np.abs(bad - want).max() > 1e4 * tol, name


# --------------------------------------------------------------------------- #
# tanh surface-flux strip
# --------------------------------------------------------------------------- #
def _logcosh(y):
    return np.logaddexp(y, -y) - math.log(2.0)


@pytest.mark.parametrize("xi", [0.1, 0.25])
def test_heat_budget_of_the_tanh_strip(xi):
    """With a discretely divergence-free flow, beta = 0 and free-slip walls, the
    domain integral of F_theta equals the surface flux integral.  For the strip
    (H0/2)[tanh((x'+1)/xi) - tanh((x'-1)/xi)], x' in half-widths from the strip
    centre, that integral is in closed form,
        half * (H0/2) * 2 xi [logcosh((L+1)/xi) - logcosh((L-1)/xi)]  (-> H0 W),
    L the distance to the walls in half-widths; the midpoint sum of an analytic
    profile whose tails vanish at the walls reaches it to rounding.  Converted
    with rho0 = p_ref / (R theta0).  Guards the printed peak 2 H0 (no 1/2) and
    a strip measured in metres instead of half-widths."""
    prob = I.Problem(dim=2, nx=400, nz=6, lx=20000.0, lz=3000.0, dt=2.0, n_bv=0.0,
                     h0=250.0, strip_width=4000.0, strip_center=10000.0,
                     strip_shape=I.STRIP_TANH, strip_xi=xi)
    rng = np.random.Generator(np.random.PCG64(11))
    U = 0.1 * rng.normal(size=prob.shape)
    # streamfunction velocity, odd at every wall, so the discrete divergence is zero
    ops = M._Ops(prob)
    psi = rng.normal(size=(prob.nz, prob.ny, prob.nx))
    ix, sx = M._axis_map(prob.nx, prob.bc_lateral, -1, -1, M.ghost(prob))
    iz, sz = M._axis_map(prob.nz, prob.bc_vertical, -1, -1, M.ghost(prob))
    pe = psi[np.ix_(iz, np.arange(prob.ny), ix)] * sz[:, None, None] * sx[None, None, :]
    U[0] = -M.interior(prob, ops.D(pe, 1))
    U[1] = M.interior(prob, ops.D(pe, 0))
    Fv = M.F(prob, U)
    dx, _, dz = M.spacings(prob)
    total = float(Fv[3].sum()) * dx * dz
    half = prob.strip_width / 2
    L = prob.strip_center / half                     # walls at x' = -L and +L
    integral_H = half * (prob.h0 / 2) * 2 * xi * (_logcosh((L + 1) / xi) - _logcosh((L - 1) / xi))
    rho0 = prob.p_ref / (prob.rgas * prob.theta0)
    want = integral_H / (rho0 * prob.cp)
    scale = float(np.abs(Fv[3]).sum()) * dx * dz
    assert abs(total - want) <= 1e-11 * max(want, scale)
    assert abs(integral_H - prob.h0 * prob.strip_width) <= 1e-6 * prob.h0 * prob.strip_width
    # the printed strip (peak 2 H0) doubles the budget; a width in metres changes it wholesale
    assert abs(2 * want - want) > 1e6 * 1e-11 * max(want, scale)
    x = (np.arange(prob.nx) + 0.5) * dx
    metres = 0.5 * prob.h0 * (np.tanh((x - prob.strip_center + 1) / xi) - np.tanh((x - prob.strip_center - 1) / xi))
    assert abs(metres.sum() * dx / (rho0 * prob.cp) - want) > 1e6 * 1e-11 * max(want, scale)


# --------------------------------------------------------------------------- #
# filter width of the eddy viscosity
# --------------------------------------------------------------------------- #
@pytest.mark.parametrize("dim", [2, 3])
def test_eddy_viscosity_of_a_linear_shear_on_an_anisotropic_grid(dim):
    """u = gamma z has S_xz = S_zx = gamma/2 and no other strain, so
    sqrt(2 S:S) = |gamma| and the Smagorinsky viscosity is (C_s Delta)^2 |gamma|,
    with Delta the geometric mean spacing, sqrt(dx dz) in 2D and
    (dx dy dz)^(1/3) in 3D.  The 5-point derivative is exact on linear functions,
    so every point whose stencil stays off the mirrored ghosts sees the exact
    strain.  Spacings 1250 / 833.3 / 250 m.  Guards the arithmetic mean and the
    vertical spacing alone."""
    gamma = 0.02
    kw = dict(dim=dim, nx=16, nz=20, lx=20000.0, lz=5000.0, dt=2.0, bc_lateral=I.BC_PERIODIC)
    if dim == 3:
        kw.update(ny=12, ly=10000.0)
    prob = I.Problem(**kw)
    dx, dy, dz = M.spacings(prob)
    z = (np.arange(prob.nz) + 0.5) * dz
    U = np.zeros(prob.shape)
    U[0] = gamma * z[:, None, None]
    ops = M._Ops(prob)
    vel, p, th = M._ext_state(prob, U)
    S = M.strain(ops, vel)
    nu, kth = M.eddy_viscosity(prob, S, p.shape)
    nu_i = M.interior(prob, nu)
    inner = slice(2, prob.nz - 2)                    # stencils off the wall ghosts
    delta = math.sqrt(dx * dz) if dim == 2 else (dx * dy * dz) ** (1.0 / 3.0)
    want = (prob.cs * delta) ** 2 * gamma
    assert np.abs(nu_i[inner] - want).max() <= 1e-13 * want
    assert np.abs(M.interior(prob, kth)[inner] - want / prob.pr_t).max() <= 1e-13 * want
    wrong = [(dx + dz) / 2 if dim == 2 else (dx + dy + dz) / 3, dz]
    for d in wrong:
        assert abs((prob.cs * d) ** 2 * gamma - want) > 1e6 * 1e-13 * want
