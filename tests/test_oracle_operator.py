"""Pins of the oracle's F(u) against what the paper and the mathematics fix:
skew-symmetry of the convective form (section 2.2), symmetric dissipative
diffusion (section 2.4), global mass and heat budgets, the energy of the inviscid
operator (sections 2.2, 3.1.3), the rest state, the internal-wave dispersion
relation omega = N cos(alpha) (section 3.1.2) and mirror symmetry.  No GPU."""
import math

import numpy as np
import pytest

from oracle import model as M
from paper_2007_10411_amd import inputs as I


def _prob(**kw):
    base = dict(dim=2, nx=24, nz=16, lx=20000.0, lz=10000.0, dt=2.0)
    base.update(kw)
    return I.Problem(**base)


def _rand(prob, seed):
    return np.random.Generator(np.random.PCG64(seed)).normal(size=prob.shape)


def _inner(a, b):
    return float(np.sum(a * b))


BCS = [(0, 0), (0, 1), (2, 2), (0, 2)]


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("bcl,bcv", BCS)
@pytest.mark.parametrize("dim", [2, 3])
def test_skew_symmetry_for_any_velocity(dim, bcl, bcv, p):
    """<phi, C(a; phi)> = 0 for every field phi and any velocity a (both stencils)."""
    prob = _prob(dim=dim, nx=12, ny=(10 if dim == 3 else 1), nz=(8 if p == 2 else 9), ly=15000.0,
                 bc_lateral=bcl, bc_vertical=bcv, dd_p=p)
    U = _rand(prob, 1)
    ops = M._Ops(prob)
    vel, p, th = M._ext_state(prob, U)
    names = M.field_names(prob)
    for k, name in enumerate(names):
        phi = M.extend(prob, U[k] if k < prob.nf else U[k], name)
        c = M.interior(prob, M.convection(ops, vel, phi))
        scale = float(np.sum(np.abs(c * U[k])))
        assert abs(_inner(U[k], c)) <= 1e-13 * scale, (name, _inner(U[k], c), scale)


def _streamfunction_velocity(prob, seed):
    """Discretely divergence-free velocity u = -D_z psi, w = D_x psi from a
    random psi that is odd at every wall."""
    ops = M._Ops(prob)
    psi = np.random.Generator(np.random.PCG64(seed)).normal(size=(prob.nz, prob.ny, prob.nx))
    # extend psi as odd in x and z (same parity as a normal velocity in both)
    ix, sx = M._axis_map(prob.nx, prob.bc_lateral, -1, -1, M.ghost(prob))
    iz, sz = M._axis_map(prob.nz, prob.bc_vertical, -1, -1, M.ghost(prob))
    pe = psi[np.ix_(iz, np.arange(prob.ny), ix)] * sz[:, None, None] * sx[None, None, :]
    u = -M.interior(prob, ops.D(pe, 1))
    w = M.interior(prob, ops.D(pe, 0))
    return u, w


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("bcl,bcv", [(0, 0), (2, 2), (0, 1)])
def test_mass_conservation_and_divergence_free_convection(bcl, bcv, p):
    prob = _prob(bc_lateral=bcl, bc_vertical=bcv, dd_p=p)
    ops = M._Ops(prob)
    U = _rand(prob, 3)
    vel, p, th = M._ext_state(prob, U)
    S = M.strain(ops, vel)
    div = M.interior(prob, M._trace(S))
    # sum of the discrete divergence vanishes for any velocity with odd normal component
    assert abs(div.sum()) <= 1e-13 * np.abs(div).sum()
    # sum C(a; theta) = -1/2 sum theta div a
    c = M.interior(prob, M.convection(ops, vel, th))
    lhs, rhs = c.sum(), -0.5 * float(np.sum(U[-1] * div))
    assert abs(lhs - rhs) <= 1e-13 * np.abs(c).sum()
    # discretely divergence-free velocity: flux and advective forms agree, and
    # the convective heat transport sums to zero
    u, w = _streamfunction_velocity(prob, 4)
    U[0], U[1] = u, w
    vel, p, th = M._ext_state(prob, U)
    divd = M.interior(prob, M._trace(M.strain(ops, vel)))
    assert np.abs(divd).max() <= 1e-13 * (np.abs(u).max() + np.abs(w).max()) / 100.0
    flux = sum(ops.D(vel[j] * th, j) for j in range(2))
    adv = sum(vel[j] * ops.D(th, j) for j in range(2))
    f_i, a_i = M.interior(prob, flux), M.interior(prob, adv)
    # a discrete D has no product rule, so the two forms differ pointwise; their
    # global sums agree (both vanish) once the discrete divergence is zero
    assert abs(f_i.sum()) <= 1e-13 * np.abs(f_i).sum()
    assert abs(a_i.sum()) <= 1e-13 * np.abs(a_i).sum()
    c = M.interior(prob, M.convection(ops, vel, th))
    assert abs(c.sum()) <= 1e-13 * np.abs(c).sum()


def test_heat_budget_equals_surface_flux():
    """With a divergence-free flow, beta = 0 and walls, sum F_theta dV equals the
    surface flux integral (diffusive fluxes telescope, convection conserves).
    Free-slip walls: at a no-slip bottom the eddy viscosity formed from the
    mirrored velocity is not even in z, and the wall picks up a diffusive flux."""
    prob = _prob(bc_vertical=0, h0=250.0, strip_width=4000.0, strip_center=10000.0)
    U = _rand(prob, 5) * 0.1
    u, w = _streamfunction_velocity(prob, 6)
    U[0], U[1] = u, w
    Fu = M.F(prob, U)
    dx, _, dz = M.spacings(prob)
    total = Fu[3].sum() * dx * dz
    rho0 = prob.p_ref / (prob.rgas * prob.theta0)
    x = (np.arange(prob.nx) + 0.5) * dx
    Hx = np.where(np.abs(x - 10000.0) <= 2000.0, 250.0, 0.0)
    expect = float(np.sum(Hx / (rho0 * prob.cp))) * dx
    assert abs(total - expect) <= 1e-11 * max(abs(expect), np.abs(Fu[3]).sum() * dx * dz)
    assert abs(expect - 0.214392 * 4000.0 * (Hx > 0).sum() * dx / 4000.0) < 1e-5 * expect


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("bcl,bcv", [(0, 0), (2, 2)])
def test_symmetric_dissipative_diffusion(bcl, bcv, p):
    """<u, D.tau> = -sum tau:S <= 0 and <theta, D.q> = -sum K_theta |D theta|^2 <= 0."""
    prob = _prob(bc_lateral=bcl, bc_vertical=bcv, convection=0, n_bv=0.0, dd_p=p)
    ops = M._Ops(prob)
    U = _rand(prob, 7)
    U[2] = 0.0                                       # no pressure gradient
    Fv = M.F(prob, U)
    vel, p, th = M._ext_state(prob, U)
    S = M.strain(ops, vel)
    nu, kth = M.eddy_viscosity(prob, S, p.shape)
    tau = M.stress(S, nu)
    tS = M.interior(prob, sum(tau[i][j] * S[i][j] for i in range(2) for j in range(2)))
    Fm = Fv[:2].copy()
    Fm[1] = Fm[1] - prob.g / prob.theta0 * U[3]      # remove buoyancy
    lhs = _inner(U[:2], Fm)
    assert lhs < 0
    assert abs(lhs + tS.sum()) <= 1e-12 * np.abs(tS).sum()
    gth = [M.interior(prob, ops.D(th, j)) for j in range(2)]
    qd = float(np.sum(M.interior(prob, kth) * (gth[0] ** 2 + gth[1] ** 2)))
    lt = _inner(U[3], Fv[3])
    assert lt < 0 and abs(lt + qd) <= 1e-12 * qd


def test_constant_coefficient_stress_closed_form():
    """Const-K closure, u = sin(kx) on a periodic grid: F_u = -(4/3) K k~^2 sin(kx),
    F_w = 0 (deviatoric stress with the 1/3 trace term)."""
    prob = _prob(nx=32, nz=8, bc_lateral=2, bc_vertical=2, closure=0, k_m=7.0,
                 convection=0, n_bv=0.0)
    dx = prob.lx / prob.nx
    x = (np.arange(prob.nx) + 0.5) * dx
    k = 2 * np.pi * 3 / prob.lx
    U = np.zeros(prob.shape)
    U[0] = np.sin(k * x)[None, None, :]
    Fv = M.F(prob, U)
    kt = ((4.0 / 3.0) * np.sin(k * dx) - (1.0 / 6.0) * np.sin(2 * k * dx)) / dx
    assert np.allclose(Fv[0], -(4.0 / 3.0) * 7.0 * kt ** 2 * U[0], atol=1e-16, rtol=1e-12)
    assert np.abs(Fv[1]).max() < 1e-18
    # the Exner equation sees the divergence k~ cos(kx) times kappa p_bar
    _, pb, _ = M.background(prob)
    assert np.allclose(Fv[2], -M.kappa(prob) * pb[:, None, None] * kt * np.cos(k * x)[None, None, :],
                       rtol=1e-12, atol=1e-14)


def test_rest_state_is_balanced():
    for prob in (I.thermal_stable_2d(64, 32), I.heat_island_2d(64, 16, h0=0.0),
                 I.thermal_neutral_3d(16, 12, 8)):
        U = I.rest_state(prob)
        assert np.abs(M.F(prob, U)).max() == 0.0
        f = M.rhs(prob, U)
        assert np.abs(M.residual(prob, U, f)).max() == 0.0


def test_background_profile_is_hydrostatic():
    """p_bar(0) = c_p and dp_bar/dz = -g/theta_bar (checked by differentiating the
    closed form numerically)."""
    prob = I.thermal_stable_2d(8, 400)
    z = M.z_centres(prob)
    thb, pb, dpb = M.background(prob)
    num = np.gradient(pb, z)
    assert np.allclose(num[2:-2], dpb[2:-2], rtol=1e-5)
    b = M.beta(prob)
    assert abs(b - 0.01 ** 2 * 300.0 / 9.81) < 1e-15
    assert abs(prob.cp - (pb[0] - dpb[0] * z[0])) < 1e-4      # linear extrapolation to z = 0


@pytest.mark.parametrize("bcl,bcv", [(0, 0), (2, 2)])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("p", [2, 3])
def test_inviscid_operator_conserves_wave_energy(dim, bcl, bcv, p):
    """Energy-test form (no closure, frozen Exner coefficient): <grad E_W, F(u)> = 0
    for any u, convection included."""
    prob = _prob(dim=dim, nx=12, ny=(10 if dim == 3 else 1), nz=(8 if p == 2 else 9), ly=15000.0,
                 bc_lateral=bcl, bc_vertical=bcv, closure=2, energy_test=1, n_bv=0.012, dd_p=p)
    U = _rand(prob, 11)
    Fv = M.F(prob, U)
    Gr = M.wave_energy_gradient(prob, U)
    assert abs(_inner(Gr, Fv)) <= 1e-13 * float(np.sum(np.abs(Gr * Fv)))


# modified-wavenumber weights: k~ dx = 2 sum_m c_m sin(m k dx), c_m the stencil's
# one-sided coefficients (p = 2: 2/3, -1/12; p = 3: 272/365, -53/365, 16/1095, 1/2920)
_KW = {2: (2 / 3, -1 / 12), 3: (272 / 365, -53 / 365, 16 / 1095, 1 / 2920)}


def _ktilde(k, h, p):
    return 2.0 * sum(c * np.sin((m + 1) * k * h) for m, c in enumerate(_KW[p])) / h


def _dispersion_setup(mx=2, mz=1, p=2):
    prob = _prob(nx=32, nz=16, bc_lateral=2, bc_vertical=2, closure=2, energy_test=1,
                 convection=0, n_bv=0.01, dd_p=p)
    dx, _, dz = M.spacings(prob)
    kx, kz = 2 * np.pi * mx / prob.lx, 2 * np.pi * mz / prob.lz
    ktx = _ktilde(kx, dx, p)
    ktz = _ktilde(kz, dz, p)
    c2 = (287.0 / 717.0) * 1004.0 * 300.0
    N2 = 0.01 ** 2
    kt2 = ktx ** 2 + ktz ** 2
    s = N2 + c2 * kt2
    disc = math.sqrt(s * s - 4 * c2 * N2 * ktx ** 2)
    om_g = math.sqrt((s - disc) / 2)      # gravity-wave branch
    om_a = math.sqrt((s + disc) / 2)      # acoustic branch
    x = (np.arange(prob.nx) + 0.5) * dx
    z = (np.arange(prob.nz) + 0.5) * dz
    Z, X = np.meshgrid(z, x, indexing="ij")
    ph = np.exp(1j * (kx * X + kz * Z))[:, None, :]
    beta = N2 * 300.0 / 9.81
    return prob, ktx, ktz, om_g, om_a, ph, beta


def _mode(prob, lam, ktx, ktz, ph, beta):
    N2 = 0.01 ** 2
    p = 1.0
    u = -300.0 * 1j * ktx * p / lam
    w = -300.0 * 1j * ktz * p * lam / (lam * lam + N2)
    th = -beta * w / lam
    U = np.zeros(prob.shape, dtype=complex)
    for k, a in enumerate((u, w, p, th)):
        U[k] = a * ph
    return U


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("branch", ["gravity", "acoustic"])
def test_internal_wave_dispersion(branch, p):
    """Single Fourier mode on a doubly periodic grid is an eigenvector of the linear
    operator with eigenvalue i omega, omega^4 - omega^2 (N^2 + c^2 k~^2) + c^2 N^2 k~_x^2 = 0."""
    prob, ktx, ktz, om_g, om_a, ph, beta = _dispersion_setup(p=p)
    om = om_g if branch == "gravity" else om_a
    lam = 1j * om
    U = _mode(prob, lam, ktx, ktz, ph, beta)
    Fv = M.F(prob, U)
    assert np.abs(Fv - lam * U).max() <= 1e-11 * np.abs(lam * U).max()
    if branch == "gravity":
        # incompressible limit: omega = N cos(alpha) = N k~_x / |k~|
        cos_a = ktx / math.hypot(ktx, ktz)
        assert abs(om / (0.01 * cos_a) - 1.0) < 1e-3


def test_trapezoidal_step_multiplies_mode_by_cayley_factor():
    from oracle import krylov as K
    prob, ktx, ktz, om_g, om_a, ph, beta = _dispersion_setup()
    prob = prob.replace(dt=30.0)
    lam = 1j * om_g
    Uc = _mode(prob, lam, ktx, ktz, ph, beta) * 0.01
    U0 = Uc.real.copy()
    opts = K.NewtonOpts(rtol=1e-13, jv="analytic", forcing="fixed", eta=1e-13, pc="none",
                        m=60, max_restarts=10)
    U1, info = K.newton_step(prob, U0, opts)
    amp = (1 + lam * prob.dt / 2) / (1 - lam * prob.dt / 2)
    expect = (amp * Uc).real
    assert np.abs(U1 - expect).max() <= 1e-9 * np.abs(expect).max()
    assert abs(M.wave_energy(prob, U1) / M.wave_energy(prob, U0) - 1.0) < 1e-10


def test_reflection_symmetry_of_centred_thermal():
    """Centred bubble between mirror walls: u(x) = -u(L_x - x), w, p, theta even."""
    from oracle import krylov as K
    prob = I.thermal_neutral_2d(64, 32)
    U = I.bubble_state(prob)
    for _ in range(2):
        U, info = K.newton_step(prob, U)
        assert info.converged
    umax = np.abs(U[0]).max()
    assert umax > 0
    assert np.abs(U[0] + U[0][..., ::-1]).max() <= 1e-10 * umax
    for k in (1, 2, 3):
        assert np.abs(U[k] - U[k][..., ::-1]).max() <= 1e-10 * np.abs(U[k]).max()
