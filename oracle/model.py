"""Spatially discrete nonhydrostatic dry model F(u), the trapezoidal residual
R(u) and the Jacobian-vector product (sections 2.1, 2.2, 2.4 and 2.5.2;
equations 1-5 and 9).

ORACLE - test infrastructure only.  Plain FP64 numpy, no blocking or fusion:
every term is formed on the whole ghost-extended grid and cropped at the end.
Nothing in the product path may import it.

Readings of points the paper leaves open (each also listed in the design notes):

* State u = (u_i, p, theta): p is the Exner perturbation p' = c_p pi', theta the
  potential-temperature perturbation.  The Exner equation (eq. 1) holds for the
  total p_bar(z) + p', which adds -w dp_bar/dz and uses (p_bar + p') in the
  divergence term; the momentum equation (eq. 2) uses grad p'.  Its coefficient is
  kappa = R/c_v (the printed c_p/c_v gives an unphysical 649 m/s sound speed for
  p = c_p pi); ``kappa_div`` overrides it.
* Hydrostatic background theta_bar = theta0 + beta z with beta = N^2 theta0/g,
  dp_bar/dz = -g/theta_bar, p_bar(0) = c_p (closed form below).
* Large-scale pressure forcing dp0/dx, dp0/dy of eq. 2 is zero.
* Skew-symmetric convection (section 2.2) for every field:
  C(a; phi) = 1/2 sum_j [ D_j(a_j phi) + a_j D_j phi ].
* Smagorinsky closure (section 2.4): nu = (C_s Delta)^2 sqrt(2 S:S),
  Delta = geometric mean of the spacings, deviatoric tau = 2 nu (S - tr(S)/3 I),
  heat flux q_j = (nu / Pr_t) D_j theta.  Divergences use the same D.
* Grid: cell centres x_i = (i + 1/2) dx; walls on the faces; fields extended by
  mirror reflection with a parity (wall-normal velocity odd; at a no-slip bottom
  the tangential velocity is odd too; p, theta even).  Ghost depth twice the
  stencil's half-width (4 for p = 2, 8 for the 9-point p = 3 stencil); derived
  quantities are formed from the extended primitives and then differentiated.
* Surface heat flux H(x) enters the first cell as Q / dz with
  Q = H / (rho0 c_p), rho0 = p_ref / (R theta0).
"""
from __future__ import annotations

import math

import numpy as np

from .stencil import deriv, stencil


def half_width(p: int) -> int:
    """Reach of the derivative stencil of order parameter p (2 for p = 2, 4 for p = 3)."""
    return len(stencil(p)[0]) // 2


def ghost(prob) -> int:
    """Ghost depth: D(2 nu S(u)) reaches twice the stencil's half-width."""
    return 2 * half_width(prob.dd_p)


# --------------------------------------------------------------------------- #
# parameters derived from the problem (background / boundary set-up)
# --------------------------------------------------------------------------- #
def kappa(prob) -> float:
    return prob.kappa_div if prob.kappa_div > 0 else prob.rgas / prob.cv


def beta(prob) -> float:
    """beta = d theta_bar / dz for a Brunt-Vaisala frequency N (N^2 = g beta / theta0)."""
    return prob.n_bv ** 2 * prob.theta0 / prob.g


def spacings(prob):
    return prob.lx / prob.nx, prob.ly / prob.ny, prob.lz / prob.nz


def z_centres(prob):
    return (np.arange(prob.nz) + 0.5) * (prob.lz / prob.nz)


def background(prob):
    """theta_bar(z), p_bar(z), dp_bar/dz(z) at the cell centres.
    Hydrostatic Exner balance dp_bar/dz = -g / theta_bar with p_bar(0) = c_p:
    p_bar = c_p - (g/beta) ln(1 + beta z / theta0)   (beta > 0)
    p_bar = c_p - g z / theta0                        (beta = 0)."""
    z = z_centres(prob)
    b = beta(prob)
    thb = prob.theta0 + b * z
    if b > 0:
        pb = prob.cp - (prob.g / b) * np.log1p(b * z / prob.theta0)
    else:
        pb = prob.cp - prob.g * z / prob.theta0
    dpb = -prob.g / thb
    return thb, pb, dpb


def surface_flux(prob):
    """Kinematic surface heat flux Q(x[, y]) [K m/s] (section 3.2 boundary
    condition).  Top-hat strip of width W, or the smooth tanh strip with the
    half-width as length unit, (H0/2)[tanh((x'+1)/xi) - tanh((x'-1)/xi)]."""
    dx, dy, _ = spacings(prob)
    x = (np.arange(prob.nx) + 0.5) * dx
    if prob.h0 == 0.0 or prob.bc_vertical == 2:
        return np.zeros((prob.ny, prob.nx))
    half = 0.5 * prob.strip_width
    if prob.strip_shape == 0:
        H = np.where(np.abs(x - prob.strip_center) <= half, prob.h0, 0.0)
    else:
        xp = (x - prob.strip_center) / half
        H = 0.5 * prob.h0 * (np.tanh((xp + 1) / prob.strip_xi) - np.tanh((xp - 1) / prob.strip_xi))
    rho0 = prob.p_ref / (prob.rgas * prob.theta0)
    Q = H / (rho0 * prob.cp)
    return np.broadcast_to(Q[None, :], (prob.ny, prob.nx)).copy()


def les_width(prob) -> float:
    dx, dy, dz = spacings(prob)
    return math.sqrt(dx * dz) if prob.dim == 2 else (dx * dy * dz) ** (1.0 / 3.0)


# --------------------------------------------------------------------------- #
# ghost extension
# --------------------------------------------------------------------------- #
def _axis_map(n, kind, s_lo, s_hi, g=4):
    """Source index and sign of every extended position -g..n+g-1."""
    e = np.arange(-g, n + g)
    if kind == 2:                               # periodic
        return e % n, np.ones(e.shape)
    src = e.copy()
    sgn = np.ones(e.shape)
    lo = e < 0
    hi = e >= n
    src[lo] = -1 - e[lo]
    sgn[lo] = s_lo
    src[hi] = 2 * n - 1 - e[hi]
    sgn[hi] = s_hi
    return src, sgn


def field_names(prob):
    return ["u", "w", "p", "theta"] if prob.dim == 2 else ["u", "v", "w", "p", "theta"]


def parities(prob, name):
    """(x_lo, x_hi), (y_lo, y_hi), (z_lo, z_hi) reflection signs of a field."""
    px = (-1, -1) if name == "u" else (1, 1)
    py = (-1, -1) if name == "v" else (1, 1)
    if name == "w":
        pz = (-1, -1)
    elif name in ("u", "v") and prob.bc_vertical == 1:
        pz = (-1, 1)                            # no-slip bottom, free-slip top
    else:
        pz = (1, 1)
    return px, py, pz


def extend(prob, a, name):
    """Ghost-extended copy of one (nz, ny, nx) field; y is not extended in 2D."""
    px, py, pz = parities(prob, name)
    g = ghost(prob)
    ix, sx = _axis_map(prob.nx, prob.bc_lateral, *px, g)
    iz, sz = _axis_map(prob.nz, prob.bc_vertical, *pz, g)
    if prob.dim == 3:
        iy, sy = _axis_map(prob.ny, prob.bc_lateral, *py, g)
    else:
        iy, sy = np.arange(prob.ny), np.ones(prob.ny)
    out = a[np.ix_(iz, iy, ix)]
    return out * sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


def interior(prob, a):
    g = ghost(prob)
    ys = slice(g, -g) if prob.dim == 3 else slice(None)
    return a[g:-g, ys, g:-g]


class _Ops:
    """Derivative operators on extended arrays (axis order z, y, x)."""

    def __init__(self, prob):
        self.prob = prob
        dx, dy, dz = spacings(prob)
        if prob.dim == 2:
            self.axes = [(2, dx), (0, dz)]          # velocity components (u, w)
        else:
            self.axes = [(2, dx), (1, dy), (0, dz)]  # (u, v, w)

    def D(self, a, j):
        ax, h = self.axes[j]
        return deriv(a, ax, h, self.prob.dd_p)


def _split(prob, U):
    nd = prob.dim
    return [U[i] for i in range(nd)], U[nd], U[nd + 1]


def _ext_state(prob, U):
    names = field_names(prob)
    E = [extend(prob, U[k], names[k]) for k in range(prob.nf)]
    nd = prob.dim
    return E[:nd], E[nd], E[nd + 1]


def convection(ops, a, phi):
    """Skew-symmetric form 1/2 sum_j [D_j(a_j phi) + a_j D_j phi]."""
    out = 0.0
    for j in range(len(a)):
        out = out + 0.5 * (ops.D(a[j] * phi, j) + a[j] * ops.D(phi, j))
    return out


def strain(ops, vel):
    nd = len(vel)
    grad = [[ops.D(vel[i], j) for j in range(nd)] for i in range(nd)]
    S = [[0.5 * (grad[i][j] + grad[j][i]) for j in range(nd)] for i in range(nd)]
    return S


def _frob(S, T):
    nd = len(S)
    return sum(S[i][j] * T[i][j] for i in range(nd) for j in range(nd))


def _trace(S):
    return sum(S[i][i] for i in range(len(S)))


def eddy_viscosity(prob, S, shape):
    """(nu for momentum, K_theta for heat) on the extended grid."""
    if prob.closure == 1:
        c = (prob.cs * les_width(prob)) ** 2
        nu = c * np.sqrt(2.0 * _frob(S, S))
        return nu, nu / prob.pr_t
    if prob.closure == 0:
        return np.full(shape, prob.k_m), np.full(shape, prob.k_h)
    return np.zeros(shape), np.zeros(shape)


def stress(S, nu):
    nd = len(S)
    tr = _trace(S)
    return [[2.0 * nu * (S[i][j] - (tr / 3.0 if i == j else 0.0)) for j in range(nd)]
            for i in range(nd)]


# --------------------------------------------------------------------------- #
# Anisotropic exchange coefficients (section 2.4, Eq. 7, after Deardorff)
# --------------------------------------------------------------------------- #
def deardorff_coefficients(prob, S):
    """Eq. 7: K_m = C_s^(4/3) eps^(1/3) (dx dy)^(2/3), K_M = C_s^(4/3) eps^(1/3) dz^(4/3)
    with eps = nu_tau S_ij S_ij, nu_tau the Smagorinsky coefficient; the heat
    coefficients K_h = (1 + 2 l / sqrt(dx dy)) K_m and K_H = (1 + 2 l / dz) K_M.
    Readings: dy = dx in 2D; l from ``mixing_length``.  Returns (K_m, K_M, K_h, K_H)."""
    dx, dy, dz = spacings(prob)
    dh2 = dx * dy if prob.dim == 3 else dx * dx
    SS = _frob(S, S)
    nu = (prob.cs * les_width(prob)) ** 2 * np.sqrt(2.0 * SS)
    eps = nu * SS
    e13 = eps ** (1.0 / 3.0)
    c43 = prob.cs ** (4.0 / 3.0)
    Km = c43 * e13 * dh2 ** (2.0 / 3.0)
    KM = c43 * e13 * dz ** (4.0 / 3.0)
    l = mixing_length(prob, eps)
    Kh = (1.0 + 2.0 * l / math.sqrt(dh2)) * Km
    KH = (1.0 + 2.0 * l / dz) * KM
    return Km, KM, Kh, KH


def mixing_length(prob, eps):
    """l = 0.75 sqrt(tau_kk) / N.  Readings: tau_kk is twice the subgrid kinetic
    energy e of local equilibrium, eps = e^(3/2) / Delta (so e = (eps Delta)^(2/3));
    N is the background Brunt-Vaisala frequency; l is capped at the filter width
    Delta, which is also its value at N = 0 (Deardorff's limit for neutral and
    unstable layers)."""
    delta = les_width(prob)
    if prob.n_bv <= 0.0:
        return np.full(np.shape(eps), delta)
    e = (eps * delta) ** (2.0 / 3.0)
    return np.minimum(0.75 * np.sqrt(2.0 * e) / prob.n_bv, delta)


def exchange_coefficients(prob, S, shape):
    """(momentum, heat) coefficients as (horizontal, vertical) pairs on the
    extended grid; the isotropic closures give the same array both ways."""
    if prob.closure == 3:
        Km, KM, Kh, KH = deardorff_coefficients(prob, S)
        return (Km, KM), (Kh, KH)
    nu, kth = eddy_viscosity(prob, S, shape)
    return (nu, nu), (kth, kth)


def stress_aniso(S, Kmom):
    """tau_ij = 2 K_ij (S_ij - delta_ij tr S / 3) with K_ij the vertical coefficient
    when i or j is the vertical axis and the horizontal one otherwise (reading of
    Eq. 7: the vertical exchange coefficient carries every flux through or along z)."""
    nd = len(S)
    tr = _trace(S)
    Kh, Kv = Kmom
    return [[2.0 * (Kv if (i == nd - 1 or j == nd - 1) else Kh) * (S[i][j] - (tr / 3.0 if i == j else 0.0))
             for j in range(nd)] for i in range(nd)]


def _axis_coeff(K, j, nd):
    return K[1] if j == nd - 1 else K[0]


def _zcol(prob, prof):
    """Broadcast a (nz,) cell-centre profile against interior arrays."""
    return prof[:, None, None]


# --------------------------------------------------------------------------- #
# F(u), eq. 4
# --------------------------------------------------------------------------- #
def F(prob, U):
    """du/dt = F(u) for the state U of shape (n_f, nz, ny, nx)."""
    ops = _Ops(prob)
    nd = prob.dim
    vel, p, th = _ext_state(prob, U)
    S = strain(ops, vel)
    Kmom, Kheat = exchange_coefficients(prob, S, p.shape)
    tau = stress_aniso(S, Kmom)
    div = _trace(S)
    conv_on = prob.convection != 0
    out = np.zeros(U.shape, dtype=U.dtype)
    I = lambda a: interior(prob, a)
    g_over = prob.g / prob.theta0
    # momentum (eq. 2)
    for i in range(nd):
        t = -prob.theta0 * ops.D(p, i)
        for j in range(nd):
            t = t + ops.D(tau[i][j], j)
        if conv_on:
            t = t - convection(ops, vel, vel[i])
        r = I(t)
        if i == nd - 1:
            r = r + g_over * U[nd + 1]
        out[i] = r
    # Exner pressure (eq. 1, total p_bar + p')
    _, pb, dpb = background(prob)
    k = kappa(prob)
    tp = I(-convection(ops, vel, p)) if conv_on else 0.0
    if prob.energy_test:
        tp = tp - k * prob.cp * I(div)
    else:
        tp = tp - U[nd - 1] * _zcol(prob, dpb) - k * (_zcol(prob, pb) + U[nd]) * I(div)
    out[nd] = tp
    # potential temperature (eq. 3)
    tt = 0.0
    for j in range(nd):
        tt = tt + ops.D(_axis_coeff(Kheat, j, nd) * ops.D(th, j), j)
    if conv_on:
        tt = tt - convection(ops, vel, th)
    tt = I(tt) - beta(prob) * U[nd - 1]
    if not prob.energy_test:
        dz = spacings(prob)[2]
        tt[0] = tt[0] + surface_flux(prob) / dz
    out[nd + 1] = tt
    return out


# --------------------------------------------------------------------------- #
# trapezoidal step, eq. 5
# --------------------------------------------------------------------------- #
def rhs(prob, Un):
    """f(u^n) = 2 u^n / dt + F(u^n)."""
    return 2.0 * Un / prob.dt + F(prob, Un)


def residual(prob, U, f):
    """R(u) = L(u) - f = 2 u / dt - F(u) - f."""
    return 2.0 * U / prob.dt - F(prob, U) - f


# --------------------------------------------------------------------------- #
# Jacobian-vector product, eq. 9
# --------------------------------------------------------------------------- #
def fd_eps(prob, U, V, eps_mach=2.0 ** -52):
    """Finite-difference step eps = sqrt(eps_mach) max(||u||, sqrt(N)) / ||v||."""
    nv = math.sqrt(float(np.sum(V * V)))
    if nv == 0.0:
        return 0.0
    nu = math.sqrt(float(np.sum(U * U)))
    return math.sqrt(eps_mach) * max(nu, math.sqrt(U.size)) / nv


def jv_literal(prob, U, V, eps, f=None):
    """[R(u + eps v) - R(u)] / eps, evaluated literally."""
    if f is None:
        f = np.zeros(U.shape)
    return (residual(prob, U + eps * V, f) - residual(prob, U, f)) / eps


def F_difference(prob, U, V, eps):
    """[F(u + eps v) - F(u)] / eps with every bilinear term expanded so that no
    two nearly equal quantities are subtracted:
      B(a+eps b, c+eps d) - B(a, c) = eps [B(a, d) + B(b, c) + eps B(b, d)].
    The eddy viscosity difference uses
      |S+eps T| - |S| = eps (2 S:T + eps T:T) / (|S+eps T| + |S|)   (0/0 -> 0).
    eps = 0 gives the exact directional derivative."""
    ops = _Ops(prob)
    nd = prob.dim
    a, pU, thU = _ext_state(prob, U)
    b, pV, thV = _ext_state(prob, V)
    SU = strain(ops, a)
    SV = strain(ops, b)
    I = lambda x: interior(prob, x)
    shape = pU.shape
    # eddy coefficients at u and their difference quotient
    KmomU, KheatU = exchange_coefficients(prob, SU, shape)
    SW = [[SU[i][j] + eps * SV[i][j] for j in range(nd)] for i in range(nd)]
    if prob.closure in (1, 3):
        magU = np.sqrt(_frob(SU, SU))
        magW = np.sqrt(_frob(SW, SW))
        num = 2.0 * _frob(SU, SV) + eps * _frob(SV, SV)
        den = magU + magW
        with np.errstate(invalid="ignore", divide="ignore"):
            dmag = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)   # (|S_W| - |S_U|) / eps
        dmag = np.where(np.isnan(den), np.nan, dmag)
    if prob.closure == 1:
        c = (prob.cs * les_width(prob)) ** 2 * math.sqrt(2.0)
        with np.errstate(invalid="ignore", divide="ignore"):
            dnu = np.where(den > 0, c * num / np.where(den > 0, den, 1.0), 0.0)
        dnu = np.where(np.isnan(den), np.nan, dnu)
        dkth = dnu / prob.pr_t
        dKmom, dKheat = (dnu, dnu), (dkth, dkth)
    elif prob.closure == 3:
        dKmom, dKheat = _deardorff_difference(prob, magU, dmag, eps)
    else:
        z = np.zeros(shape)
        dKmom, dKheat = (z, z), (z, z)
    # d tau / eps = 2 dK S_dev(u + eps v) + 2 K(u) S_dev(v)
    tW = stress_aniso(SW, dKmom)
    tV = stress_aniso(SV, KmomU)
    dtau = [[tW[i][j] + tV[i][j] for j in range(nd)] for i in range(nd)]
    conv_on = prob.convection != 0

    def dconv(phiU, phiV):
        return convection(ops, a, phiV) + convection(ops, b, phiU) + eps * convection(ops, b, phiV)

    out = np.zeros(U.shape, dtype=np.result_type(U.dtype, V.dtype))
    g_over = prob.g / prob.theta0
    for i in range(nd):
        t = -prob.theta0 * ops.D(pV, i)
        for j in range(nd):
            t = t + ops.D(dtau[i][j], j)
        if conv_on:
            t = t - dconv(a[i], b[i])
        r = I(t)
        if i == nd - 1:
            r = r + g_over * V[nd + 1]
        out[i] = r
    _, pb, dpb = background(prob)
    k = kappa(prob)
    divU = I(_trace(SU))
    divV = I(_trace(SV))
    tp = I(-dconv(pU, pV)) if conv_on else 0.0
    if prob.energy_test:
        tp = tp - k * prob.cp * divV
    else:
        tp = tp - V[nd - 1] * _zcol(prob, dpb) - k * (
            (_zcol(prob, pb) + U[nd]) * divV + V[nd] * divU + eps * V[nd] * divV)
    out[nd] = tp
    thW = thU + eps * thV
    tt = 0.0
    for j in range(nd):
        tt = tt + ops.D(_axis_coeff(dKheat, j, nd) * ops.D(thW, j) + _axis_coeff(KheatU, j, nd) * ops.D(thV, j), j)
    if conv_on:
        tt = tt - dconv(thU, thV)
    out[nd + 1] = I(tt) - beta(prob) * V[nd - 1]
    return out


def _deardorff_difference(prob, magU, dmag, eps):
    """[K(u + eps v) - K(u)] / eps of the four Eq. 7 coefficients without
    subtracting nearly equal values.  With eps^(1/3) = (C_s Delta)^(2/3) 2^(1/6) |S|
    (|S| = sqrt(S:S)) every coefficient is linear in |S| up to the mixing length:
    K_m = a_h |S|, K_M = a_v |S|, l = min(b |S|, Delta) (b = 0.75 2^(2/3) (C_s Delta)^(2/3)
    Delta^(1/3) / N), K_h = K_m + (2 a_h / sqrt(dx dy)) l |S|, and likewise K_H.
    dmag = (|S_W| - |S_U|) / eps is formed stably by the caller."""
    dx, dy, dz = spacings(prob)
    dh = math.sqrt(dx * dy if prob.dim == 3 else dx * dx)
    delta = les_width(prob)
    g = (prob.cs * delta) ** (2.0 / 3.0) * 2.0 ** (1.0 / 6.0)
    c43 = prob.cs ** (4.0 / 3.0)
    a_h = c43 * g * dh ** (4.0 / 3.0)
    a_v = c43 * g * dz ** (4.0 / 3.0)
    if prob.n_bv <= 0.0:
        lU = np.full(magU.shape, delta)
        dl = np.zeros(magU.shape)
    else:
        b = 0.75 * 2.0 ** (2.0 / 3.0) * (prob.cs * delta) ** (2.0 / 3.0) * delta ** (1.0 / 3.0) / prob.n_bv
        xU = b * magU
        lU = np.minimum(xU, delta)
        with np.errstate(invalid="ignore", divide="ignore"):
            if eps == 0.0:
                dl = np.where(xU < delta, b * dmag, np.where(xU > delta, 0.0, np.minimum(b * dmag, 0.0)))
            else:
                dl = np.where(xU >= delta, np.minimum((xU - delta) / eps + b * dmag, 0.0),
                              np.minimum(b * dmag, (delta - xU) / eps))
    lW = lU + eps * dl
    dlS = lW * dmag + magU * dl           # (l_W |S_W| - l_U |S_U|) / eps
    dKm = a_h * dmag
    dKM = a_v * dmag
    dKh = dKm + 2.0 * a_h / dh * dlS
    dKH = dKM + 2.0 * a_v / dz * dlS
    return (dKm, dKM), (dKh, dKH)


def jv(prob, U, V, eps):
    """Stable finite-difference Jv = 2 v/dt - [F(u+eps v) - F(u)]/eps (equal to
    the literal quotient in exact arithmetic); eps = 0 gives the analytic Jv."""
    return 2.0 * V / prob.dt - F_difference(prob, U, V, eps)


# --------------------------------------------------------------------------- #
# Jacobian at the state of rest without closure (acoustic-gravity operator)
# --------------------------------------------------------------------------- #
def rest_jacobian(prob, V):
    """J0 v: the Jacobian of R (eq. 5) at the state of rest (u = 0, p' = 0,
    theta' = 0) with the turbulence closure off.  There every convective
    product and the surface source drop out, leaving the acoustic-gravity
    terms of eqs. 1-3 about the hydrostatic background:
        (J0 v)_i     = 2 v_i / dt + theta0 D_i p  - delta_iz (g/theta0) theta
        (J0 v)_p     = 2 p / dt + w dp_bar/dz + kappa p_bar div v
        (J0 v)_theta = 2 theta / dt + beta w
    (v_i, p, theta the components of v)."""
    assert not prob.energy_test
    ops = _Ops(prob)
    nd = prob.dim
    names = field_names(prob)
    I = lambda a: interior(prob, a)
    _, pb, dpb = background(prob)
    k = kappa(prob)
    out = 2.0 * V / prob.dt
    pe = extend(prob, V[nd], names[nd])
    for i in range(nd):
        out[i] = out[i] + prob.theta0 * I(ops.D(pe, i))
    out[nd - 1] = out[nd - 1] - (prob.g / prob.theta0) * V[nd + 1]
    div = 0.0
    for j in range(nd):
        div = div + I(ops.D(extend(prob, V[j], names[j]), j))
    out[nd] = out[nd] + V[nd - 1] * _zcol(prob, dpb) + k * _zcol(prob, pb) * div
    out[nd + 1] = out[nd + 1] + beta(prob) * V[nd - 1]
    return out


def rest_jacobian_transpose(prob, Y):
    """J0^T y.  With mirror extension, the transpose of the derivative of a field
    of one parity is minus the derivative of a field of the opposite parity
    (fold the ghost rows back onto their sources); for the terms of J0 this is
    every field's own parity, so
        (J0^T y)_i     = 2 y_i / dt - D_i(kappa p_bar y_p) + delta_iz (dp_bar/dz y_p + beta y_theta)
        (J0^T y)_p     = 2 y_p / dt - theta0 div(y_vel)
        (J0^T y)_theta = 2 y_theta / dt - (g/theta0) y_w
    with kappa p_bar y_p extended like p (the product formed at the interior
    points, then reflected)."""
    assert not prob.energy_test
    ops = _Ops(prob)
    nd = prob.dim
    names = field_names(prob)
    I = lambda a: interior(prob, a)
    _, pb, dpb = background(prob)
    k = kappa(prob)
    out = 2.0 * Y / prob.dt
    q = extend(prob, k * _zcol(prob, pb) * Y[nd], names[nd])
    for i in range(nd):
        out[i] = out[i] - I(ops.D(q, i))
    out[nd - 1] = out[nd - 1] + _zcol(prob, dpb) * Y[nd] + beta(prob) * Y[nd + 1]
    div = 0.0
    for j in range(nd):
        div = div + I(ops.D(extend(prob, Y[j], names[j]), j))
    out[nd] = out[nd] - prob.theta0 * div
    out[nd + 1] = out[nd + 1] - (prob.g / prob.theta0) * Y[nd - 1]
    return out


# --------------------------------------------------------------------------- #
# diagnostics (section 3.1.3)
# --------------------------------------------------------------------------- #
def energies(prob, U):
    """Kinetic E_k = 1/2 int |u|^2 dV and potential E_p = int (z_max - z) theta dV."""
    dx, dy, dz = spacings(prob)
    dV = dx * dz * (dy if prob.dim == 3 else 1.0)
    nd = prob.dim
    ek = 0.5 * sum(float(np.sum(U[i] ** 2)) for i in range(nd)) * dV
    z = z_centres(prob)
    ep = float(np.sum((prob.lz - z)[:, None, None] * U[nd + 1])) * dV
    return ek, ep


def wave_energy(prob, U):
    """Quadratic energy E_W = 1/2 sum |u|^2 + 1/2 theta0/(kappa c_p) sum p'^2
    + 1/2 g/(theta0 beta) sum theta^2 conserved by the inviscid operator in the
    frozen-coefficient (energy-test) form."""
    nd = prob.dim
    k = kappa(prob)
    e = 0.5 * float(np.sum(U[:nd] ** 2))
    e += 0.5 * prob.theta0 / (k * prob.cp) * float(np.sum(U[nd] ** 2))
    b = beta(prob)
    if b > 0:
        e += 0.5 * prob.g / (prob.theta0 * b) * float(np.sum(U[nd + 1] ** 2))
    return e


def wave_energy_gradient(prob, U):
    nd = prob.dim
    k = kappa(prob)
    Gr = np.zeros(U.shape)
    Gr[:nd] = U[:nd]
    Gr[nd] = prob.theta0 / (k * prob.cp) * U[nd]
    Gr[nd + 1] = prob.g / (prob.theta0 * beta(prob)) * U[nd + 1]
    return Gr
