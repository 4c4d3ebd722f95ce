"""Pins of the oracle's anisotropic exchange coefficients (section 2.4, Eq. 7).

Closed forms the formula must reduce to: on a grid with equal spacings the
coefficients are a fixed multiple of the Smagorinsky viscosity (the exponents
4/3 and 1/3 combine to (C_s Delta)^2 |S| 2^(1/6)); their ratio is (dz/dx)^(4/3);
the mixing length scales as |S| / N below its cap, and the heat coefficients
follow 1 + 2l/h at both ends (l = Delta at N = 0, l -> 0 for strong
stratification).  With C_s = 0 the operator is the closure-free one exactly.
The Jacobian pins (complex step, stable vs literal quotient) run with the other
closures in test_oracle_jv.py."""
import math

import numpy as np
import pytest

from oracle import model as M
from oracle import precond as PC
from paper_2007_10411_amd import inputs as I


def _strain(prob, seed):
    U = I.smooth_flow_state(prob, seed=seed)
    vel, p, th = M._ext_state(prob, U)
    return M.strain(M._Ops(prob), vel), p.shape


def test_equal_spacing_reduces_to_scaled_smagorinsky():
    # 20 km x 10 km on 64 x 32: dx = dz = 312.5 m, Delta = dx
    prob = I.thermal_stable_2d(64, 32).replace(closure=I.CLOSURE_DEARDORFF)
    S, shape = _strain(prob, 1)
    Km, KM, _, _ = M.deardorff_coefficients(prob, S)
    nu, _ = M.eddy_viscosity(prob.replace(closure=I.CLOSURE_SMAGORINSKY), S, shape)
    np.testing.assert_allclose(Km, 2.0 ** (-1.0 / 3.0) * nu, rtol=1e-13, atol=0)
    np.testing.assert_allclose(KM, Km, rtol=1e-13, atol=0)


def test_equal_spacing_3d_reduces_to_scaled_smagorinsky():
    # 20 x 20 x 10 km on 32 x 32 x 16: dx = dy = dz = 625 m
    prob = I.thermal_neutral_3d(32, 32, 16).replace(closure=I.CLOSURE_DEARDORFF, n_bv=0.01)
    S, shape = _strain(prob, 7)
    Km, KM, _, _ = M.deardorff_coefficients(prob, S)
    nu, _ = M.eddy_viscosity(prob.replace(closure=I.CLOSURE_SMAGORINSKY), S, shape)
    np.testing.assert_allclose(Km, 2.0 ** (-1.0 / 3.0) * nu, rtol=1e-13, atol=0)
    np.testing.assert_allclose(KM, Km, rtol=1e-13, atol=0)


def test_vertical_over_horizontal_is_spacing_ratio_to_four_thirds():
    prob = I.thermal_stable_2d(48, 40).replace(closure=I.CLOSURE_DEARDORFF)   # dx 417 m, dz 250 m
    S, _ = _strain(prob, 2)
    Km, KM, _, _ = M.deardorff_coefficients(prob, S)
    dx, _, dz = M.spacings(prob)
    m = Km > 0
    np.testing.assert_allclose(KM[m] / Km[m], (dz / dx) ** (4.0 / 3.0), rtol=1e-13)


def test_heat_coefficients_at_the_mixing_length_limits():
    base = I.thermal_stable_2d(48, 40).replace(closure=I.CLOSURE_DEARDORFF)
    dx, _, dz = M.spacings(base)
    delta = M.les_width(base)
    S, _ = _strain(base, 3)
    # N = 0: l = Delta
    Km, KM, Kh, KH = M.deardorff_coefficients(base.replace(n_bv=0.0), S)
    np.testing.assert_allclose(Kh, (1 + 2 * delta / dx) * Km, rtol=1e-14)
    np.testing.assert_allclose(KH, (1 + 2 * delta / dz) * KM, rtol=1e-14)
    # very strong stratification: l -> 0 and the heat coefficients approach the momentum ones
    Km, KM, Kh, KH = M.deardorff_coefficients(base.replace(n_bv=1e9), S)
    np.testing.assert_allclose(Kh, Km, rtol=1e-6)
    np.testing.assert_allclose(KH, KM, rtol=1e-6)


def test_mixing_length_scaling_below_the_cap():
    prob = I.thermal_stable_2d(48, 40).replace(closure=I.CLOSURE_DEARDORFF, n_bv=0.05)
    S, _ = _strain(prob, 4)
    SS = M._frob(S, S)
    delta = M.les_width(prob)
    eps = M.interior(prob, (prob.cs * delta) ** 2 * np.sqrt(2.0 * SS) * SS)
    l1 = M.mixing_length(prob, eps)
    assert np.all(l1 < delta) and np.all(l1 > 0)       # below the cap everywhere here
    # l is proportional to 1/N ...
    l2 = M.mixing_length(prob.replace(n_bv=0.1), eps)
    np.testing.assert_allclose(l1, 2.0 * l2, rtol=1e-14)
    # ... and to |S|: doubling the strain multiplies eps by 8
    l3 = M.mixing_length(prob, 8.0 * eps)
    np.testing.assert_allclose(l3, 2.0 * l1, rtol=1e-13)
    # the cap: a tiny N puts every point at Delta
    l4 = M.mixing_length(prob.replace(n_bv=1e-9), eps)
    np.testing.assert_array_equal(l4, np.full(l4.shape, delta))


def test_zero_constant_gives_the_closure_free_operator():
    prob = I.thermal_stable_2d(40, 24).replace(closure=I.CLOSURE_DEARDORFF, cs=0.0)
    U = I.smooth_flow_state(prob, seed=5)
    np.testing.assert_array_equal(M.F(prob, U), M.F(prob.replace(closure=I.CLOSURE_NONE), U))


def test_anisotropic_pc_diagonal_is_the_block_operator_diagonal():
    """For a uniform shear u = alpha (z - lz/2) the coefficients are constant away
    from the walls, and there the Jacobi diagonal sum_j c^2 K_j / h_j^2 of the
    anisotropic preconditioner is the exact diagonal entry of its frozen block
    operator (probed with unit vectors)."""
    prob = I.thermal_stable_2d(24, 16).replace(closure=I.CLOSURE_DEARDORFF, convection=0)
    dx, _, dz = M.spacings(prob)
    z = (np.arange(prob.nz) + 0.5) * dz
    U = np.zeros(prob.shape)
    U[0] = (2e-3 * (z - prob.lz / 2.0))[:, None, None]
    fr = PC.frozen_coefficients(prob, U)
    Km, KM = M.interior(prob, fr[1][0]), M.interior(prob, fr[1][1])
    assert Km[8, 0, 12] != KM[8, 0, 12]                     # anisotropic here
    d = PC.diagonal(prob, U, fr)
    for (k, zz, x) in [(0, 8, 12), (1, 7, 11), (3, 8, 10), (2, 6, 12)]:
        E = np.zeros(prob.shape)
        E[k, zz, 0, x] = 1.0
        P = PC.apply_blocks(prob, U, E, fr)
        assert P[k, zz, 0, x] == pytest.approx(d[k, zz, 0, x], rel=1e-12)
