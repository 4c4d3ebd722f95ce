"""Pins of the oracle's Jacobian-vector product (equation 9): the exact
directional derivative against a complex-step derivative of F (an independent
route through the residual code), the stable finite-difference form against the
literal quotient, and the O(eps) structure of the finite-difference error."""
import math

import numpy as np
import pytest

from oracle import model as M
from paper_2007_10411_amd import inputs as I


def _cases():
    return [
        ("neutral-smag", I.thermal_neutral_2d(24, 16)),
        ("stable-smag", I.thermal_stable_2d(24, 16)),
        ("island-noslip", I.heat_island_2d(32, 12, h0=400.0, width=8000.0)),
        ("constK-periodic", I.Problem(nx=20, nz=12, closure=0, bc_lateral=2, bc_vertical=2, n_bv=0.01)),
        ("3d", I.thermal_neutral_3d(12, 10, 8)),
        ("stable-smag-p3", I.thermal_stable_2d(24, 16).replace(dd_p=3)),
        ("island-noslip-p3", I.heat_island_2d(32, 12, h0=400.0, width=8000.0).replace(dd_p=3)),
        # anisotropic Eq. 7 coefficients: mixing length below the cap (N = 0.01) and at it (N = 0)
        ("deardorff-stable", I.thermal_stable_2d(24, 16).replace(closure=I.CLOSURE_DEARDORFF)),
        ("deardorff-neutral", I.thermal_neutral_2d(24, 16).replace(closure=I.CLOSURE_DEARDORFF)),
        ("deardorff-island-noslip", I.heat_island_2d(32, 12, h0=400.0, width=8000.0)
         .replace(closure=I.CLOSURE_DEARDORFF)),
        ("deardorff-3d", I.thermal_neutral_3d(12, 10, 8).replace(closure=I.CLOSURE_DEARDORFF, n_bv=0.01)),
    ]


@pytest.mark.parametrize("name,prob", _cases())
def test_analytic_jv_equals_complex_step_derivative(name, prob):
    U = I.smooth_flow_state(prob, seed=3)
    V = I.random_vector(prob, seed=4)
    h = 1e-30
    Fc = M.F(prob, U + 1j * h * V)
    dF = Fc.imag / h
    jv_cs = 2.0 * V / prob.dt - dF
    jv_an = M.jv(prob, U, V, 0.0)
    for k in range(prob.nf):
        err = np.linalg.norm(jv_an[k] - jv_cs[k]) / max(np.linalg.norm(jv_cs[k]), 1e-300)
        assert err < 1e-12, (name, k, err)


@pytest.mark.parametrize("name,prob", _cases())
def test_stable_fd_equals_literal_fd_within_rounding(name, prob):
    U = I.smooth_flow_state(prob, seed=5)
    V = I.random_vector(prob, seed=6)
    eps = M.fd_eps(prob, U, V)
    a = M.jv(prob, U, V, eps)
    b = M.jv_literal(prob, U, V, eps)
    # literal quotient carries the rounding of R amplified by 1/eps
    R = M.residual(prob, U, np.zeros(U.shape))
    bound = 64 * 2.0 ** -52 * (np.abs(R).max() + np.abs(2 * U / prob.dt).max()) / eps
    assert np.abs(a - b).max() <= bound


@pytest.mark.parametrize("name,prob", _cases())
def test_fd_error_is_first_order_in_eps(name, prob):
    """(Jv(eps) - Jv(0))/eps tends to a limit: the FD bias is linear in eps, and for
    the constant-coefficient closure (F quadratic) it is exactly linear."""
    U = I.smooth_flow_state(prob, seed=7)
    V = I.random_vector(prob, seed=8)
    j0 = M.jv(prob, U, V, 0.0)
    # F quadratic: the bias is exactly linear in eps, checked at large eps where
    # rounding (amplified by 1/eps) stays far below the bias itself
    e1, e2 = (1.0, 0.25) if prob.closure == 0 else (1e-4, 1e-5)
    d1 = (M.jv(prob, U, V, e1) - j0) / e1
    d2 = (M.jv(prob, U, V, e2) - j0) / e2
    rel = np.linalg.norm(d1 - d2) / np.linalg.norm(d2)
    if prob.closure == 0:
        assert rel < 1e-11
    else:
        assert rel < 0.2
    assert np.linalg.norm(d2) > 0


def test_literal_fd_error_has_the_v_shape():
    """Total error of the literal quotient vs eps: truncation O(eps) for large
    eps, rounding O(eps_mach/eps) for small eps, smallest near sqrt(eps_mach)."""
    prob = I.thermal_stable_2d(24, 16)
    U = I.smooth_flow_state(prob, seed=9)
    V = I.random_vector(prob, seed=10)
    j0 = M.jv(prob, U, V, 0.0)
    scale = math.sqrt(float(np.sum(U * U)))
    errs = {}
    for e in (1e-3, 1e-8, 1e-13):
        errs[e] = np.linalg.norm(M.jv_literal(prob, U, V, e * scale) - j0)
    assert errs[1e-8] < errs[1e-3] and errs[1e-8] < errs[1e-13]


def test_fd_eps_choice():
    prob = I.thermal_neutral_2d(16, 8)
    U = np.ones(prob.shape) * 0.5
    V = np.ones(prob.shape) * 2.0
    n = U.size
    e = M.fd_eps(prob, U, V)
    assert abs(e - math.sqrt(2.0 ** -52) * max(0.5 * math.sqrt(n), math.sqrt(n)) / (2.0 * math.sqrt(n))) < 1e-22
    assert M.fd_eps(prob, U, np.zeros(prob.shape)) == 0.0
