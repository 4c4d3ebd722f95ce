"""Pins of the nonlinear physics-based preconditioning (section 2.5.2): R~ has
the roots of R, Newton-Krylov on R~ reaches the plain Newton solution, for a
linear operator without closure R~ is (dt/2) R exactly (the block preconditioner
is then (dt/2) I) and its finite-difference Jacobian is (dt/2) J, and the fixed
point converges linearly where the time step is small."""
import numpy as np

from oracle import krylov as K
from oracle import model as M
from oracle import nlpc as NL
from oracle import precond as PC
from paper_2007_10411_amd import inputs as I


def _nrm(a):
    return float(np.linalg.norm(a.ravel()))


def test_rtilde_vanishes_at_the_newton_solution():
    prob = I.thermal_stable_2d(16, 12)
    Un = I.bubble_state(prob)
    U, info = K.newton_step(prob, Un, K.NewtonOpts(rtol=1e-13))
    assert info.converged
    f = M.rhs(prob, Un)
    assert _nrm(NL.rtilde(prob, U, f)) <= 1e-10 * _nrm(NL.rtilde(prob, Un, f))


def test_newton_krylov_on_rtilde_reaches_the_plain_solution():
    for prob in (I.thermal_stable_2d(16, 12), I.heat_island_2d(24, 8)):
        Un = I.bubble_state(prob)
        Uref, _ = K.newton_step(prob, Un, K.NewtonOpts(rtol=1e-13))
        U, info = NL.newton_krylov_step(prob, Un, K.NewtonOpts(rtol=1e-10))
        assert info.converged and info.iters <= 8
        assert _nrm(U - Uref) <= 1e-7 * _nrm(Uref - Un)


def test_linear_operator_without_closure():
    prob = I.Problem(nx=12, nz=10, closure=2, convection=0, n_bv=0.01)
    rng = np.random.Generator(np.random.PCG64(3))
    U = rng.normal(size=prob.shape)
    f = rng.normal(size=prob.shape)
    # no diffusion and no convection: every block is (2/dt) I
    assert np.allclose(NL.rtilde(prob, U, f), 0.5 * prob.dt * M.residual(prob, U, f), rtol=1e-14, atol=1e-14)
    v = rng.normal(size=prob.shape)
    eps = M.fd_eps(prob, U, v)
    fd = (NL.rtilde(prob, U + eps * v, f) - NL.rtilde(prob, U, f)) / eps
    ref = 0.5 * prob.dt * M.jv(prob, U, v, 0.0)
    assert _nrm(fd - ref) <= 1e-6 * _nrm(ref)


def test_fixed_point_converges_for_a_small_step():
    prob = I.thermal_stable_2d(16, 12).replace(dt=0.05)
    Un = I.bubble_state(prob)
    Uref, _ = K.newton_step(prob, Un, K.NewtonOpts(rtol=1e-13))
    U, info = NL.fixed_point_step(prob, Un, rtol=1e-11, max_iter=100)
    assert info.converged
    assert _nrm(U - Uref) <= 1e-8 * _nrm(Uref - Un)
    # linear convergence: the residual contracts by a roughly constant factor
    r = np.array(info.res)
    q = r[2:] / r[1:-1]
    assert np.all(q < 0.5)
    # the preconditioner is the physics block inverse, not the identity
    fr = PC.frozen_coefficients(prob, Un)
    R = M.residual(prob, Un, M.rhs(prob, Un) + 1.0)
    assert _nrm(PC.physics_pc(prob, Un, R, 2, fr) - 0.5 * prob.dt * R) > 0.0
