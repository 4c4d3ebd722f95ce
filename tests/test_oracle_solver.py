"""Pins of the oracle's GMRES, Newton and physics preconditioner: full GMRES
against a dense LU solve, residual estimates against true residuals, MGS against
CGS2, quadratic Newton convergence with exact Jacobian solves, and the
block-diagonal structure of the preconditioner (section 2.5.2)."""
import numpy as np
import pytest

from oracle import krylov as K
from oracle import model as M
from oracle import precond as PC
from paper_2007_10411_amd import inputs as I


def _tiny():
    prob = I.thermal_stable_2d(8, 4)
    U = I.smooth_flow_state(prob, seed=12, kmax=2)
    return prob, U


def test_full_gmres_equals_dense_solve():
    prob, U = _tiny()
    J = K.dense_jacobian(prob, U)
    b = I.random_vector(prob, seed=13)
    x_dense = np.linalg.solve(J, b.ravel()).reshape(b.shape)
    mv = lambda v: M.jv(prob, U, v, 0.0)
    x, info = K.fgmres(mv, lambda r: r, b, m=prob.n, tol=1e-15, max_iters=prob.n)
    cond = np.linalg.cond(J)
    assert np.linalg.norm(x - x_dense) / np.linalg.norm(x_dense) < 1e-13 * cond
    h = np.array(info.history)
    assert np.all(np.diff(h) <= 1e-12 * h[0])            # estimates never increase
    # estimate equals the true residual
    x5, i5 = K.fgmres(mv, lambda r: r, b, m=prob.n, tol=0.0, max_iters=7)
    true = np.linalg.norm(b - mv(x5))
    assert abs(i5.res_est - true) <= 1e-10 * true + 1e-14 * np.linalg.norm(b)


def test_restarted_gmres_with_preconditioner_and_orthogonalisations_agree():
    prob, U = _tiny()
    J = K.dense_jacobian(prob, U)
    b = I.random_vector(prob, seed=14)
    mv = lambda v: M.jv(prob, U, v, 0.0)
    fr = PC.frozen_coefficients(prob, U)
    pc = lambda r: PC.physics_pc(prob, U, r, 2, fr)
    xa, ia = K.fgmres(mv, pc, b, m=6, tol=0.0, max_iters=20, ortho="cgs2")
    xb, ib = K.fgmres(mv, pc, b, m=6, tol=0.0, max_iters=20, ortho="mgs")
    assert ia.restarts == 3 and ia.iters == 20
    assert np.linalg.norm(xa - xb) <= 1e-12 * np.linalg.norm(xa)
    assert abs(ia.res_est - np.linalg.norm(b.ravel() - J @ xa.ravel())) <= 1e-10 * ia.res_est + 1e-14
    # converged preconditioned solve equals the dense solution
    xc, ic = K.fgmres(mv, pc, b, m=30, tol=1e-13, max_iters=600)
    x_dense = np.linalg.solve(J, b.ravel()).reshape(b.shape)
    assert ic.converged
    assert np.linalg.norm(xc - x_dense) <= 1e-10 * np.linalg.norm(x_dense)


def test_arnoldi_relation_holds():
    """A Z_k = V_{k+1} H_k for the flexible Arnoldi process (checked on the
    unpreconditioned tiny operator through the Hessenberg the solver returns)."""
    prob, U = _tiny()
    J = K.dense_jacobian(prob, U)
    b = I.random_vector(prob, seed=15).ravel()
    k = 5
    mv = lambda v: (J @ v.ravel()).reshape(v.shape)
    x, info = K.fgmres(mv, lambda r: r, b.reshape(prob.shape), m=k, tol=0.0, max_iters=k)
    # rebuild the Krylov basis independently by Householder QR of [b, Jb, J^2 b, ...]
    Kry = np.empty((b.size, k + 1))
    v = b / np.linalg.norm(b)
    for j in range(k + 1):
        Kry[:, j] = v
        v = J @ v
        v = v / np.linalg.norm(v)
    Q, _ = np.linalg.qr(Kry)
    H = info.H
    # the Hessenberg is Q^T J Q up to column signs
    Hq = Q.T @ J @ Q[:, :k]
    assert np.allclose(np.abs(H), np.abs(Hq), atol=1e-9 * np.abs(Hq).max())


def test_newton_converges_quadratically_with_exact_solves():
    prob = I.thermal_neutral_2d(32, 16).replace(dt=20.0)
    U0 = I.bubble_state(prob)
    U0[0] = I.smooth_flow_state(prob, seed=16)[0]
    U0[1] = I.smooth_flow_state(prob, seed=16)[1]
    opts = K.NewtonOpts(rtol=1e-14, jv="analytic", forcing="fixed", eta=1e-13,
                        m=60, max_restarts=30)
    U, info = K.newton_step(prob, U0, opts)
    r = np.array(info.res)
    floor = 1e-13 * r[0]
    use = [k for k in range(len(r) - 1) if r[k + 1] > 100 * floor and r[k] < 0.5 * r[0]]
    assert len(use) >= 1, r
    for k in use:
        # r_{k+1} <= C r_k^2 with a C that does not blow up: order ~2
        order = np.log(r[k + 1] / r[0]) / np.log(r[k] / r[0])
        assert order > 1.7, (r, order)


def test_newton_step_with_stable_fd_matches_analytic_solution():
    prob = I.thermal_neutral_2d(32, 16)
    U0 = I.bubble_state(prob)
    a, ia = K.newton_step(prob, U0, K.NewtonOpts(rtol=1e-12, jv="analytic"))
    b, ib = K.newton_step(prob, U0, K.NewtonOpts(rtol=1e-12, jv="stable"))
    assert ia.converged and ib.converged
    assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(a)
    f = M.rhs(prob, U0)
    assert np.linalg.norm(M.residual(prob, b, f)) <= 1e-12 * ib.res[0] * 1.0001


def test_physics_pc_is_field_block_diagonal():
    prob = I.thermal_stable_2d(16, 8)
    U = I.smooth_flow_state(prob, seed=17)
    Z = I.random_vector(prob, seed=18)
    full = PC.apply_blocks(prob, U, Z)
    for k in range(prob.nf):
        Zk = np.zeros_like(Z)
        Zk[k] = Z[k]
        part = PC.apply_blocks(prob, U, Zk)
        others = [j for j in range(prob.nf) if j != k]
        assert np.abs(part[others]).max() == 0.0
        assert np.allclose(part[k], full[k], rtol=1e-13, atol=1e-15)


def test_physics_pc_theta_block_equals_jacobian_block_for_constant_coefficients():
    """With const-K diffusion the theta block of P(u) is exactly the theta-theta
    block of the Jacobian: 2/dt + C(a; .) - D.(K_h D .)."""
    prob = I.Problem(nx=16, nz=8, closure=0, n_bv=0.01)
    U = I.smooth_flow_state(prob, seed=19)
    Z = np.zeros(prob.shape)
    Z[3] = I.random_vector(prob, seed=20)[3]
    jz = M.jv(prob, U, Z, 0.0)
    pz = PC.apply_blocks(prob, U, Z)
    assert np.allclose(pz[3], jz[3], rtol=1e-12, atol=1e-14 * np.abs(jz[3]).max())


def test_physics_pc_sweeps_converge_to_block_inverse():
    prob = I.thermal_stable_2d(16, 8)
    U = I.smooth_flow_state(prob, seed=21, umax=2.0)
    R = I.random_vector(prob, seed=22)
    errs = []
    for s in (0, 2, 8, 40):
        z = PC.physics_pc(prob, U, R, sweeps=s)
        errs.append(np.linalg.norm(PC.apply_blocks(prob, U, z) - R) / np.linalg.norm(R))
    assert errs[1] < errs[0] and errs[2] < errs[1] and errs[3] < 1e-8, errs
