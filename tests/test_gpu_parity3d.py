"""3D GPU-vs-oracle parity through the C ABI (fields u, v, w, p', theta'):
residual / F, stable and analytic Jv, the physics preconditioner, fixed-count
GMRES and a Newton step on small ragged grids, and the residual and FP32 Jv of
the full 256 x 256 x 128 neutral thermal."""
import numpy as np
import pytest

from oracle import krylov as K
from oracle import model as M
from oracle import precond as PC
from paper_2007_10411_amd import inputs as I

from gpu_util import assert_fields_close, dev, host

pytestmark = pytest.mark.gpu

F64_TOL = 1e-11
F32_TOL = 1e-5


def _ctx(prob, max_m=30):
    from paper_2007_10411_amd.jfnk import Context
    return Context(prob, max_m=max_m)


CASES3 = {
    "neutral-3d-20x12x10": I.thermal_neutral_3d(20, 12, 10),
    "stable-noslip-3d-17x9x11": I.Problem(dim=3, nx=17, ny=9, nz=11, lx=8000.0, ly=5000.0, lz=4000.0, dt=2.0,
                                          n_bv=0.01, bc_vertical=1, h0=300.0, strip_width=3000.0,
                                          strip_center=4000.0),
    "constK-periodic-3d-12x10x8": I.Problem(dim=3, nx=12, ny=10, nz=8, ly=15000.0, closure=0, bc_lateral=2,
                                            bc_vertical=2, n_bv=0.01),
}


@pytest.mark.parametrize("name", list(CASES3))
def test_residual_and_F_3d(name):
    prob = CASES3[name]
    U = I.smooth_flow_state(prob, seed=3)
    Un = I.smooth_flow_state(prob, seed=4)
    f = M.rhs(prob, Un)
    c = _ctx(prob)
    out = dev(np.zeros(prob.shape))
    c.rhs(dev(Un), out)
    assert_fields_close(host(out), f, F64_TOL, name + " rhs")
    c.residual(dev(U), out.clone(), out)
    assert_fields_close(host(out), M.residual(prob, U, f), F64_TOL, name + " residual")
    U32 = U.astype(np.float32).astype(np.float64)
    o32 = dev(np.zeros(prob.shape), "f32")
    c.apply_F(dev(U32, "f32"), o32, what=0)
    assert_fields_close(host(o32), M.F(prob, U32), F32_TOL, name + " F32")


@pytest.mark.parametrize("name", list(CASES3))
@pytest.mark.parametrize("mode", ["stable", "analytic"])
def test_jv_3d(name, mode):
    prob = CASES3[name]
    U = I.smooth_flow_state(prob, seed=5)
    V = I.random_vector(prob, seed=6)
    eps = M.fd_eps(prob, U, V) if mode == "stable" else 0.0
    c = _ctx(prob)
    out = dev(np.zeros(prob.shape))
    c.jv(dev(U), dev(V), out, mode=mode)
    assert_fields_close(host(out), M.jv(prob, U, V, eps), F64_TOL, f"{name} jv {mode}")


@pytest.mark.parametrize("name", list(CASES3))
@pytest.mark.parametrize("sweeps", [0, 2])
def test_physics_pc_3d(name, sweeps):
    prob = CASES3[name]
    U = I.smooth_flow_state(prob, seed=7)
    R = I.random_vector(prob, seed=8)
    c = _ctx(prob)
    z = dev(np.zeros(prob.shape))
    c.precond_apply(dev(U), dev(R), z, pc="physics", sweeps=sweeps)
    assert_fields_close(host(z), PC.physics_pc(prob, U, R, sweeps=sweeps), F64_TOL, f"{name} pc{sweeps}")


@pytest.mark.parametrize("closure", [I.CLOSURE_SMAGORINSKY, I.CLOSURE_DEARDORFF])
def test_physics_pc_diagonal_3d_grid_stride(closure):
    """The preconditioner's diagonal start on 96 x 96 x 64 points (more than the
    2048 blocks x 256 threads of its grid-stride launch, so threads handle two
    points), FP64 and FP32, against the oracle."""
    prob = I.thermal_neutral_3d(96, 96, 64).replace(closure=closure, n_bv=0.01)
    assert prob.npts > 2048 * 256
    U = I.smooth_flow_state(prob, seed=17)
    R = I.random_vector(prob, seed=18)
    ref = PC.physics_pc(prob, U, R, sweeps=0)
    c = _ctx(prob, max_m=2)
    z = dev(np.zeros(prob.shape))
    c.precond_apply(dev(U), dev(R), z, pc="physics", sweeps=0)
    assert_fields_close(host(z), ref, F64_TOL, f"pc diag grid-stride closure {closure}")
    U32 = U.astype(np.float32).astype(np.float64)
    R32 = R.astype(np.float32).astype(np.float64)
    z32 = dev(np.zeros(prob.shape), "f32")
    c.precond_apply(dev(U32, "f32"), dev(R32, "f32"), z32, pc="physics", sweeps=0)
    assert_fields_close(host(z32), PC.physics_pc(prob, U32, R32, sweeps=0), F32_TOL,
                        f"pc diag grid-stride f32 closure {closure}")


@pytest.mark.parametrize("name", ["neutral-70x20x37", "noslip-stable-45x17x21", "periodic-constK-40x9x18"])
@pytest.mark.parametrize("sweeps", [1, 2])
def test_physics_pc_3d_multiblock(name, sweeps):
    """The z-marching sweep across several 32 x 8 column blocks and 16-plane
    chunks with ragged edges in every direction, FP64 and FP32."""
    prob = {"neutral-70x20x37": I.thermal_neutral_3d(70, 20, 37),
            "noslip-stable-45x17x21": I.Problem(dim=3, nx=45, ny=17, nz=21, lx=9000.0, ly=6000.0, lz=4000.0,
                                                dt=2.0, n_bv=0.01, bc_vertical=1),
            "periodic-constK-40x9x18": I.Problem(dim=3, nx=40, ny=9, nz=18, ly=15000.0, closure=0, bc_lateral=2,
                                                 bc_vertical=2, n_bv=0.01)}[name]
    U = I.smooth_flow_state(prob, seed=9)
    R = I.random_vector(prob, seed=10)
    c = _ctx(prob)
    z = dev(np.zeros(prob.shape))
    c.precond_apply(dev(U), dev(R), z, pc="physics", sweeps=sweeps)
    assert_fields_close(host(z), PC.physics_pc(prob, U, R, sweeps=sweeps), F64_TOL, f"{name} pc{sweeps}")
    U32 = U.astype(np.float32).astype(np.float64)
    R32 = R.astype(np.float32).astype(np.float64)
    z32 = dev(np.zeros(prob.shape), "f32")
    c.precond_apply(dev(U32, "f32"), dev(R32, "f32"), z32, pc="physics", sweeps=sweeps)
    assert_fields_close(host(z32), PC.physics_pc(prob, U32, R32, sweeps=sweeps), F32_TOL, f"{name} pc{sweeps} f32")


@pytest.mark.parametrize("sweeps", [2, 0])
@pytest.mark.parametrize("ortho", ["cgs2", "one_reduction"])
def test_gmres_fixed_iterations_3d(ortho, sweeps):
    prob = CASES3["neutral-3d-20x12x10"]
    U = I.smooth_flow_state(prob, seed=9)
    b = I.random_vector(prob, seed=10)
    mv = lambda v: M.jv(prob, U, v, M.fd_eps(prob, U, v))
    fr = PC.frozen_coefficients(prob, U)
    xo, io = K.fgmres(mv, lambda r: PC.physics_pc(prob, U, r, sweeps, fr), b, m=6, tol=0.0, max_iters=11,
                      ortho="cgs2")
    c = _ctx(prob, max_m=6)
    x = dev(np.zeros(prob.shape))
    r = c.gmres(dev(U), dev(b), x, m=6, max_restarts=5, tol=0.0, pc="physics", sweeps=sweeps, max_iters=11,
                want_H=True, ortho=ortho)
    assert r.iters == 11
    assert np.linalg.norm(host(x) - xo) <= F64_TOL * np.linalg.norm(xo)


def test_newton_step_3d_f64_and_mixed():
    prob = I.thermal_neutral_3d(24, 20, 16)
    U0 = I.bubble_state(prob)
    ref, info = K.newton_step(prob, U0, K.NewtonOpts(rtol=1e-13))
    c = _ctx(prob)
    un = dev(U0)
    u = un.clone()
    assert c.newton_step(un, u, rtol=1e-13).converged
    assert_fields_close(host(u), ref, F64_TOL, "newton 3d")
    u2 = un.clone()
    r2 = c.newton_step(un, u2, rtol=1e-8, inner="f32", eta_floor=1e-4)
    assert r2.converged
    d = np.linalg.norm((host(u2) - ref).ravel()) / np.linalg.norm((ref - U0).ravel())
    assert d < 1e-6


def test_full_size_3d_thermal_residual_and_jv32():
    prob = I.thermal_neutral_3d()             # 256 x 256 x 128
    U = I.bubble_state(prob)
    U[:3] = I.smooth_flow_state(prob, seed=11, kmax=4, p_std=0.0)[:3]
    c = _ctx(prob, max_m=2)
    out = dev(np.zeros(prob.shape))
    f = np.zeros(prob.shape)
    c.residual(dev(U), dev(f), out)
    assert_fields_close(host(out), M.residual(prob, U, f), F64_TOL, "C5 residual")
    del out
    U32 = U.astype(np.float32).astype(np.float64)
    V32 = I.random_vector(prob, seed=12).astype(np.float32).astype(np.float64)
    e32 = M.fd_eps(prob, U32, V32, eps_mach=2.0 ** -23)
    o32 = dev(np.zeros(prob.shape), "f32")
    c.jv(dev(U32, "f32"), dev(V32, "f32"), o32, mode="stable", eps=e32)
    assert_fields_close(host(o32), M.jv(prob, U32, V32, e32), F32_TOL, "C5 jv f32")


JV32_CASES = {
    "neutral-70x20x37": lambda: I.thermal_neutral_3d(70, 20, 37),
    "noslip-stable-flux-45x17x21": lambda: I.Problem(dim=3, nx=45, ny=17, nz=21, lx=9000.0, ly=6000.0, lz=4000.0,
                                                     dt=2.0, n_bv=0.01, bc_vertical=1, h0=300.0,
                                                     strip_width=3000.0, strip_center=4500.0),
    "periodic-constK-40x9x18": lambda: I.Problem(dim=3, nx=40, ny=9, nz=18, ly=15000.0, closure=0, bc_lateral=2,
                                                 bc_vertical=2, n_bv=0.01),
    "deardorff-stable-33x16x12": lambda: I.Problem(dim=3, nx=33, ny=16, nz=12, lx=8000.0, ly=6000.0, lz=3000.0,
                                                   dt=2.0, n_bv=0.01, closure=I.CLOSURE_DEARDORFF),
    "energy-test-no-closure-32x8x9": lambda: I.Problem(dim=3, nx=32, ny=8, nz=9, lx=8000.0, ly=4000.0, lz=3000.0,
                                                       dt=2.0, n_bv=0.01, closure=I.CLOSURE_NONE, energy_test=1),
    "no-convection-36x11x10": lambda: I.Problem(dim=3, nx=36, ny=11, nz=10, lx=8000.0, ly=4000.0, lz=3000.0,
                                                dt=2.0, n_bv=0.005, convection=0),
}


@pytest.mark.parametrize("name", list(JV32_CASES))
@pytest.mark.parametrize("mode", ["stable", "analytic"])
def test_jv32_3d_single_pass_and_two_pass(name, mode):
    """The FP32 Jv of both 3D forms (variant 7: one z-marching launch, variant 6:
    two launches with the derived components in HBM) against the FP64 oracle on
    FP32-rounded inputs, across several 32 x 16 column blocks and z chunks with
    ragged edges, every boundary kind and closure."""
    prob = JV32_CASES[name]()
    U = I.smooth_flow_state(prob, seed=21).astype(np.float32).astype(np.float64)
    V = I.random_vector(prob, seed=22).astype(np.float32).astype(np.float64)
    eps = M.fd_eps(prob, U, V, eps_mach=2.0 ** -23) if mode == "stable" else 0.0
    ref = M.jv(prob, U, V, eps)
    c = _ctx(prob, max_m=2)
    outs = []
    for variant in (7, 6):
        c.set_variant("jv", "f32", variant)
        o = dev(np.zeros(prob.shape), "f32")
        c.jv(dev(U, "f32"), dev(V, "f32"), o, mode=mode, eps=eps)
        assert_fields_close(host(o), ref, F32_TOL, f"{name} jv32 {mode} variant {variant}")
        outs.append(host(o))
    assert_fields_close(outs[0], outs[1], F32_TOL, f"{name} single vs two pass")


P3_CASES = {
    "neutral-p3-20x12x10": lambda: I.thermal_neutral_3d(20, 12, 10).replace(dd_p=3),
    "noslip-stable-flux-p3-17x9x11": lambda: CASES3["stable-noslip-3d-17x9x11"].replace(dd_p=3),
    "periodic-constK-p3-12x10x8": lambda: CASES3["constK-periodic-3d-12x10x8"].replace(dd_p=3),
    "deardorff-p3-16x9x10": lambda: I.Problem(dim=3, nx=16, ny=9, nz=10, lx=8000.0, ly=5000.0, lz=3000.0, dt=2.0,
                                              n_bv=0.01, closure=I.CLOSURE_DEARDORFF, dd_p=3),
}


@pytest.mark.parametrize("name", list(P3_CASES))
def test_p3_residual_jv_pc_3d(name):
    """The 9-point derivative (p = 3, halos of 8) in 3D: residual and F (FP64,
    FP32), stable and analytic Jv (FP64, FP32) and the physics preconditioner
    with 0 and 2 sweeps against the oracle."""
    prob = P3_CASES[name]()
    U = I.smooth_flow_state(prob, seed=13)
    Un = I.smooth_flow_state(prob, seed=14)
    f = M.rhs(prob, Un)
    c = _ctx(prob)
    out = dev(np.zeros(prob.shape))
    c.rhs(dev(Un), out)
    assert_fields_close(host(out), f, F64_TOL, name + " rhs")
    c.residual(dev(U), dev(f), out)
    assert_fields_close(host(out), M.residual(prob, U, f), F64_TOL, name + " residual")
    U32 = U.astype(np.float32).astype(np.float64)
    o32 = dev(np.zeros(prob.shape), "f32")
    c.apply_F(dev(U32, "f32"), o32, what=0)
    assert_fields_close(host(o32), M.F(prob, U32), F32_TOL, name + " F32")
    V = I.random_vector(prob, seed=15)
    V32 = V.astype(np.float32).astype(np.float64)
    for mode in ("stable", "analytic"):
        eps = M.fd_eps(prob, U, V) if mode == "stable" else 0.0
        c.jv(dev(U), dev(V), out, mode=mode)
        assert_fields_close(host(out), M.jv(prob, U, V, eps), F64_TOL, f"{name} jv {mode}")
        e32 = M.fd_eps(prob, U32, V32, eps_mach=2.0 ** -23) if mode == "stable" else 0.0
        c.jv(dev(U32, "f32"), dev(V32, "f32"), o32, mode=mode, eps=e32)
        assert_fields_close(host(o32), M.jv(prob, U32, V32, e32), F32_TOL, f"{name} jv32 {mode}")
    R = I.random_vector(prob, seed=16)
    for sweeps in (0, 2):
        z = dev(np.zeros(prob.shape))
        c.precond_apply(dev(U), dev(R), z, pc="physics", sweeps=sweeps)
        assert_fields_close(host(z), PC.physics_pc(prob, U, R, sweeps=sweeps), F64_TOL, f"{name} pc{sweeps}")


def test_p3_newton_step_3d():
    prob = I.thermal_neutral_3d(16, 12, 10).replace(dd_p=3)
    U0 = I.bubble_state(prob)
    ref, info = K.newton_step(prob, U0, K.NewtonOpts(rtol=1e-13))
    c = _ctx(prob)
    un = dev(U0)
    u = un.clone()
    assert c.newton_step(un, u, rtol=1e-13).converged
    assert_fields_close(host(u), ref, F64_TOL, "newton 3d p3")
    u2 = un.clone()
    r2 = c.newton_step(un, u2, rtol=1e-8, inner="f32", eta_floor=1e-4)
    assert r2.converged
    d = np.linalg.norm((host(u2) - ref).ravel()) / np.linalg.norm((ref - U0).ravel())
    assert d < 1e-6


def test_one_reduction_f32_256x256x128_matches_cgs2():
    """The 3D thermal at 256 x 256 x 128 (rows of 168 MB, where the one-reduction
    update pass and the cycle-end update x += Z y stream their loads and stores
    past the caches): 40 FP32 iterations (one restart) of the one-reduction step
    against CGS2 (cached accesses throughout) on the same inputs, and each
    solve's true residual ||b - J x|| against its estimate."""
    import torch
    prob = I.thermal_neutral_3d()
    U = I.bubble_state(prob)
    c = _ctx(prob, max_m=30)
    u64 = dev(U)
    f = u64.clone()
    c.rhs(u64, f)
    R = u64.clone()
    c.residual(u64, f, R)
    u32, b32 = u64.float(), (-R).float()
    del f, R
    out = {}
    for ortho in ("cgs2", "one_reduction"):
        x = torch.zeros_like(b32)
        r = c.gmres(u32, b32, x, m=30, max_restarts=5, tol=0.0, pc="physics", sweeps=0, max_iters=40,
                    ortho=ortho)
        assert r.iters == 40 and r.restarts == 1
        # x is assembled from the cycle-end updates: its true residual must match the
        # Givens estimate to the FP32 Krylov rounding
        assert r.res_true > 0 and abs(r.res_true - r.res_est) <= 2e-3 * r.res0, (ortho, r)
        out[ortho] = (x.cpu().double().numpy(), r.res_est)
        del x
    xa, ra = out["cgs2"]
    xb, rb = out["one_reduction"]
    assert np.all(np.isfinite(xb))
    assert np.linalg.norm(xb - xa) <= 1e-5 * np.linalg.norm(xa)
    assert abs(rb - ra) <= 1e-3 * ra


def test_one_reduction_f64_streaming_rows_match_cgs2():
    """FP64 rows of 42 MB (128 x 128 x 64): the one-reduction update pass and the
    cycle-end update take their streaming path in FP64 too; 40 iterations (one
    restart) against CGS2 to the FP64 bar, and the true residual against the
    estimate."""
    import torch
    prob = I.thermal_neutral_3d(128, 128, 64)
    assert prob.n * 8 >= 32 << 20
    U = I.bubble_state(prob)
    c = _ctx(prob, max_m=30)
    u64 = dev(U)
    f = u64.clone()
    c.rhs(u64, f)
    R = u64.clone()
    c.residual(u64, f, R)
    b = -R
    out = {}
    for ortho in ("cgs2", "one_reduction"):
        x = torch.zeros_like(b)
        r = c.gmres(u64, b, x, m=30, max_restarts=5, tol=0.0, pc="physics", sweeps=0, max_iters=40, ortho=ortho)
        assert r.iters == 40 and r.restarts == 1
        assert abs(r.res_true - r.res_est) <= 1e-8 * r.res0, (ortho, r)
        out[ortho] = (host(x), r.res_est)
    xa, ra = out["cgs2"]
    xb, rb = out["one_reduction"]
    assert np.linalg.norm(xb - xa) <= 1e-10 * np.linalg.norm(xa)
    assert abs(rb - ra) <= 1e-8 * ra
