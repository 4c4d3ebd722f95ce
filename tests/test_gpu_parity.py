"""GPU-vs-oracle parity of every hot-path operator through the C ABI.

Bars: FP64 kernels within 1e-11 relative 2-norm error per field of the FP64
oracle; FP32 kernels within 1e-5 of the FP64 oracle (on the same inputs, FP32
rounded on entry).  Sizes span several 64 x 8 tiles with ragged tails; the
full-size grids of the stable thermal (1024 x 512) and heat island (2048 x 256)
are compared whole because the oracle evaluates them in about a second."""
import math

import numpy as np
import pytest

from oracle import krylov as K
from oracle import model as M
from oracle import precond as PC
from paper_2007_10411_amd import inputs as I

from gpu_util import assert_fields_close, dev, field_errors, host

pytestmark = pytest.mark.gpu

F64_TOL = 1e-11
F32_TOL = 1e-5


def _ctx(prob, max_m=30):
    from paper_2007_10411_amd.jfnk import Context
    return Context(prob, max_m=max_m)


def _cases():
    return {
        "neutral-130x70": (I.thermal_neutral_2d(130, 70), 0),
        "stable-200x100": (I.thermal_stable_2d(200, 100), 1),
        "island-noslip-260x36": (I.heat_island_2d(260, 36, h0=400.0, width=8000.0), 2),
        "island-tanh-96x20": (I.heat_island_2d(96, 20, h0=300.0, width=6000.0).replace(strip_shape=1), 3),
        "constK-periodic-72x24": (I.Problem(nx=72, nz=24, closure=0, bc_lateral=2, bc_vertical=2, n_bv=0.01), 4),
        "energy-test-64x16": (I.Problem(nx=64, nz=16, closure=2, energy_test=1, n_bv=0.012), 5),
        "minimal-8x8": (I.thermal_stable_2d(8, 8), 6),
        "inviscid-lin-33x9": (I.Problem(nx=33, nz=9, closure=2, convection=0, n_bv=0.01), 7),
        # 9-point stencil (p = 3): halo 8 in LDS, stress on a ring of 4
        "stable-p3-200x100": (I.thermal_stable_2d(200, 100).replace(dd_p=3), 8),
        "island-noslip-p3-130x36": (I.heat_island_2d(130, 36, h0=400.0, width=8000.0).replace(dd_p=3), 9),
        "constK-periodic-p3-72x24": (I.Problem(nx=72, nz=24, closure=0, bc_lateral=2, bc_vertical=2, n_bv=0.01,
                                               dd_p=3), 10),
        "minimal-p3-8x9": (I.thermal_stable_2d(8, 9).replace(dd_p=3), 11),
    }


CASES = _cases()


def _state(prob, seed):
    return I.smooth_flow_state(prob, seed=seed)


@pytest.mark.parametrize("name", list(CASES))
def test_residual_f64(name):
    prob, seed = CASES[name]
    U = _state(prob, seed)
    Un = I.smooth_flow_state(prob, seed=seed + 100)
    f = M.rhs(prob, Un)
    R = M.residual(prob, U, f)
    Fo = M.F(prob, U)
    c = _ctx(prob)
    u_d, f_d = dev(U), dev(Un)
    out = dev(np.zeros(prob.shape))
    c.rhs(f_d, out)
    assert_fields_close(host(out), f, F64_TOL, name + " rhs")
    c.residual(u_d, out.clone(), out)
    assert_fields_close(host(out), R, F64_TOL, name + " residual")
    c.apply_F(u_d, out, what=0)
    assert_fields_close(host(out), Fo, F64_TOL, name + " F")


@pytest.mark.parametrize("name", list(CASES))
def test_apply_F_f32(name):
    prob, seed = CASES[name]
    U = _state(prob, seed)
    U32 = U.astype(np.float32).astype(np.float64)
    Fo = M.F(prob, U32)
    c = _ctx(prob)
    out = dev(np.zeros(prob.shape), "f32")
    c.apply_F(dev(U32, "f32"), out, what=0)
    assert_fields_close(host(out), Fo, F32_TOL, name + " F32")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("mode", ["stable", "analytic"])
def test_jv_f64(name, mode):
    prob, seed = CASES[name]
    U = _state(prob, seed)
    V = I.random_vector(prob, seed=seed + 7)
    eps = M.fd_eps(prob, U, V) if mode == "stable" else 0.0
    ref = M.jv(prob, U, V, eps)
    c = _ctx(prob)
    out = dev(np.zeros(prob.shape))
    c.jv(dev(U), dev(V), out, mode=mode, eps=0.0)           # eps chosen by the library
    assert_fields_close(host(out), ref, F64_TOL, f"{name} jv {mode}")


@pytest.mark.parametrize("name", ["neutral-130x70", "island-noslip-260x36", "stable-200x100"])
def test_jv_f32(name):
    prob, seed = CASES[name]
    U = _state(prob, seed).astype(np.float32).astype(np.float64)
    V = I.random_vector(prob, seed=seed + 7).astype(np.float32).astype(np.float64)
    eps = M.fd_eps(prob, U, V, eps_mach=2.0 ** -23)
    ref = M.jv(prob, U, V, eps)
    c = _ctx(prob)
    out = dev(np.zeros(prob.shape), "f32")
    c.jv(dev(U, "f32"), dev(V, "f32"), out, mode="stable", eps=eps)
    assert_fields_close(host(out), ref, F32_TOL, f"{name} jv f32")


def test_jv_literal_within_rounding_bound():
    prob, seed = CASES["stable-200x100"]
    U = _state(prob, seed)
    V = I.random_vector(prob, seed=3)
    eps = M.fd_eps(prob, U, V)
    ref = M.jv(prob, U, V, eps)
    c = _ctx(prob)
    out = dev(np.zeros(prob.shape))
    c.jv(dev(U), dev(V), out, mode="literal", eps=eps)
    R = M.residual(prob, U, np.zeros(U.shape))
    bound = 64 * 2.0 ** -52 * (np.abs(R).max() + np.abs(2 * U / prob.dt).max()) / eps
    assert np.abs(host(out) - ref).max() <= bound


@pytest.mark.parametrize("name", ["neutral-130x70", "stable-200x100", "island-noslip-260x36",
                                  "stable-p3-200x100", "island-noslip-p3-130x36", "constK-periodic-p3-72x24",
                                  "minimal-p3-8x9",
                                  "constK-periodic-72x24", "minimal-8x8"])
@pytest.mark.parametrize("sweeps", [0, 1, 2])
def test_physics_pc(name, sweeps):
    prob, seed = CASES[name]
    U = _state(prob, seed)
    R = I.random_vector(prob, seed=seed + 11)
    ref = PC.physics_pc(prob, U, R, sweeps=sweeps)
    c = _ctx(prob)
    z = dev(np.zeros(prob.shape))
    c.precond_apply(dev(U), dev(R), z, pc="physics", sweeps=sweeps)
    assert_fields_close(host(z), ref, F64_TOL, f"{name} pc{sweeps}")
    z32 = dev(np.zeros(prob.shape), "f32")
    U32 = U.astype(np.float32).astype(np.float64)
    R32 = R.astype(np.float32).astype(np.float64)
    ref32 = PC.physics_pc(prob, U32, R32, sweeps=sweeps)
    c.precond_apply(dev(U32, "f32"), dev(R32, "f32"), z32, pc="physics", sweeps=sweeps)
    assert_fields_close(host(z32), ref32, F32_TOL, f"{name} pc{sweeps} f32")


@pytest.mark.parametrize("ortho", ["cgs2", "one_reduction"])
@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("pc", ["physics", "physics0", "none"])
def test_gmres_fixed_iterations_f64(pc, p, ortho):
    """physics0: the preconditioner's diagonal alone (no sweeps), which the
    one-reduction form applies inside its update pass."""
    prob = I.thermal_stable_2d(96, 40).replace(dd_p=p)
    U = _state(prob, 21)
    b = I.random_vector(prob, seed=22)
    mv = lambda v: M.jv(prob, U, v, M.fd_eps(prob, U, v))
    sweeps = 0 if pc == "physics0" else 2
    if pc.startswith("physics"):
        fr = PC.frozen_coefficients(prob, U)
        pcf = lambda r: PC.physics_pc(prob, U, r, sweeps, fr)
    else:
        pcf = lambda r: r
    m, iters = 8, 19                      # two restarts and a partial cycle
    xo, io = K.fgmres(mv, pcf, b, m=m, tol=0.0, max_iters=iters, ortho="cgs2")
    c = _ctx(prob, max_m=m)
    x = dev(np.zeros(prob.shape))
    r = c.gmres(dev(U), dev(b), x, m=m, max_restarts=10, tol=0.0, pc=pc[:7] if pc != "none" else pc,
                sweeps=sweeps, max_iters=iters, want_H=True, ortho=ortho)
    assert r.iters == iters and r.restarts == io.restarts
    assert np.linalg.norm(host(x) - xo) <= F64_TOL * np.linalg.norm(xo)
    k = io.H.shape[1]
    assert np.abs(r.H[: k + 1, :k] - io.H).max() <= F64_TOL * np.abs(io.H).max()
    assert abs(r.res_est - io.res_est) <= 1e-9 * io.res_est


@pytest.mark.parametrize("ortho", ["cgs2", "one_reduction"])
@pytest.mark.parametrize("m", [1, 2])
def test_gmres_short_cycles_f64(m, ortho):
    """Restart lengths of one and two vectors: every cycle closes after one or two
    columns, so each iteration of the one-reduction form is followed at once by
    the cycle's closing reduction."""
    prob = I.thermal_stable_2d(96, 40)
    U = _state(prob, 23)
    b = I.random_vector(prob, seed=24)
    mv = lambda v: M.jv(prob, U, v, M.fd_eps(prob, U, v))
    fr = PC.frozen_coefficients(prob, U)
    pcf = lambda r: PC.physics_pc(prob, U, r, 2, fr)
    iters = 3 * m + 1
    xo, io = K.fgmres(mv, pcf, b, m=m, tol=0.0, max_iters=iters, ortho="cgs2")
    c = _ctx(prob, max_m=m)
    x = dev(np.zeros(prob.shape))
    r = c.gmres(dev(U), dev(b), x, m=m, max_restarts=20, tol=0.0, pc="physics", max_iters=iters, ortho=ortho)
    assert r.iters == iters and r.restarts == io.restarts
    assert np.linalg.norm(host(x) - xo) <= F64_TOL * np.linalg.norm(xo)
    assert abs(r.res_est - io.res_est) <= 1e-9 * io.res_est


@pytest.mark.parametrize("ortho", ["cgs2", "one_reduction"])
def test_gmres_full_cycle_of_30_f64(ortho):
    """One full cycle of m = 30: every register form of the Gram-Schmidt passes
    (up to 31 basis vectors) and the closing reduction against the oracle's CGS2."""
    prob = I.thermal_stable_2d(96, 40)
    U = _state(prob, 27)
    b = I.random_vector(prob, seed=28)
    mv = lambda v: M.jv(prob, U, v, M.fd_eps(prob, U, v))
    fr = PC.frozen_coefficients(prob, U)
    pcf = lambda r: PC.physics_pc(prob, U, r, 2, fr)
    m = iters = 30
    xo, io = K.fgmres(mv, pcf, b, m=m, tol=0.0, max_iters=iters, ortho="cgs2")
    c = _ctx(prob, max_m=m)
    x = dev(np.zeros(prob.shape))
    r = c.gmres(dev(U), dev(b), x, m=m, max_restarts=5, tol=0.0, pc="physics", max_iters=iters, want_H=True,
                ortho=ortho)
    assert r.iters == iters and r.restarts == io.restarts == 0
    assert np.linalg.norm(host(x) - xo) <= F64_TOL * np.linalg.norm(xo)
    k = io.H.shape[1]
    assert k == iters
    assert np.abs(r.H[: k + 1, :k] - io.H).max() <= F64_TOL * np.abs(io.H).max()


@pytest.mark.parametrize("ortho", ["one_reduction", "cgs2"])
@pytest.mark.parametrize("dim", [2, 3])
def test_gmres_fixed_iterations_f32_vs_oracle(dim, ortho):
    """The FP32 Krylov solve of the timed configuration (preconditioner diagonal,
    FP32 Jv with its FD step) against the oracle's FP64 CGS2 FGMRES on the same
    FP32-rounded inputs, at a fixed count of 8 iterations in one cycle: the
    solution and the Hessenberg matrix per field and entry, to the FP32 bar."""
    prob = I.thermal_stable_2d(96, 40) if dim == 2 else I.thermal_neutral_3d(40, 20, 18)
    U = I.smooth_flow_state(prob, seed=25).astype(np.float32).astype(np.float64)
    b = I.random_vector(prob, seed=26).astype(np.float32).astype(np.float64)
    mv = lambda v: M.jv(prob, U, v, M.fd_eps(prob, U, v, eps_mach=2.0 ** -23))
    fr = PC.frozen_coefficients(prob, U)
    pcf = lambda r: PC.physics_pc(prob, U, r, 0, fr)
    m = iters = 8
    xo, io = K.fgmres(mv, pcf, b, m=m, tol=0.0, max_iters=iters, ortho="cgs2")
    c = _ctx(prob, max_m=m)
    x = dev(np.zeros(prob.shape), "f32")
    r = c.gmres(dev(U, "f32"), dev(b, "f32"), x, m=m, max_restarts=1, tol=0.0, pc="physics", sweeps=0,
                max_iters=iters, want_H=True, ortho=ortho)
    assert r.iters == iters
    assert_fields_close(host(x), xo, F32_TOL, f"gmres f32 {dim}d {ortho} x")
    k = io.H.shape[1]
    assert np.abs(r.H[: k + 1, :k] - io.H).max() <= F32_TOL * np.abs(io.H).max()
    assert abs(r.res_true - np.linalg.norm(b - mv(host(x)))) <= 1e-4 * r.res0


def test_one_reduction_f32_full_size_matches_cgs2():
    """FP32 at 1024 x 512, two restarts of 30: the one-reduction step against
    CGS2 on the same inputs.  Regression test for the scale of the lagged
    basis vector, which once compounded over a cycle and overflowed the FP32
    products inside the Jv (non-finite result after 29 iterations)."""
    import torch
    prob = I.thermal_stable_2d(1024, 512)
    U = I.bubble_state(prob)
    c = _ctx(prob, max_m=30)
    u64 = dev(U)
    f = u64.clone()
    c.rhs(u64, f)
    R = u64.clone()
    c.residual(u64, f, R)
    u32, b32 = u64.float(), (-R).float()
    out = {}
    for ortho in ("cgs2", "one_reduction"):
        x = torch.zeros_like(b32)
        r = c.gmres(u32, b32, x, m=30, max_restarts=5, tol=0.0, pc="physics", sweeps=0, max_iters=70,
                    ortho=ortho)
        assert r.iters == 70 and r.restarts == 2
        out[ortho] = (host(x), r.res_est)
    xa, ra = out["cgs2"]
    xb, rb = out["one_reduction"]
    assert np.all(np.isfinite(xb))
    assert np.linalg.norm(xb - xa) <= 1e-5 * np.linalg.norm(xa)
    assert abs(rb - ra) <= 1e-3 * ra


def test_gmres_basis_beyond_32_vectors_f64():
    """One cycle of 36 iterations: the Gram-Schmidt passes run with the basis in
    registers up to 32 vectors (8-, 16- and 32-row forms) and staged in LDS
    beyond; the Hessenberg matrix matches the oracle's CGS2 column by column."""
    prob = I.thermal_stable_2d(96, 40)
    U = _state(prob, 25)
    b = I.random_vector(prob, seed=26)
    mv = lambda v: M.jv(prob, U, v, M.fd_eps(prob, U, v))
    m = iters = 36
    xo, io = K.fgmres(mv, lambda r: r, b, m=m, tol=0.0, max_iters=iters, ortho="cgs2")
    c = _ctx(prob, max_m=40)
    x = dev(np.zeros(prob.shape))
    r = c.gmres(dev(U), dev(b), x, m=40, max_restarts=1, tol=0.0, pc="none", max_iters=iters, want_H=True)
    assert r.iters == iters and r.restarts == 0
    assert np.linalg.norm(host(x) - xo) <= F64_TOL * np.linalg.norm(xo)
    k = io.H.shape[1]
    assert k == iters
    assert np.abs(r.H[: k + 1, :k] - io.H).max() <= F64_TOL * np.abs(io.H).max()


@pytest.mark.parametrize("ortho", ["cgs2", "one_reduction"])
def test_gmres_converges_and_estimate_is_true_residual(ortho):
    prob = I.thermal_neutral_2d(128, 64)
    U = _state(prob, 23)
    b = I.random_vector(prob, seed=24)
    c = _ctx(prob)
    x = dev(np.zeros(prob.shape))
    r = c.gmres(dev(U), dev(b), x, m=30, max_restarts=20, tol=1e-8, pc="physics", ortho=ortho)
    assert r.converged
    true = np.linalg.norm(M.jv(prob, U, host(x), M.fd_eps(prob, U, host(x))) - b)
    assert true <= 2e-8 * np.linalg.norm(b)


@pytest.mark.parametrize("ortho", ["cgs2", "one_reduction"])
@pytest.mark.parametrize("p", [2, 3])
def test_newton_step_f64_matches_oracle(p, ortho):
    prob = I.thermal_neutral_2d(128, 64).replace(dd_p=p)
    U0 = I.bubble_state(prob)
    ref, info = K.newton_step(prob, U0, K.NewtonOpts(rtol=1e-13))
    assert info.converged
    c = _ctx(prob)
    un = dev(U0)
    u = un.clone()
    r = c.newton_step(un, u, rtol=1e-13, ortho=ortho)
    assert r.converged
    assert_fields_close(host(u), ref, F64_TOL, "newton f64")


@pytest.mark.parametrize("ortho", ["cgs2", "one_reduction"])
def test_newton_mixed_precision_error_vs_fp64_oracle(ortho):
    """FP32 Krylov/Jv inside the FP64 Newton: converges to the same 1e-8
    tolerance; the per-field error against the FP64 oracle solution is reported
    and stays within what the tolerance allows."""
    prob = I.thermal_stable_2d(128, 64)
    U0 = I.bubble_state(prob)
    ref, info = K.newton_step(prob, U0, K.NewtonOpts(rtol=1e-12))
    c = _ctx(prob)
    un = dev(U0)
    u = un.clone()
    r = c.newton_step(un, u, rtol=1e-8, inner="f32", eta_floor=1e-4, ortho=ortho)
    assert r.converged and r.res_final <= 1e-8 * r.res0
    errs = field_errors(host(u), ref)
    step = np.array([np.linalg.norm((ref[k] - U0[k]).ravel()) for k in range(prob.nf)])
    for k, (e2, em, nr) in enumerate(errs):
        # error relative to the size of the step's change in that field
        assert e2 * nr <= 1e-5 * max(step[k], 1e-30) + 1e-12 * nr, (k, e2, step[k])


MARCH_CASES = ["neutral-130x70", "island-noslip-260x36", "constK-periodic-72x24", "energy-test-64x16",
               "minimal-8x8", "inviscid-lin-33x9", "stable-p3-200x100", "island-noslip-p3-130x36",
               "constK-periodic-p3-72x24", "minimal-p3-8x9"]


@pytest.mark.parametrize("variant", [3, 4, 5])
@pytest.mark.parametrize("name", MARCH_CASES)
def test_row_marching_residual_and_jv(name, variant):
    """The row-marching kernels (strips of 124 x 2 rows per step for FP32 with
    p = 2, (64 - 2W) x 4 otherwise, over chunks of 32, 64 or 256 rows; ragged
    strips, chunks and steps) against the oracle: F and the
    residual in FP64 and FP32, the stable Jv in FP64 and FP32."""
    prob, seed = CASES[name]
    U = _state(prob, seed)
    Un = I.smooth_flow_state(prob, seed=seed + 100)
    V = I.random_vector(prob, seed=seed + 7)
    c = _ctx(prob)
    for dt in ("f64", "f32"):
        c.set_variant("residual", dt, variant)
        c.set_variant("jv", dt, variant)
    f = M.rhs(prob, Un)
    out = dev(np.zeros(prob.shape))
    c.apply_F(dev(U), out, what=0)
    assert_fields_close(host(out), M.F(prob, U), F64_TOL, f"{name} v{variant} F")
    c.residual(dev(U), dev(f), out)
    assert_fields_close(host(out), M.residual(prob, U, f), F64_TOL, f"{name} v{variant} residual")
    c.jv(dev(U), dev(V), out, mode="stable")
    assert_fields_close(host(out), M.jv(prob, U, V, M.fd_eps(prob, U, V)), F64_TOL, f"{name} v{variant} jv")
    U32 = U.astype(np.float32).astype(np.float64)
    V32 = V.astype(np.float32).astype(np.float64)
    out32 = dev(np.zeros(prob.shape), "f32")
    c.apply_F(dev(U32, "f32"), out32, what=0)
    assert_fields_close(host(out32), M.F(prob, U32), F32_TOL, f"{name} v{variant} F32")
    e32 = M.fd_eps(prob, U32, V32, eps_mach=2.0 ** -23)
    c.jv(dev(U32, "f32"), dev(V32, "f32"), out32, mode="stable", eps=e32)
    assert_fields_close(host(out32), M.jv(prob, U32, V32, e32), F32_TOL, f"{name} v{variant} jv f32")


def test_set_variant_rejects_invalid_shapes():
    from paper_2007_10411_amd._lib import JfnkError
    c = _ctx(I.thermal_stable_2d(64, 32))
    for args in [("pc_sweep", "f32", 3), ("jv", "f64", 2), ("residual", "f64", 6), ("jv", "f32", -1)]:
        with pytest.raises(JfnkError):
            c.set_variant(*args)


@pytest.mark.parametrize("variant", [1, 4])
def test_full_size_residual_and_jv_stable_thermal(variant):
    """Tile (64 x 8) and row-marching (64 rows) kernels on the whole 1024 x 512 grid."""
    prob = I.thermal_stable_2d()          # 1024 x 512
    U = _state(prob, 31)
    V = I.random_vector(prob, seed=32)
    c = _ctx(prob, max_m=4)
    for dt in ("f64", "f32"):
        c.set_variant("residual", dt, variant)
        c.set_variant("jv", dt, variant)
    out = dev(np.zeros(prob.shape))
    f = M.rhs(prob, I.bubble_state(prob))
    c.residual(dev(U), dev(f), out)
    assert_fields_close(host(out), M.residual(prob, U, f), F64_TOL, "C2 residual")
    eps = M.fd_eps(prob, U, V)
    c.jv(dev(U), dev(V), out, mode="stable")
    assert_fields_close(host(out), M.jv(prob, U, V, eps), F64_TOL, "C2 jv")
    out32 = dev(np.zeros(prob.shape), "f32")
    U32 = U.astype(np.float32).astype(np.float64)
    V32 = V.astype(np.float32).astype(np.float64)
    e32 = M.fd_eps(prob, U32, V32, eps_mach=2.0 ** -23)
    c.jv(dev(U32, "f32"), dev(V32, "f32"), out32, mode="stable", eps=e32)
    assert_fields_close(host(out32), M.jv(prob, U32, V32, e32), F32_TOL, "C2 jv f32")


def test_full_size_heat_island_residual():
    prob = I.heat_island_2d()             # 2048 x 256, no-slip bottom, 250 W/m^2 strip
    U = _state(prob, 33)
    c = _ctx(prob, max_m=4)
    out = dev(np.zeros(prob.shape))
    f = M.rhs(prob, I.rest_state(prob))
    c.residual(dev(U), dev(f), out)
    assert_fields_close(host(out), M.residual(prob, U, f), F64_TOL, "C3 residual")


def test_rest_state_residual_is_exactly_zero():
    prob = I.thermal_stable_2d(200, 100)
    c = _ctx(prob)
    z = dev(np.zeros(prob.shape))
    f = dev(np.zeros(prob.shape))
    c.rhs(z, f)
    out = dev(np.ones(prob.shape))
    c.residual(z, f, out)
    assert np.abs(host(out)).max() == 0.0


def test_nonfinite_state_is_reported():
    from paper_2007_10411_amd import _lib as L
    prob = I.thermal_neutral_2d(64, 32)
    U = I.bubble_state(prob)
    U[3, 5, 0, 7] = np.nan
    c = _ctx(prob)
    un = dev(U)
    u = un.clone()
    with pytest.raises(L.JfnkError) as e:
        c.newton_step(un, u)
    assert e.value.code == L.JFNK_ERR_NONFINITE


def test_invalid_gmres_options_are_rejected():
    from paper_2007_10411_amd import _lib as L
    prob = I.thermal_neutral_2d(64, 32)
    c = _ctx(prob, max_m=10)
    z = dev(np.zeros(prob.shape))
    with pytest.raises(L.JfnkError) as e:
        c.gmres(z, z, z.clone(), m=11)
    assert e.value.code == L.JFNK_ERR_ARG
    # an unknown Gram-Schmidt form
    import ctypes as C
    o = L.GmresOpts(m=4, max_restarts=2, tol=1e-6, pc=L.PC_NONE, jv=L.JV_STABLE, sweeps=0, max_iters=0, ortho=7)
    info = L.GmresInfo()
    code = c.lib.jfnk_gmres(c.h, L.F64, C.c_void_p(z.data_ptr()), C.c_void_p(z.data_ptr()),
                            C.c_void_p(z.clone().data_ptr()), C.byref(o), C.byref(info))
    assert code == L.JFNK_ERR_ARG
