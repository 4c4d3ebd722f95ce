"""GPU parity of the learned preconditioner against the FP64 oracle network:
FP32 forward (1e-5), BF16 MFMA forward (within the BF16 rounding bound), FP32
loss and gradient, the Adam step, FGMRES with the learned preconditioner, and
what the trained network gains over the untrained (diagonal-only) form."""
import numpy as np
import pytest
import torch

from oracle import net as N
from paper_2007_10411_amd import inputs as I

from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _ctx(prob, max_m=30, dils=(1, 1, 1, 1)):
    from paper_2007_10411_amd.jfnk import Context
    c = Context(prob, max_m=max_m)
    c.net_init(dils)
    return c


def _theta(nf, seed=1):
    th = I.net_init_params(nf, seed=seed, out_scale=1.0)
    th = th + np.random.Generator(np.random.PCG64(seed + 50)).normal(scale=0.05, size=th.size)
    return th.astype(np.float32).astype(np.float64)


def _r(prob, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.normal(size=prob.shape) * np.array([1.0, 0.5, 1e-3, 2.0])[:, None, None, None]
    return r.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("dils", [(1, 1, 1, 1), (1, 2, 4, 8), (3, 8, 1, 5)])
@pytest.mark.parametrize("nx,nz", [(100, 40), (64, 8), (200, 9)])
def test_net_forward_f32_and_bf16(nx, nz, dils):
    prob = I.thermal_stable_2d(nx, nz)
    c = _ctx(prob, dils=dils)
    th = _theta(prob.nf)
    c.net_set_params(th)
    r = _r(prob, 2)
    ref = N.forward(th, r, prob.dt, dils=dils)
    netpart = ref - 0.5 * prob.dt * r
    z = dev(np.zeros(prob.shape), "f32")
    c.net_apply(dev(r, "f32"), z, bf16=False)
    gp = host(z) - 0.5 * prob.dt * r
    for k in range(prob.nf):
        e = np.linalg.norm(gp[k] - netpart[k]) / np.linalg.norm(netpart[k])
        assert e < 1e-5, ("f32", k, e)
    c.net_apply(dev(r, "f32"), z, bf16=True)
    gp = host(z) - 0.5 * prob.dt * r
    for k in range(prob.nf):
        e = np.linalg.norm(gp[k] - netpart[k]) / np.linalg.norm(netpart[k])
        # four layers of BF16 operands (8-bit significands) with FP32 accumulation
        assert e < 3e-2, ("bf16", k, e)


def test_net_forward_bf16_with_a_separate_scale_launch():
    """Above about 260 K points the input scale is finished by its own launch
    instead of inside the first layer (more partial sums than the first
    layer's blocks add themselves): the BF16 forward there against the oracle."""
    prob = I.thermal_stable_2d(600, 480)
    dils = (1, 2, 4, 8)
    c = _ctx(prob, dils=dils)
    th = _theta(prob.nf, seed=4)
    c.net_set_params(th)
    r = _r(prob, 8)
    netpart = N.forward(th, r, prob.dt, dils=dils) - 0.5 * prob.dt * r
    z = dev(np.zeros(prob.shape), "f32")
    c.net_apply(dev(r, "f32"), z, bf16=True)
    gp = host(z) - 0.5 * prob.dt * r
    for k in range(prob.nf):
        e = np.linalg.norm(gp[k] - netpart[k]) / np.linalg.norm(netpart[k])
        assert e < 3e-2, ("bf16", k, e)


@pytest.mark.parametrize("dils", [(1, 1, 1, 1), (1, 2, 4, 8), (8, 3, 1, 2)])
def test_net_loss_gradient_matches_oracle(dils):
    prob = I.thermal_stable_2d(70, 20)
    c = _ctx(prob, dils=dils)
    th = _theta(prob.nf, seed=3)
    c.net_set_params(th)
    R = [_r(prob, 4), _r(prob, 5)]
    DU = [_r(prob, 6), _r(prob, 7)]
    lo, go = N.loss_and_grad(th, R, DU, prob.dt, dils=dils)
    Rd = dev(np.stack(R), "f32")
    Dd = dev(np.stack(DU), "f32")
    lg, gg = c.net_loss_grad(Rd, Dd)
    assert abs(lg - lo) <= 1e-5 * lo
    assert np.linalg.norm(gg - go) <= 1e-4 * np.linalg.norm(go)
    # per layer as well (the small first / last layers must not hide in the norm)
    o = 0
    for ws, bs in I.net_layer_shapes(prob.nf):
        nw = int(np.prod(ws)) + int(np.prod(bs))
        sl = slice(o, o + nw)
        assert np.linalg.norm(gg[sl] - go[sl]) <= 1e-4 * np.linalg.norm(go[sl])
        o += nw


@pytest.mark.parametrize("case", ["stable", "heat_island", "periodic"])
def test_rest_jacobian_loss_gradient_matches_oracle(case):
    from oracle import model as M
    prob = {"stable": I.thermal_stable_2d(70, 20),
            "heat_island": I.heat_island_2d(96, 16),
            "periodic": I.thermal_stable_2d(64, 12).replace(bc_lateral=2)}[case]
    dils = (1, 2, 4, 1)
    c = _ctx(prob, dils=dils)
    c.net_set_loss("rest_jacobian")
    th = _theta(prob.nf, seed=3)
    c.net_set_params(th)
    R = [_r(prob, 14), _r(prob, 15)]
    DU = [_r(prob, 16), _r(prob, 17)]
    op = (lambda a: M.rest_jacobian(prob, a), lambda a: M.rest_jacobian_transpose(prob, a))
    lo, go = N.loss_and_grad(th, R, DU, prob.dt, dils=dils, op=op)
    lg, gg = c.net_loss_grad(dev(np.stack(R), "f32"), dev(np.stack(DU), "f32"))
    assert abs(lg - lo) <= 1e-5 * lo, (lg, lo)
    o = 0
    for ws, bs in I.net_layer_shapes(prob.nf):
        nw = int(np.prod(ws)) + int(np.prod(bs))
        sl = slice(o, o + nw)
        assert np.linalg.norm(gg[sl] - go[sl]) <= 1e-4 * np.linalg.norm(go[sl])
        o += nw
    # switching back restores the solution-space loss
    c.net_set_loss("solution")
    ls, _ = c.net_loss_grad(dev(np.stack(R), "f32"), dev(np.stack(DU), "f32"))
    assert abs(ls - N.loss_and_grad(th, R, DU, prob.dt, dils=dils)[0]) <= 1e-5 * ls


def test_net_adam_step_matches_oracle():
    dils = (1, 2, 4, 8)
    prob = I.thermal_stable_2d(64, 16)
    c = _ctx(prob, dils=dils)
    th = _theta(prob.nf, seed=8)
    c.net_set_params(th)
    R = [_r(prob, 9)]
    DU = [_r(prob, 10)]
    lo, go = N.loss_and_grad(th, R, DU, prob.dt, dils=dils)
    lr = 1e-3
    ref, _, _ = N.adam_step(th, go, np.zeros_like(th), np.zeros_like(th), 1, lr)
    loss = c.net_train_step(dev(R[0], "f32"), dev(DU[0], "f32"), lr)
    assert abs(loss - lo) <= 1e-5 * lo
    got = c.net_get_params().astype(np.float64)
    # first Adam step moves each weight by lr * g / (|g| + eps): compare the moves
    dg, dr = got - th, ref - th
    big = np.abs(go) > 1e-3 * np.abs(go).max()
    assert np.abs(dg[big] - dr[big]).max() <= 1e-3 * lr
    assert np.abs(dg).max() <= 1.0001 * lr


def test_net_rejects_bad_dilation():
    from paper_2007_10411_amd._lib import JfnkError
    from paper_2007_10411_amd.jfnk import Context
    c = Context(I.thermal_stable_2d(64, 8))
    for bad in [(0, 1, 1, 1), (1, 9, 1, 1)]:
        with pytest.raises(JfnkError):
            c.net_init(bad)


def test_learned_pc_in_fgmres_converges_and_falls_back():
    prob = I.thermal_stable_2d(128, 64)
    c = _ctx(prob)
    th = I.net_init_params(prob.nf, seed=0)
    c.net_set_params(th)
    U0 = I.bubble_state(prob)
    un = dev(U0)
    u = un.clone()
    r = c.newton_step(un, u, rtol=1e-8, inner="f32", pc="learned", eta_floor=1e-4, judge=False)
    assert r.converged and r.fallbacks == 0
    # two iterations cannot reach a forcing term of 1e-10: the learned solve fails
    # and is redone with the physics-based preconditioner
    u2 = un.clone()
    r2 = c.newton_step(un, u2, rtol=1e-8, inner="f32", pc="learned", forcing="fixed", eta=1e-10,
                       max_restarts=1, m=2, max_newton=1, judge=False)
    assert r2.fallbacks == 1 and not r2.converged


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("ortho", ["one_reduction", "cgs2"])
def test_learned_fgmres_fixed_iterations_vs_oracle(dim, ortho):
    """FGMRES with the learned preconditioner (BF16 network, unjudged) against
    the oracle's FGMRES with its FP64 network at a fixed 8 iterations: x per
    field within 1e-1.  The one-reduction form hands the network the input
    scale from the Arnoldi update pass's partial sums, CGS2 from its own pass;
    both form the FD step from the last layer's partial sums of ||z||^2.  A
    scale 1.5 times off moves x by about 0.3 here, BF16 rounding by about 0.01."""
    from oracle import krylov as K
    from oracle import model as M
    if dim == 2:
        prob, dils = I.thermal_stable_2d(96, 40), (1, 2, 4, 8)
        th = _theta(prob.nf)
    else:
        prob, dils = I.thermal_neutral_3d(40, 20, 18), (1, 1, 1, 1)
        th = _theta3(prob.nf)
    U = I.smooth_flow_state(prob, seed=25).astype(np.float32).astype(np.float64)
    b = I.random_vector(prob, seed=26).astype(np.float32).astype(np.float64)
    mv = lambda v: M.jv(prob, U, v, M.fd_eps(prob, U, v, eps_mach=2.0 ** -23))
    pcf = lambda r: N.forward(th, r, prob.dt, dils=dils)
    xo, io = K.fgmres(mv, pcf, b, m=8, tol=0.0, max_iters=8, ortho="cgs2")
    c = _ctx(prob, max_m=8, dils=dils)
    c.net_set_params(th)
    x = dev(np.zeros(prob.shape), "f32")
    r = c.gmres(dev(U, "f32"), dev(b, "f32"), x, m=8, max_restarts=1, tol=0.0, pc="learned", max_iters=8,
                ortho=ortho, judge=False, fallback=False)
    assert r.iters == 8 and not r.fallback
    got = host(x)
    for k in range(prob.nf):
        e = np.linalg.norm(got[k] - xo[k]) / np.linalg.norm(xo[k])
        assert e < 1e-1, (k, e)


def test_physics_preconditioner_judges_the_learned_one():
    """Section 2.5.2's preconditioner as the judge: with no physics-preconditioned
    solve on record the system goes to the physics-based preconditioner; a network
    whose residual reduction per iteration falls short of the record is stopped
    at the end of its first cycle and the rest of the step stays on the physics
    preconditioner, so the step costs at most m iterations more than the physics
    step, whose result it then equals bit for bit."""
    prob = I.thermal_stable_2d(128, 64)
    U0 = I.bubble_state(prob)
    un = dev(U0)
    m = 10
    # the step with the physics-based preconditioner alone
    cp = _ctx(prob)
    up = un.clone()
    opts = dict(rtol=1e-8, inner="f32", forcing="fixed", eta=1e-5, m=m, sweeps=0)
    rp = cp.newton_step(un, up, pc="physics", **opts)
    assert rp.converged
    # a fresh context: no record, so every solve of the first step would calibrate
    c = _ctx(prob)
    bad = I.net_init_params(prob.nf, seed=3, out_scale=30.0)
    c.net_set_params(bad)
    b = dev(np.random.Generator(np.random.PCG64(5)).normal(size=prob.shape), "f32")
    x = torch.zeros_like(b)
    g = c.gmres(dev(U0, "f32"), b, x, m=m, tol=1e-6, pc="learned", sweeps=0)
    assert g.fallback and g.converged and g.res_true > 0
    # record the physics rate, then judge the (poor) network on the same step
    u1 = un.clone()
    r1 = c.newton_step(un, u1, pc="physics", **opts)
    u2 = un.clone()
    r2 = c.newton_step(un, u2, pc="learned", **opts)
    assert r2.converged
    assert r2.fallbacks == r2.newton_iters
    # the first judged-out solve costs at most one cycle; the rest of the step
    # stays on the physics-based preconditioner
    assert rp.gmres_iters_total < r2.gmres_iters_total <= rp.gmres_iters_total + m
    assert torch.equal(u2, up) and torch.equal(u1, up)


def test_trained_network_beats_untrained_form():
    """Train on pairs the solver generates on the stable thermal (Krylov
    directions and their images, noise directions through the solver's Jv); the
    trained preconditioner needs fewer Krylov iterations per step than the same
    form with N = 0 (z = (dt/2) r, its starting point) and than the physics-based
    preconditioner."""
    from paper_2007_10411_amd import learned as LRN
    prob = I.thermal_stable_2d(256, 128)
    c = _ctx(prob)
    u0 = dev(I.bubble_state(prob))
    R, DU, u_end = LRN.collect_pairs(c, u0, steps=4, cap=256)
    assert R.shape[0] >= 64
    ntest = 16
    theta, losses = LRN.train_mixed(c, R[:-ntest], DU[:-ntest], u_end, iters=1500, lr=2e-3, batch=8)
    held = LRN.held_out_loss(c, R[-ntest:], DU[-ntest:])
    zero = np.zeros(c.n_params, dtype=np.float32)
    c.net_set_params(zero)
    held0 = LRN.held_out_loss(c, R[-ntest:], DU[-ntest:])
    assert held < 0.1 * held0

    def iters(pc, params):
        if params is not None:
            c.net_set_params(params)
        u = u_end.clone()
        tot = 0
        for _ in range(2):
            nxt = u.clone()
            res = c.newton_step(u, nxt, rtol=1e-8, inner="f32", pc=pc, eta_floor=1e-4, judge=False)
            assert res.converged and res.fallbacks == 0
            tot += res.gmres_iters_total
            u.copy_(nxt)
        return tot

    it_zero = iters("learned", zero)
    it_trained = iters("learned", theta)
    it_phys = iters("physics", None)
    print(f"GMRES iterations over 2 steps: N=0 {it_zero}, trained {it_trained}, physics {it_phys}; "
          f"held-out loss {held:.3e} (N=0 {held0:.3e}), train loss {losses[0]:.3e} -> {np.mean(losses[-20:]):.3e}")
    assert it_trained < it_zero
    assert it_trained < it_phys


# ---- 3D network (3 x 3 x 3 kernels) ---------------------------------------- #
def _r3(prob, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.normal(size=prob.shape) * np.array([1.0, 0.7, 0.5, 1e-3, 2.0])[:, None, None, None]
    return r.astype(np.float32).astype(np.float64)


def _theta3(nf, seed=1):
    th = I.net_init_params(nf, seed=seed, out_scale=1.0, dim=3)
    th = th + np.random.Generator(np.random.PCG64(seed + 50)).normal(scale=0.05, size=th.size)
    return th.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("nx,ny,nz", [(70, 9, 8), (64, 8, 8), (17, 10, 9)])
def test_net3d_forward_f32_and_bf16(nx, ny, nz):
    prob = I.thermal_neutral_3d(nx, ny, nz)
    c = _ctx(prob)
    th = _theta3(prob.nf)
    c.net_set_params(th)
    r = _r3(prob, 2)
    ref = N.forward(th, r, prob.dt)
    netpart = ref - 0.5 * prob.dt * r
    z = dev(np.zeros(prob.shape), "f32")
    for bf16, tol in [(False, 1e-5), (True, 3e-2)]:
        c.net_apply(dev(r, "f32"), z, bf16=bf16)
        gp = host(z) - 0.5 * prob.dt * r
        for k in range(prob.nf):
            e = np.linalg.norm(gp[k] - netpart[k]) / np.linalg.norm(netpart[k])
            assert e < tol, (bf16, k, e)


def test_net3d_loss_gradient_matches_oracle():
    prob = I.thermal_neutral_3d(40, 9, 8)
    c = _ctx(prob)
    th = _theta3(prob.nf, seed=3)
    c.net_set_params(th)
    R = [_r3(prob, 4), _r3(prob, 5)]
    DU = [_r3(prob, 6), _r3(prob, 7)]
    lo, go = N.loss_and_grad(th, R, DU, prob.dt)
    lg, gg = c.net_loss_grad(dev(np.stack(R), "f32"), dev(np.stack(DU), "f32"))
    assert abs(lg - lo) <= 1e-5 * lo
    o = 0
    for ws, bs in I.net_layer_shapes(prob.nf, 3):
        nw = int(np.prod(ws)) + int(np.prod(bs))
        sl = slice(o, o + nw)
        assert np.linalg.norm(gg[sl] - go[sl]) <= 1e-4 * np.linalg.norm(go[sl])
        o += nw


def test_net3d_rejects_dilation_and_rest_jacobian_loss():
    from paper_2007_10411_amd._lib import JfnkError
    from paper_2007_10411_amd.jfnk import Context
    c = Context(I.thermal_neutral_3d(16, 8, 8))
    with pytest.raises(JfnkError):
        c.net_init((1, 2, 1, 1))
    c.net_init()
    with pytest.raises(JfnkError):
        c.net_set_loss("rest_jacobian")


def test_trained_network_3d_beats_untrained_form():
    """3D thermal on a coarse grid: the trained 3x3x3 network needs fewer Krylov
    iterations per step than its untrained form z = (dt/2) r."""
    from paper_2007_10411_amd import learned as LRN
    prob = I.thermal_neutral_3d(48, 48, 24)
    c = _ctx(prob)
    u0 = dev(I.bubble_state(prob))
    R, DU, u_end = LRN.collect_pairs(c, u0, steps=3, cap=96)
    assert R.shape[0] >= 32
    theta, losses = LRN.train_mixed(c, R, DU, u_end, iters=600, lr=2e-3, batch=4, dilations=(1, 1, 1, 1))
    zero = np.zeros(c.n_params, dtype=np.float32)

    def iters(params):
        c.net_set_params(params)
        u = u_end.clone()
        tot = 0
        for _ in range(2):
            nxt = u.clone()
            res = c.newton_step(u, nxt, rtol=1e-8, inner="f32", pc="learned", eta_floor=1e-4, judge=False)
            assert res.converged and res.fallbacks == 0
            tot += res.gmres_iters_total
            u.copy_(nxt)
        return tot

    it_zero, it_trained = iters(zero), iters(theta)
    print(f"3D GMRES iterations over 2 steps: N=0 {it_zero}, trained {it_trained}; "
          f"train loss {losses[0]:.3e} -> {np.mean(losses[-20:]):.3e}")
    assert it_trained < it_zero
