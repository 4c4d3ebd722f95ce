"""Batched ensemble (one launch per stage over all instances) against the FP64
oracle per instance: residuals to 1e-11, a mixed-precision implicit step of
uneven instances (one with the anisotropic coefficients of Eq. 7) against the
oracle's step, the 64-instance heat-island ensemble, and the autotuner's choice
not changing results."""
import time

import numpy as np
import pytest

from oracle import krylov as K
from oracle import model as M
from paper_2007_10411_amd import inputs as I

from gpu_util import assert_fields_close, dev, host

pytestmark = pytest.mark.gpu


def _small_ensemble():
    return [I.heat_island_2d(64, 16, h0=300.0, width=6000.0),
            I.thermal_stable_2d(80, 32).replace(closure=I.CLOSURE_DEARDORFF),
            I.thermal_stable_2d(96, 40),
            I.heat_island_2d(130, 24, h0=80.0, width=3000.0, n_bv=0.015),
            I.thermal_neutral_2d(72, 36),
            I.Problem(nx=40, nz=12, closure=0, bc_lateral=2, bc_vertical=2, n_bv=0.01)]


def test_batched_residual_matches_oracle():
    from paper_2007_10411_amd.jfnk import Batch
    probs = _small_ensemble()
    b = Batch(probs, max_m=8)
    states = [I.smooth_flow_state(p, seed=40 + i) for i, p in enumerate(probs)]
    prev = [I.smooth_flow_state(p, seed=60 + i) for i, p in enumerate(probs)]
    u = b.pack(states)
    un = b.pack(prev)
    f = un.clone()
    b.apply_F(un, f, what=1)
    R = f.clone()
    b.apply_F(u, R, what=2, f=f)
    got = b.unpack(R)
    for i, p in enumerate(probs):
        ref = M.residual(p, states[i], M.rhs(p, prev[i]))
        assert_fields_close(got[i], ref, 1e-11, f"batch residual {i}")


@pytest.mark.parametrize("ortho,m", [("cgs2", 30), ("one_reduction", 30), ("one_reduction", 6)])
def test_batched_step_matches_oracle_steps(ortho, m):
    """m = 6 forces restarts (and closing reductions) inside the lockstep loop."""
    from paper_2007_10411_amd.jfnk import Batch
    probs = _small_ensemble()[:4]
    b = Batch(probs, max_m=30)
    U0 = [I.bubble_state(p) if p.h0 == 0 else I.rest_state(p) for p in probs]
    un = b.pack(U0)
    u = un.clone()
    res = b.newton_step(un, u, rtol=1e-10, ortho=ortho, m=m, max_restarts=100)
    assert all(r.converged for r in res), res
    got = b.unpack(u)
    for i, p in enumerate(probs):
        ref, info = K.newton_step(p, U0[i], K.NewtonOpts(rtol=1e-12))
        d = np.linalg.norm((got[i] - ref).ravel()) / np.linalg.norm((ref - U0[i]).ravel())
        assert d < 1e-7, (i, d)


def test_heat_island_ensemble_64_instances():
    from paper_2007_10411_amd.jfnk import Batch
    import torch
    probs = I.heat_island_ensemble(64, seed=0)
    b = Batch(probs, max_m=30)
    rows = b.tune()
    U0 = [I.rest_state(p) for p in probs]
    un = b.pack(U0)
    u = un.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = b.newton_step(un, u)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert all(r.converged for r in res)
    npts = sum(p.npts for p in probs)
    print(f"64-instance heat-island ensemble ({npts} points): one mixed step {el*1e3:.1f} ms, tiles {rows}, "
          f"GMRES iterations per instance {min(r.gmres_iters_total for r in res)}.."
          f"{max(r.gmres_iters_total for r in res)}")
    # spot-check two instances against the oracle's residual at the batch's answer
    got = b.unpack(u)
    for i in (0, 37):
        p = probs[i]
        R = M.residual(p, got[i], M.rhs(p, U0[i]))
        assert np.linalg.norm(R) <= 2e-8 * np.linalg.norm(M.residual(p, U0[i], M.rhs(p, U0[i])))
