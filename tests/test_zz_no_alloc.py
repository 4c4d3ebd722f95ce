"""The context-free Jv entry point that allocates nothing (jfnk_jv_noalloc)
against the context entry point jfnk_jv and the FP64 oracle: two calls in a
row on one GPU, the second on a smaller problem, in 2D (p = 2 and 3) and 3D."""
import numpy as np
import pytest

from oracle import model as M
from paper_2007_10411_amd import inputs as I

from gpu_util import assert_fields_close, dev, host

pytestmark = pytest.mark.gpu

F64_TOL = 1e-11
F32_TOL = 1e-5

PAIRS = {
    "2d-p2": (lambda: I.thermal_stable_2d(1024, 512), lambda: I.thermal_stable_2d(200, 96)),
    "2d-p3-noslip": (lambda: I.heat_island_2d(512, 64).replace(dd_p=3), lambda: I.heat_island_2d(96, 40).replace(dd_p=3)),
    "3d": (lambda: I.thermal_neutral_3d(70, 20, 37), lambda: I.thermal_neutral_3d(40, 9, 18)),
}


def _inputs(prob, seed):
    U = I.smooth_flow_state(prob, seed=seed, kmax=6)
    V = I.random_vector(prob, seed=seed + 1)
    return U, V


@pytest.mark.parametrize("name", list(PAIRS))
def test_jv_noalloc_matches_context_entry_point(name):
    from paper_2007_10411_amd.jfnk import Context, jv_noalloc
    dtypes = ["f32"] if name == "3d" else ["f64", "f32"]
    for k, make in enumerate(PAIRS[name]):            # the second call is on a smaller problem
        prob = make()
        U, V = _inputs(prob, 30 + k)
        c = Context(prob, max_m=1)
        for dt in dtypes:
            tol = F32_TOL if dt == "f32" else F64_TOL
            Ur = U.astype(np.float32).astype(np.float64) if dt == "f32" else U
            Vr = V.astype(np.float32).astype(np.float64) if dt == "f32" else V
            u, v = dev(Ur, dt), dev(Vr, dt)
            for mode in ("stable", "analytic"):
                ref_ctx = dev(np.zeros(prob.shape), dt)
                c.jv(u, v, ref_ctx, mode=mode)           # automatic eps
                got = dev(np.full(prob.shape, np.nan), dt)
                jv_noalloc(prob, u, v, got, mode=mode)
                assert_fields_close(host(got), host(ref_ctx), tol, f"{name} {dt} {mode} call {k} vs jfnk_jv")
                eps = 0.0 if mode == "analytic" else M.fd_eps(prob, Ur, Vr, 2.0 ** (-23 if dt == "f32" else -52))
                assert_fields_close(host(got), M.jv(prob, Ur, Vr, eps), tol, f"{name} {dt} {mode} call {k} vs oracle")
        c.close()


def test_jv_noalloc_rejects_what_it_cannot_hold():
    import torch

    from paper_2007_10411_amd._lib import JfnkError
    from paper_2007_10411_amd.jfnk import jv_noalloc
    tall = I.thermal_stable_2d(16, 4097)
    u = torch.zeros(tall.n, dtype=torch.float64, device="cuda")
    with pytest.raises(JfnkError):
        jv_noalloc(tall, u, u, torch.empty_like(u))
    p3 = I.thermal_neutral_3d(16, 8, 8)
    u3 = torch.zeros(p3.n, dtype=torch.float64, device="cuda")
    with pytest.raises(JfnkError):                     # 3D FP64 needs a context
        jv_noalloc(p3, u3, u3, torch.empty_like(u3))
