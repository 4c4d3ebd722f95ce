"""Constant-coefficient dry thermal (section 3.1.1, Tables 1-3): the first
implicit steps against the FP64 oracle, the diagnostics against the oracle's
energies, and the run to t = 1000 s.  The paper's extreme values come from an
unstated grid and time step, so the long runs are held to loose plausibility
only (parity unpinned): the orderings Table 2 shows across K_M, the mirror
symmetry of the centred thermal, and an approximately constant
E_k + (g/theta0) E_p (diffusion and the elastic energy of the compressible
Exner equation are outside that sum)."""
import numpy as np
import pytest

from oracle import krylov as K
from oracle import model as M
from paper_2007_10411_amd import cases as CS
from paper_2007_10411_amd import inputs as I

from gpu_util import assert_fields_close, dev, host

pytestmark = pytest.mark.gpu

F64_TOL = 1e-11


def _ctx(prob):
    from paper_2007_10411_amd.jfnk import Context
    return Context(prob, max_m=30)


def test_case_a_steps_match_oracle_and_diagnostics():
    prob = CS.case_problem(10.0, 14.1, nx=128, nz=64)
    U = I.bubble_state(prob)
    c = _ctx(prob)
    u = dev(U)
    for step in range(2):
        ref, info = K.newton_step(prob, U, K.NewtonOpts(rtol=1e-13))
        assert info.converged
        nxt = u.clone()
        r = c.newton_step(u, nxt, rtol=1e-13)
        assert r.converged
        assert_fields_close(host(nxt), ref, F64_TOL, f"case A step {step}")
        U = ref
        u = dev(ref)
    ext, ek, ep = CS.diagnostics(prob, u)
    ek_o, ep_o = M.energies(prob, U)
    assert abs(ek - ek_o) <= 1e-11 * abs(ek_o) and abs(ep - ep_o) <= 1e-11 * abs(ep_o)
    th = U[3, :, 0, :]
    assert ext["theta_max"] == pytest.approx(th.max(), rel=1e-12)


def test_case_a_to_1000s_plausibility():
    out = {}
    for km, kh in CS.CASE_A:
        prob = CS.case_problem(km, kh)
        ext, series, tot = CS.run_case(_ctx(prob), prob, t_end=1000.0, every=25)
        out[km] = (ext, series, tot)
        e = np.array([CS.total_energy(prob, s[1], s[2]) for s in series])
        print(f"K_M={km}: " + " ".join(f"{k}={v:.4f}" for k, v in ext.items()) +
              f"; E drift {abs(e[-1] - e[0]) / e[0]:.2e}; {tot['gmres_iters'] / tot['steps']:.1f} GMRES it/step, "
              f"{tot['wall_s']:.1f} s")
        # centred thermal: u antisymmetric, extremes mirrored
        assert ext["u_min"] == pytest.approx(-ext["u_max"], rel=1e-3)
        assert ext["omega_min"] == pytest.approx(-ext["omega_max"], rel=1e-3)
        # a rising thermal: up-draught stronger than the return flow, warm core kept
        assert ext["w_max"] > abs(ext["w_min"]) > 0.0
        assert 0.5 < ext["theta_max"] < 2.0 and ext["theta_min"] > -0.5
        # potential energy released into kinetic energy; total approximately constant
        ek = np.array([s[1] for s in series])
        ep = prob.g / prob.theta0 * np.array([s[2] for s in series])
        assert ep[-1] < ep[0] and ek[-1] > ek[0]
        released = ep[0] - ep.min()
        gained = ek.max() - ek[0]
        print(f"   E_k gain {gained:.3e}, (g/theta0) E_p released {released:.3e}, "
              f"max |E - E(0)| {np.max(np.abs(e - e[0])):.3e}")
        # the kinetic energy comes from the released potential energy; the two
        # agree to the compressible pressure work that the Boussinesq budget of
        # section 3.1.3 leaves out (about 28 % here, independent of K_M)
        assert 0.5 < gained / released < 2.0
    kms = [km for km, _ in CS.CASE_A]
    # Table 2's orderings: weaker diffusion keeps a warmer core, stronger updraught and vorticity
    assert all(out[a][0]["theta_max"] < out[b][0]["theta_max"] for a, b in zip(kms, kms[1:]))
    assert all(out[a][0]["w_max"] < out[b][0]["w_max"] for a, b in zip(kms, kms[1:]))
    assert all(out[a][0]["omega_max"] < out[b][0]["omega_max"] for a, b in zip(kms, kms[1:]))


def test_case_b_to_1000s_plausibility():
    """Case B (K_H = 5, Pr from 2 to 0.5): Table 3 shows the same orderings in
    K_M with smaller spread than Case A."""
    out = {}
    for km, kh in CS.CASE_B:
        prob = CS.case_problem(km, kh)
        ext, series, tot = CS.run_case(_ctx(prob), prob, t_end=1000.0, every=50)
        out[km] = ext
        print(f"K_M={km} K_H={kh}: " + " ".join(f"{k}={v:.4f}" for k, v in ext.items()))
        assert ext["u_min"] == pytest.approx(-ext["u_max"], rel=1e-3)
        assert ext["w_max"] > abs(ext["w_min"]) > 0.0
    kms = [km for km, _ in CS.CASE_B]
    assert all(out[a]["w_max"] < out[b]["w_max"] for a, b in zip(kms, kms[1:]))
    assert all(out[a]["omega_max"] < out[b]["omega_max"] for a, b in zip(kms, kms[1:]))
