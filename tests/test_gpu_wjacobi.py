"""Parity of the weighted-Jacobi smoother (the alternative smoother, weight
6/7) with the oracle, through the C ABI.

* Fixed-cycle mode in float64: forward, push-forward and pull-back equal the
  oracle's (which transposes every step literally) to 1e-12 of the largest
  entry, for V(2,2) and for V(2,1), whose transpose exchanges the smoothing
  counts; the dot-product identity holds on the GPU alone.
* Tolerance mode (float64 and float32-in-float64): residuals <= 1e-10 by the
  oracle's operator, solution and gradients against the oracle's to 1e-8.
* The concurrent forward + VJP gives the bits of the separate calls.
"""
import numpy as np
import pytest

from gpu_util import dev, host, rel_max, say

pytestmark = pytest.mark.gpu


def inputs(N, seed):
    from paper_2608_00760_amd import synth
    c = synth.grf_case(N, seed)
    c.update({k: v for k, v in synth.tangents(N, seed + 100).items() if k != "rhobar"})
    return c


def plan_for(c, **kw):
    from paper_2608_00760_amd.solver import Options, Plan
    N = c["D"].shape[0] - 1
    P = Plan(Options(N, smoother="wjacobi", **kw))
    P.set_coefficients(dev(c["D"]), dev(c["mua"]))
    return P


@pytest.mark.parametrize("N,nu2", [(16, 2), (24, 1), (64, 2)])
def test_fixed_cycles_match_oracle(N, nu2):
    from oracle import ref
    say("wjacobi fixed N=%d nu2=%d" % (N, nu2))
    c = inputs(N, 500 + N)
    n = 3
    H = ref.Hierarchy(c["D"], c["mua"], smoother="wjacobi")
    P = plan_for(c, fixed_cycles=n, nu_post=nu2)
    rho, info = P.forward(dev(c["q"]))
    rr, _ = H.forward(c["q"], fixed_cycles=n, nu2=nu2)
    assert info["cycles"] == n
    assert rel_max(host(rho), rr) <= 1e-12
    drho, _ = P.jvp(rho, dev(c["dq"]), dev(c["dlogD"]), dev(c["dlogmua"]))
    dr, _ = H.jvp(rr, c["dq"], c["dlogD"], c["dlogmua"], fixed_cycles=n, nu2=nu2)
    assert rel_max(host(drho), dr) <= 1e-12
    (qb, gD, gmu), _ = P.vjp(rho, dev(c["rhobar"]))
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], fixed_cycles=n, nu2=nu2)
    for g, r in ((qb, rqb), (gD, rgD), (gmu, rgmu)):
        assert rel_max(host(g), r) <= 1e-12
    # dot-product identity of S_n on the GPU alone: <S_n dq, w> = <dq, S_n^T w>
    P2 = plan_for(c, fixed_cycles=n, nu_post=nu2)
    s_dq, _ = P2.forward(dev(c["dq"]))
    lhs = float(np.sum(host(s_dq) * c["rhobar"]))
    rhs = float(np.sum(c["dq"][1:-1, 1:-1, 1:-1] * host(qb)[1:-1, 1:-1, 1:-1]))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(host(s_dq)) * np.linalg.norm(c["rhobar"])


@pytest.mark.parametrize("precision", ["fp64", "fp32-in-fp64"])
def test_tolerance_mode_matches_oracle(precision):
    from oracle import ref
    say("wjacobi tolerance %s" % precision)
    N = 64
    c = inputs(N, 77)
    H = ref.Hierarchy(c["D"], c["mua"], smoother="wjacobi")
    P = plan_for(c, precision=precision)
    rho, info = P.forward(dev(c["q"]))
    u = host(rho)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-10
    assert np.linalg.norm(H.defect(0, u, c["q"])) <= 1e-10 * np.linalg.norm(H.defect(0, 0 * u, c["q"]))
    rr, _ = H.forward(c["q"], rtol=1e-13, max_cycles=300)
    (qb, gD, gmu), vinfo = P.vjp(rho, dev(c["rhobar"]))
    assert vinfo["status"] == 0 and vinfo["rel_residual"] <= 1e-10
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], rtol=1e-13, max_cycles=300)
    errs = {"u": rel_max(u, rr), "q": rel_max(host(qb), rqb), "logD": rel_max(host(gD), rgD),
            "logmua": rel_max(host(gmu), rgmu)}
    say("errors", {k: "%.2e" % v for k, v in errs.items()}, "cycles", info["vcycles"], vinfo["vcycles"])
    assert max(errs.values()) <= 1e-8, errs


def test_forward_vjp_concurrent_equals_separate_calls():
    say("wjacobi forward_vjp")
    c = inputs(48, 91)
    P = plan_for(c, precision="fp32-in-fp64")
    rho, _ = P.forward(dev(c["q"]))
    (qb, gD, gmu), _ = P.vjp(rho, dev(c["rhobar"]))
    (rho2, (qb2, gD2, gmu2)), i_f, i_a = P.forward_vjp(dev(c["q"]), dev(c["rhobar"]))
    assert i_f["status"] == 0 and i_a["status"] == 0
    for a, b in ((rho, rho2), (qb, qb2), (gD, gD2), (gmu, gmu2)):
        assert bool((a == b).all())
