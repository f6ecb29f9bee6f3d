"""Pull-back that repeats the forward solve's schedule (Sec. 2.4, first
stopping mode: the adjoint takes the number of cycles the forward solve took;
here it is recorded in the forward pass rather than found by a second solve).

* float64: a tolerance-mode forward solve that stopped after n cycles is
  S_n q, and the replayed pull-back is S_n^T rhobar: both equal the oracle's
  fixed-n maps to 1e-12, and <S_n q, w> = <q, S_n^T w> holds to 1e-12 on the
  GPU alone.
* float32-in-float64: the pull-back runs the forward's float32 V-cycle counts
  step for step and still meets the oracle's gradients to 1e-7.
* dmgs_forward_vjp with the option gives the bits of the separate calls; a
  pull-back on a plan with no recorded forward solve is rejected.
"""
import numpy as np
import pytest

from gpu_util import dev, host, rel_max, say

pytestmark = pytest.mark.gpu


def case(N, seed):
    from paper_2608_00760_amd import synth
    return synth.grf_case(N, seed)


def plan_for(c, **kw):
    from paper_2608_00760_amd.solver import Options, Plan
    N = c["D"].shape[0] - 1
    P = Plan(Options(N, adjoint_schedule=True, **kw))
    P.set_coefficients(dev(c["D"]), dev(c["mua"]))
    return P


@pytest.mark.parametrize("N,smoother", [(32, "rbgs"), (96, "rbgs"), (48, "wjacobi")])
def test_fp64_replay_is_exact_transpose(N, smoother):
    from oracle import ref
    say("adjoint_schedule fp64 N=%d %s" % (N, smoother))
    c = case(N, 300 + N)
    P = plan_for(c, smoother=smoother)
    rho, fi = P.forward(dev(c["q"]))
    n = fi["cycles"]
    assert fi["status"] == 0 and n >= 3
    (qb, gD, gmu), vi = P.vjp(rho, dev(c["rhobar"]))
    assert vi["cycles"] == n
    H = ref.Hierarchy(c["D"], c["mua"], smoother=smoother)
    rr, _ = H.forward(c["q"], fixed_cycles=n)
    assert rel_max(host(rho), rr) <= 1e-12
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], fixed_cycles=n)
    for g, r in ((qb, rqb), (gD, rgD), (gmu, rgmu)):
        assert rel_max(host(g), r) <= 1e-12
    # <S_n q, w> = <q, S_n^T w> over the interior (boundary values are fixed)
    q_in = dev(c["q"])[1:-1, 1:-1, 1:-1]
    lhs = float((rho * dev(c["rhobar"])).sum())
    rhs = float((q_in * qb[1:-1, 1:-1, 1:-1]).sum())
    assert abs(lhs - rhs) <= 1e-12 * float(rho.norm()) * float(np.linalg.norm(c["rhobar"]))


def test_ir_replay_matches_oracle():
    from oracle import ref
    say("adjoint_schedule fp32-in-fp64")
    N = 64
    c = case(N, 17)
    P = plan_for(c, precision="fp32-in-fp64")
    rho, fi = P.forward(dev(c["q"]))
    (qb, gD, gmu), vi = P.vjp(rho, dev(c["rhobar"]))
    say("forward", fi["cycles"], fi["vcycles"], "adjoint", vi["cycles"], vi["vcycles"], "%.2e" % vi["rel_residual"])
    assert vi["cycles"] == fi["cycles"] and vi["vcycles"] == fi["vcycles"]
    assert vi["rel_residual"] <= 1e-8
    H = ref.Hierarchy(c["D"], c["mua"])
    rr, _ = H.forward(c["q"], rtol=1e-13, max_cycles=300)
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], rtol=1e-13, max_cycles=300)
    errs = [rel_max(host(g), r) for g, r in ((qb, rqb), (gD, rgD), (gmu, rgmu))]
    say("errors", ["%.2e" % e for e in errs])
    assert max(errs) <= 1e-7


@pytest.mark.parametrize("precision", ["fp64", "fp32-in-fp64"])
def test_forward_vjp_and_errors(precision):
    from paper_2608_00760_amd import _abi
    say("adjoint_schedule forward_vjp %s" % precision)
    c = case(48, 23)
    P = plan_for(c, precision=precision)
    with pytest.raises(_abi.DMGSError) as e:
        P.vjp(dev(c["q"]), dev(c["rhobar"]))          # no forward solve recorded yet
    assert e.value.status == _abi.DMGS_ERR_INVALID
    rho, fi = P.forward(dev(c["q"]))
    (qb, gD, gmu), vi = P.vjp(rho, dev(c["rhobar"]))
    for rep in range(2):
        (rho2, (qb2, gD2, gmu2)), f2, v2 = P.forward_vjp(dev(c["q"]), dev(c["rhobar"]))
        assert f2["status"] == 0 and v2["cycles"] == f2["cycles"] == fi["cycles"]
        for a, b in ((rho, rho2), (qb, qb2), (gD, gD2), (gmu, gmu2)):
            assert bool((a == b).all()), rep
