"""Grouped execution (dmgs_batch_*, continuous batching) through the C ABI.

* A batch of requests on grids of several sizes (64^3 to 192^3), both
  request kinds and both face means returns, for every request, bitwise the
  results of Plan.forward followed by Plan.jvp / Plan.vjp on its plan, with
  the same refinement steps, V-cycle counts and residuals.  Requests added
  while others run, fixed-cycle plans and requests that share nothing but
  the batch are covered.  A 64^3 request is checked against the oracle's
  1e-13 solves as well (1e-8 of the largest entry, the Sec. 2.4 stopping
  rule at rtol 1e-10).
* Requests of one size run their passes in shared launches: the batch
  issues fewer launches than the requests recorded.
* More requests of one kernel than a grouped launch takes (16) are split
  over several launches; the smallest eligible grid (24^3) takes part.
* A request whose source is not finite ends with DMGS_ERR_NONFINITE, and one
  whose forward solve reaches max_cycles with DMGS_ERR_NOT_CONVERGED after
  the single call's steps; neither runs a second solve, and the others are
  unchanged.  Ineligible plans and a plan serving two requests at once are
  rejected.
"""
import numpy as np
import pytest

from gpu_util import dev, host, rel_max, say

pytestmark = pytest.mark.gpu


def make_plan(N, seed, **kw):
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.solver import Options, Plan
    c = synth.grf_case(N, seed)
    t = synth.tangents(N, seed + 50)
    P = Plan(Options(N, precision="fp32-in-fp64", **kw))
    P.set_log_coefficients(dev(c["logD"]), dev(c["logmua"]))
    return P, c, t


def solo(P, c, t, mode):
    rho, fi = P.forward(dev(c["q"]))
    if mode == "jvp":
        drho, si = P.jvp(rho, dev(t["dq"]), dev(t["dlogD"]), dev(t["dlogmua"]))
        return {"rho": rho, "drho": drho}, fi, si
    (qb, gD, gm), si = P.vjp(rho, dev(c["rhobar"]))
    return {"rho": rho, "qbar": qb, "logD_bar": gD, "logmua_bar": gm}, fi, si


def add(B, P, c, t, mode, tag):
    if mode == "jvp":
        return B.add(P, "jvp", dev(c["q"]), dq=dev(t["dq"]), dlogD=dev(t["dlogD"]), dlogmua=dev(t["dlogmua"]), tag=tag)
    return B.add(P, "vjp", dev(c["q"]), rhobar=dev(c["rhobar"]), tag=tag)


def same_info(a, b):
    return all(a[k] == b[k] for k in ("cycles", "vcycles", "rel_residual", "status"))


def check_against_solo(reqs, done):
    import torch
    assert sorted(d["tag"] for d in done) == sorted(reqs)
    for d in done:
        P, c, t, mode = reqs[d["tag"]]
        ref, fi, si = solo(P, c, t, mode)
        torch.cuda.synchronize()
        assert d["status"] == 0, d
        assert same_info(d["info_fwd"], fi) and same_info(d["info_second"], si), (d["tag"], d["info_fwd"], fi,
                                                                                 d["info_second"], si)
        for k, v in ref.items():
            assert torch.equal(d[k], v), (d["tag"], k)


SPECS = [(64, "jvp", "arith"), (96, "vjp", "arith"), (128, "jvp", "harmonic"), (64, "vjp", "harmonic"),
         (96, "jvp", "arith"), (192, "vjp", "arith"), (128, "vjp", "arith"), (64, "jvp", "arith")]


def test_batch_equals_single_requests():
    from paper_2608_00760_amd.solver import Batch
    say("batch: %d mixed requests" % len(SPECS))
    B = Batch()
    reqs = {}
    for i, (N, mode, fm) in enumerate(SPECS[:5]):
        P, c, t = make_plan(N, 12000 + 17 * i, face_mean=fm)
        reqs[i] = (P, c, t, mode)
        add(B, P, c, t, mode, i)
    done = B.tick() + B.tick()
    # three more join while the first five run
    for i, (N, mode, fm) in enumerate(SPECS[5:], start=5):
        P, c, t = make_plan(N, 12000 + 17 * i, face_mean=fm)
        reqs[i] = (P, c, t, mode)
        add(B, P, c, t, mode, i)
    done += B.run()
    st = B.stats()
    say("  ticks %d, grouped launches %d for %d recorded" % (st["ticks"], st["launches"], st["recorded"]))
    assert st["launches"] < st["recorded"]
    check_against_solo(reqs, done)


def test_fixed_cycles_and_grouping():
    from paper_2608_00760_amd.solver import Batch
    say("batch: fixed cycles, one size")
    B = Batch()
    reqs = {}
    for i in range(4):
        P, c, t = make_plan(96, 12500 + i, fixed_cycles=3)
        mode = ("jvp", "vjp")[i % 2]
        reqs[i] = (P, c, t, mode)
        add(B, P, c, t, mode, i)
    done = B.run()
    st = B.stats()
    say("  ticks %d, grouped launches %d for %d recorded" % (st["ticks"], st["launches"], st["recorded"]))
    # four same-size requests share most launches
    assert st["launches"] * 2 < st["recorded"]
    check_against_solo(reqs, done)


def test_batch_request_meets_oracle():
    from oracle import ref
    from paper_2608_00760_amd.solver import Batch
    say("batch: 64^3 requests against the oracle")
    B = Batch()
    P, c, t = make_plan(64, 12700)
    Q, c2, t2 = make_plan(64, 12701)
    B.add(P, "jvp", dev(c["q"]), dq=dev(t["dq"]), dlogD=dev(t["dlogD"]), dlogmua=dev(t["dlogmua"]), tag=1)
    B.add(Q, "vjp", dev(c2["q"]), rhobar=dev(c2["rhobar"]), tag=2)
    done = {d["tag"]: d for d in B.run()}
    H = ref.Hierarchy(c["D"], c["mua"])
    rr, _ = H.forward(c["q"], rtol=1e-13)
    dr, _ = H.jvp(rr, t["dq"], t["dlogD"], t["dlogmua"], rtol=1e-13)
    e1 = [rel_max(host(done[1]["rho"]), rr), rel_max(host(done[1]["drho"]), dr)]
    H2 = ref.Hierarchy(c2["D"], c2["mua"])
    r2, _ = H2.forward(c2["q"], rtol=1e-13)
    (qb, gD, gm), _ = H2.vjp(r2, c2["rhobar"], rtol=1e-13)
    e2 = [rel_max(host(done[2][k]), v) for k, v in (("rho", r2), ("qbar", qb), ("logD_bar", gD), ("logmua_bar", gm))]
    say("  jvp errors", ["%.1e" % e for e in e1], "vjp errors", ["%.1e" % e for e in e2])
    assert max(e1 + e2) <= 1e-8


def test_nonfinite_request_and_rejections():
    import torch
    from paper_2608_00760_amd import _abi
    from paper_2608_00760_amd.solver import Batch, Options, Plan
    say("batch: errors")
    B = Batch()
    P, c, t = make_plan(64, 12800)
    Q, c2, t2 = make_plan(96, 12801)
    q_bad = c["q"].copy()
    q_bad[10, 10, 10] = np.nan
    B.add(P, "jvp", dev(q_bad), dq=dev(t["dq"]), tag=1)
    add(B, Q, c2, t2, "vjp", 2)
    with pytest.raises(_abi.DMGSError):   # Q already serves a request
        add(B, Q, c2, t2, "jvp", 3)
    done = {d["tag"]: d for d in B.run()}
    assert done[1]["status"] == _abi.DMGS_ERR_NONFINITE and done[1]["info_second"]["cycles"] == 0
    check_against_solo({2: (Q, c2, t2, "vjp")}, [done[2]])
    from paper_2608_00760_amd import synth
    cc = synth.grf_case(64, 12900)
    for kw in ({"precision": "fp64"}, {"precision": "fp32-in-fp64", "nu_pre": 1, "nu_post": 1},
               {"precision": "fp32-in-fp64", "smoother": "wjacobi"}):
        R = Plan(Options(64, **kw))
        R.set_log_coefficients(dev(cc["logD"]), dev(cc["logmua"]))
        with pytest.raises(_abi.DMGSError):
            B.add(R, "jvp", dev(cc["q"]))
    torch.cuda.synchronize()


def test_more_requests_than_a_group_holds():
    """18 requests of one size (more than the 16 members a grouped launch
    takes) and the smallest grid grouped execution takes (24^3): every
    request still equals its single-request calls."""
    from paper_2608_00760_amd.solver import Batch
    say("batch: 18 requests of 32^3 and two of 24^3")
    B = Batch()
    reqs = {}
    for i in range(20):
        N = 32 if i < 18 else 24
        P, c, t = make_plan(N, 13000 + i, face_mean=("arith", "harmonic")[i % 2])
        mode = ("jvp", "vjp")[(i // 2) % 2]
        reqs[i] = (P, c, t, mode)
        add(B, P, c, t, mode, i)
    done = B.run()
    st = B.stats()
    say("  ticks %d, grouped launches %d for %d recorded" % (st["ticks"], st["launches"], st["recorded"]))
    assert st["launches"] * 4 < st["recorded"]
    check_against_solo(reqs, done)


def test_forward_that_does_not_converge():
    """A forward solve that reaches max_cycles ends its request with
    DMGS_ERR_NOT_CONVERGED after as many refinement steps as the single call
    takes, and no second solve runs."""
    from paper_2608_00760_amd import _abi
    from paper_2608_00760_amd.solver import Batch
    say("batch: max_cycles reached")
    B = Batch()
    P, c, t = make_plan(64, 13100, max_cycles=1)
    add(B, P, c, t, "vjp", 1)
    done = B.run()
    assert len(done) == 1 and done[0]["status"] == _abi.DMGS_ERR_NOT_CONVERGED
    assert done[0]["info_second"]["cycles"] == 0
    _, fi = P.forward(dev(c["q"]), check=False)
    assert fi["status"] == _abi.DMGS_ERR_NOT_CONVERGED
    assert done[0]["info_fwd"]["cycles"] == fi["cycles"] and done[0]["info_fwd"]["rel_residual"] == fi["rel_residual"]
