"""End-to-end parity of forward, push-forward and pull-back with the oracle.

* Fixed-cycle mode (Sec. 2.4, second mode) in float64: the GPU and the oracle
  apply the same linear map S_n and its transpose, so solutions and all
  gradients agree to 1e-12 of the largest entry, and the dot-product identity
  <JVP, w> = <v, VJP> holds to 1e-12 on the GPU alone.
* Tolerance mode: every GPU solution has relative residual <= 1e-10 as
  evaluated by the oracle's operator, and the gradients agree with the
  oracle's (solved to 1e-13) to 1e-8 relative (both float64 and
  float32-in-float64).
* Closed form: the 32^3 constant-coefficient workload against the DST-I
  solution.
"""
import numpy as np
import pytest

from gpu_util import dev, host, rel_max, say

pytestmark = pytest.mark.gpu


def plan_for(D, mu, **kw):
    from paper_2608_00760_amd.solver import Options, Plan
    N = D.shape[0] - 1
    P = Plan(Options(N, **kw))
    P.set_coefficients(dev(D), dev(mu))
    return P


def rel_residual(H, u, q, bc=0.0):
    N = H.N
    r = H.defect(0, u, q)
    u0 = np.zeros_like(u)
    u0[[0, -1], :, :] = bc; u0[:, [0, -1], :] = bc; u0[:, :, [0, -1]] = bc
    return np.linalg.norm(r) / np.linalg.norm(H.defect(0, u0, q))


def grf_inputs(N, seed):
    from paper_2608_00760_amd import synth
    c = synth.grf_case(N, seed)
    c.update({k: v for k, v in synth.tangents(N, seed + 100).items() if k != "rhobar"})
    return c


@pytest.mark.parametrize("N,n", [(8, 4), (32, 15), (24, 6), (96, 5), (128, 4)])
@pytest.mark.parametrize("face_mean", ["arith", "harmonic"])
def test_fixed_cycles_forward_jvp_vjp(N, n, face_mean):
    from oracle import ref
    say("fixed N=%d n=%d %s" % (N, n, face_mean))
    c = grf_inputs(N, 100 * N)
    H = ref.Hierarchy(c["D"], c["mua"], face_mean=face_mean)
    P = plan_for(c["D"], c["mua"], fixed_cycles=n, face_mean=face_mean)
    rho, info = P.forward(dev(c["q"]))
    rr, _ = H.forward(c["q"], fixed_cycles=n)
    assert info["cycles"] == n
    assert rel_max(host(rho), rr) <= 1e-12
    drho, _ = P.jvp(rho, dev(c["dq"]), dev(c["dlogD"]), dev(c["dlogmua"]))
    dr, _ = H.jvp(rr, c["dq"], c["dlogD"], c["dlogmua"], fixed_cycles=n)
    assert rel_max(host(drho), dr) <= 1e-12
    (qb, gD, gmu), _ = P.vjp(rho, dev(c["rhobar"]))
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], fixed_cycles=n)
    assert rel_max(host(qb), rqb) <= 1e-12
    assert rel_max(host(gD), rgD) <= 1e-12
    assert rel_max(host(gmu), rgmu) <= 1e-12
    # dot-product identity on the GPU alone
    lhs = float((drho * dev(c["rhobar"])).sum())
    rhs = float((dev(c["dq"]) * qb).sum() + (dev(c["dlogD"]) * gD).sum() + (dev(c["dlogmua"]) * gmu).sum())
    assert abs(lhs - rhs) <= 1e-12 * float(drho.norm()) * float(np.linalg.norm(c["rhobar"]))


def test_small_constant_workload_closed_form():
    """32^3, D = 1, mua = 0.1, centred blob; one JVP and one VJP."""
    from oracle import ref
    from paper_2608_00760_amd import synth
    from test_oracle_closed_form import dst_solve
    say("small constant workload")
    c = synth.small_constant()
    H = ref.Hierarchy(c["D"], c["mua"])
    P = plan_for(c["D"], c["mua"])
    rho, info = P.forward(dev(c["q"]))
    u = host(rho)
    assert info["rel_residual"] <= 1e-10 and rel_residual(H, u, c["q"]) <= 1e-10
    assert rel_max(u, dst_solve(c["q"], 1.0, 0.1, 1.0)) <= 1e-9
    rr, _ = H.forward(c["q"], rtol=1e-14, max_cycles=100)
    drho, _ = P.jvp(rho, dev(c["dq"]), dev(c["dlogD"]), dev(c["dlogmua"]))
    dr, _ = H.jvp(rr, c["dq"], c["dlogD"], c["dlogmua"], rtol=1e-14, max_cycles=100)
    assert rel_max(host(drho), dr) <= 1e-8
    (qb, gD, gmu), vinfo = P.vjp(rho, dev(c["rhobar"]))
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], rtol=1e-14, max_cycles=100)
    for g, r in ((qb, rqb), (gD, rgD), (gmu, rgmu)):
        assert rel_max(host(g), r) <= 1e-8
    assert rel_max(host(qb), dst_solve(c["rhobar"], 1.0, 0.1, 1.0)) <= 1e-8


@pytest.mark.parametrize("precision", ["fp64", "fp32-in-fp64"])
@pytest.mark.parametrize("N", [64, 96, 128, 192])
def test_tolerance_mode_forward_vjp_against_oracle(precision, N):
    """Forward + VJP to 1e-10 on GRF coefficients; gradients within 1e-8."""
    from oracle import ref
    say("tolerance %s N=%d" % (precision, N))
    c = grf_inputs(N, 7 * N)
    H = ref.Hierarchy(c["D"], c["mua"])
    P = plan_for(c["D"], c["mua"], precision=precision)
    rho, info = P.forward(dev(c["q"]))
    u = host(rho)
    assert info["rel_residual"] <= 1e-10
    assert rel_residual(H, u, c["q"]) <= 1e-10
    rr, _ = H.forward(c["q"], rtol=1e-13, max_cycles=200)
    (qb, gD, gmu), vinfo = P.vjp(rho, dev(c["rhobar"]))
    lam = host(qb)
    assert vinfo["rel_residual"] <= 1e-10
    assert np.linalg.norm(c["rhobar"] - H.apply(0, lam)) / np.linalg.norm(c["rhobar"]) <= 1e-10
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], rtol=1e-13, max_cycles=200)
    errs = {"u": rel_max(u, rr), "q": rel_max(lam, rqb), "logD": rel_max(host(gD), rgD),
            "logmua": rel_max(host(gmu), rgmu)}
    say("errors vs oracle", {k: "%.2e" % v for k, v in errs.items()}, "cycles", info["cycles"], vinfo["cycles"])
    assert max(errs.values()) <= 1e-8, errs
    drho, jinfo = P.jvp(rho, dev(c["dq"]), dev(c["dlogD"]), dev(c["dlogmua"]))
    dr, _ = H.jvp(rr, c["dq"], c["dlogD"], c["dlogmua"], rtol=1e-13, max_cycles=200)
    assert rel_max(host(drho), dr) <= 1e-8


def test_boundary_value_and_small_grids():
    from oracle import ref
    from paper_2608_00760_amd import synth
    say("boundary value and single-level grids")
    for N in (2, 3, 6, 12):
        logD, logmu = synth.log_coefficients(N, N, N + 1)
        D, mu = np.exp(logD), np.exp(logmu)
        q = synth.normal(N, 3)
        H = ref.Hierarchy(D, mu, bc=0.5)
        rr, _ = H.forward(q, rtol=1e-13)
        for prec in ("fp64", "fp32-in-fp64"):
            P = plan_for(D, mu, bc_value=0.5, precision=prec, rtol=1e-12)
            rho, info = P.forward(dev(q))
            assert rel_max(host(rho), rr) <= 1e-10, (N, prec, info)


def test_error_paths():
    import torch
    from paper_2608_00760_amd import _abi, synth
    from paper_2608_00760_amd.solver import Options, Plan
    say("error paths")
    N = 16
    D = np.ones(synth.shape(N)); mu = np.full(synth.shape(N), 0.1)
    with pytest.raises(_abi.DMGSError) as e:
        Plan(Options(20))
    assert e.value.status == _abi.DMGS_ERR_INVALID
    P = Plan(Options(N, max_cycles=2, rtol=1e-14))
    with pytest.raises(_abi.DMGSError):
        P.forward(dev(synth.normal(N, 1)))            # coefficients not set
    bad = D.copy(); bad[3, 4, 5] = -1.0
    with pytest.raises(_abi.DMGSError) as e:
        P.set_coefficients(dev(bad), dev(mu))
    assert e.value.status == _abi.DMGS_ERR_INVALID
    P.set_coefficients(dev(D), dev(mu))
    rho, info = P.forward(dev(synth.normal(N, 1)), check=False)
    assert info["status"] == _abi.DMGS_ERR_NOT_CONVERGED and info["cycles"] == 2
    q = synth.normal(N, 2); q[5, 5, 5] = np.nan
    rho, info = P.forward(dev(q), check=False)
    assert info["status"] == _abi.DMGS_ERR_NONFINITE
    with pytest.raises(ValueError):
        P.forward(torch.zeros((N, N, N), dtype=torch.float64, device="cuda:0"))
    zero, info = P.forward(dev(np.zeros(synth.shape(N))))
    assert info["cycles"] == 0 and float(zero.abs().max()) == 0.0


def test_out_of_memory_leaves_other_plans_working(monkeypatch):
    """A call whose work buffers do not fit on the device fails with
    DMGS_ERR_OOM (here the unrolled adjoint at 256^3 told to keep the states
    of 250 cycles, about 350 GB), and the next calls on this host thread, on
    another plan and on the same one, still succeed: the failed allocation
    is not left behind as HIP's last error for their launch checks."""
    import torch
    from paper_2608_00760_amd import _abi, synth
    from paper_2608_00760_amd.solver import Options, Plan
    say("out of memory")
    N = 32
    c = synth.grf_case(N, 555)
    P = Plan(Options(N, precision="fp32-in-fp64"))
    P.set_log_coefficients(dev(c["logD"]), dev(c["logmua"]))
    q = dev(c["q"])
    ref, _ = P.forward(q)
    torch.cuda.synchronize()
    monkeypatch.setenv("DMGS_UNROLLED_STORE", "1")
    Nb = 256
    Q = Plan(Options(Nb, fixed_cycles=250))
    zero = torch.zeros(synth.shape(Nb), dtype=torch.float64, device="cuda:0")
    Q.set_log_coefficients(zero, zero)
    with pytest.raises(_abi.DMGSError) as e:
        Q.vjp_unrolled(zero, zero)
    assert e.value.status == _abi.DMGS_ERR_OOM
    torch.cuda.synchronize()
    rho, info = P.forward(q)
    torch.cuda.synchronize()
    assert info["status"] == _abi.DMGS_OK and torch.equal(rho, ref)
    # the same plan: a plain solve (its own buffers were allocated at creation)
    r, qi = Q.forward(zero)
    torch.cuda.synchronize()
    assert qi["status"] == _abi.DMGS_OK and float(r.abs().max()) == 0.0
    Q.close()
    P.close()


def test_determinism_bitwise():
    from paper_2608_00760_amd import synth
    say("determinism")
    c = grf_inputs(64, 5)
    for prec in ("fp64", "fp32-in-fp64"):
        P = plan_for(c["D"], c["mua"], precision=prec)
        a, _ = P.forward(dev(c["q"]))
        b, _ = P.forward(dev(c["q"]))
        assert bool((a == b).all())
        (ga, _, _), _ = P.vjp(a, dev(c["rhobar"]))
        (gb, _, _), _ = P.vjp(a, dev(c["rhobar"]))
        assert bool((ga == gb).all())


def test_adaptive_refinement_steps():
    """Adaptive inner V-cycle counts reach the tolerance with no more float32
    V-cycles than fixed two-cycle steps need (plus one), in fewer steps."""
    from paper_2608_00760_amd import synth
    say("adaptive refinement")
    N = 64
    c = grf_inputs(N, 11)
    Pa = plan_for(c["D"], c["mua"], precision="fp32-in-fp64")
    Pf = plan_for(c["D"], c["mua"], precision="fp32-in-fp64", ir_inner_cycles=2, ir_adaptive=False)
    ra, ia = Pa.forward(dev(c["q"]))
    rf, if_ = Pf.forward(dev(c["q"]))
    assert ia["rel_residual"] <= 1e-10 and if_["rel_residual"] <= 1e-10
    assert if_["vcycles"] == 2 * if_["cycles"]
    assert ia["vcycles"] <= if_["vcycles"] + 1 and ia["cycles"] < if_["cycles"], (ia, if_)
    assert rel_max(host(ra), host(rf)) <= 1e-8
    (qa, _, _), va = Pa.vjp(ra, dev(c["rhobar"]))
    (qf, _, _), vf = Pf.vjp(rf, dev(c["rhobar"]))
    assert va["rel_residual"] <= 1e-10 and vf["rel_residual"] <= 1e-10
    assert va["vcycles"] <= vf["vcycles"] + 1 and va["cycles"] < vf["cycles"], (va, vf)
    assert rel_max(host(qa), host(qf)) <= 1e-8


@pytest.mark.parametrize("precision", ["fp32-in-fp64", "fp64"])
def test_forward_vjp_concurrent_equals_separate_calls(precision):
    """dmgs_forward_vjp (adjoint solve on a second stream) gives bitwise the
    results of dmgs_forward followed by dmgs_vjp."""
    say("forward_vjp %s" % precision)
    N = 64
    c = grf_inputs(N, 13)
    P = plan_for(c["D"], c["mua"], precision=precision)
    rho, inf = P.forward(dev(c["q"]))
    (qb, gD, gmu), ina = P.vjp(rho, dev(c["rhobar"]))
    for rep in range(2):
        (rho2, (qb2, gD2, gmu2)), if2, ia2 = P.forward_vjp(dev(c["q"]), dev(c["rhobar"]))
        assert if2["status"] == 0 and ia2["status"] == 0
        assert if2["vcycles"] == inf["vcycles"] and ia2["vcycles"] == ina["vcycles"]
        for a, b in ((rho, rho2), (qb, qb2), (gD, gD2), (gmu, gmu2)):
            assert bool((a == b).all()), rep


@pytest.mark.parametrize("nu1,nu2", [(2, 1), (1, 3), (0, 2)])
def test_fixed_cycles_unequal_smoothing(nu1, nu2):
    """V(nu1,nu2) with nu1 != nu2: the pull-back is the transposed cycle with
    the smoothing counts exchanged, equal to the oracle's literal reversed
    composition, and the dot-product identity holds on the GPU alone."""
    from oracle import ref
    say("fixed nu=%d,%d" % (nu1, nu2))
    N, n = 48, 3
    c = grf_inputs(N, 700 + nu1)
    H = ref.Hierarchy(c["D"], c["mua"])
    P = plan_for(c["D"], c["mua"], fixed_cycles=n, nu_pre=nu1, nu_post=nu2)
    rho, _ = P.forward(dev(c["q"]))
    rr, _ = H.forward(c["q"], fixed_cycles=n, nu1=nu1, nu2=nu2)
    assert rel_max(host(rho), rr) <= 1e-12
    (qb, gD, gmu), _ = P.vjp(rho, dev(c["rhobar"]))
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], fixed_cycles=n, nu1=nu1, nu2=nu2)
    for g, r in ((qb, rqb), (gD, rgD), (gmu, rgmu)):
        assert rel_max(host(g), r) <= 1e-12
    drho, _ = P.jvp(rho, dev(c["dq"]), dev(c["dlogD"]), dev(c["dlogmua"]))
    lhs = float((drho * dev(c["rhobar"])).sum())
    rhs = float((dev(c["dq"]) * qb).sum() + (dev(c["dlogD"]) * gD).sum() + (dev(c["dlogmua"]) * gmu).sum())
    assert abs(lhs - rhs) <= 1e-12 * float(drho.norm()) * float(np.linalg.norm(c["rhobar"]))


@pytest.mark.parametrize("N,face_mean,max_cycles", [(64, "arith", 200), (96, "harmonic", 200), (128, "arith", 4)])
def test_fp64_norm_from_next_pass_matches_explicit_residual(N, face_mean, max_cycles, monkeypatch):
    """Float64 tolerance mode takes each iterate's residual norm from the
    next cycle's first two-sweep pass.  Against the same plan with that pass
    switched off for float64 levels (DMGS_SWEEP2_FP64=0: one-sweep passes and
    an explicit residual pass after every cycle): the same number of cycles
    and the same stopping status (also when max_cycles ends the solve, where
    the returned iterate is the last complete cycle's).  The two smooth with
    different kernels, so their iterates differ in the last bits and their
    residuals near 1e-10 agree to about 1e-5; the check is 1e-3, against
    which a norm from the wrong iterate or a missing colour (factors of 2 and
    more) fails.  Each reported residual equals the oracle operator's residual
    of the returned iterate to 1e-3."""
    from oracle import ref
    say("fp64 norm from the next pass N=%d %s max_cycles=%d" % (N, face_mean, max_cycles))
    c = grf_inputs(N, 7000 + N)
    H = ref.Hierarchy(c["D"], c["mua"], face_mean=face_mean)
    res = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("DMGS_SWEEP2_FP64", flag)
        P = plan_for(c["D"], c["mua"], face_mean=face_mean, max_cycles=max_cycles)
        rho, fi = P.forward(dev(c["q"]), check=False)
        (qb, _, _), vi = P.vjp(rho, dev(c["rhobar"]), check=False)
        res[flag] = (host(rho), fi, host(qb), vi)
        say("  DMGS_SWEEP2_FP64=%s fwd %d cycles %.3e status %d, adj %d cycles %.3e" % (
            flag, fi["cycles"], fi["rel_residual"], fi["status"], vi["cycles"], vi["rel_residual"]))
    (r1, f1, l1, v1), (r0, f0, l0, v0) = res["1"], res["0"]
    for a, b in ((f1, f0), (v1, v0)):
        assert a["cycles"] == b["cycles"] and a["status"] == b["status"]
        assert abs(a["rel_residual"] - b["rel_residual"]) <= 1e-3 * b["rel_residual"]
    for rho, fi, lam, vi in (res["1"], res["0"]):
        assert abs(rel_residual(H, rho, c["q"]) - fi["rel_residual"]) <= 1e-3 * fi["rel_residual"]
        lam_res = np.linalg.norm(c["rhobar"] - H.apply(0, lam)) / np.linalg.norm(c["rhobar"])
        assert abs(lam_res - vi["rel_residual"]) <= 1e-3 * vi["rel_residual"]
    if max_cycles == 200:
        assert f1["status"] == 0 and f1["rel_residual"] <= 1e-10
    else:
        assert f1["status"] == 3 and f1["cycles"] == max_cycles
