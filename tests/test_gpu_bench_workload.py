"""The 256^3 workload at full size, in the configuration bench.py times,
against the FP64 oracle.

Inputs are bench.py's own (synth.grf_case(256, 3000): GRF log D and log mua,
16 Gaussian blobs plus noise, a seeded cotangent).  The float32-in-float64
plan with adaptive refinement steps runs the forward solve and the VJP
concurrently (dmgs_forward_vjp on two streams), and the plain float64 plan
runs them one after the other, both to a relative residual of 1e-10.

* Each solution's relative residual over the interior, taken with the
  oracle's FP64 defect on the host, is at most 1e-10 (forward: q - A u;
  adjoint: rhobar - A lam).
* u, the pull-back qbar = lam and the gradients in log D and log mua match
  the oracle's solves to 1e-13 within 1e-8 of the largest entry, and the
  gradients match the oracle's gradient formula applied to the GPU's own u
  and lam to 1e-12 (the formula is pointwise, so this checks every vertex
  of the gradient pass at full size).
* The likelihood gradient (forward solve, epilogue, pull-back, gradients)
  matches the oracle's: H and chi2 to 1e-9, gradients to 1e-8.
"""
import numpy as np
import pytest

from gpu_util import dev, host, rel_max, say

pytestmark = pytest.mark.gpu

N = 256


@pytest.fixture(scope="module")
def workload():
    from oracle import ref
    from paper_2608_00760_amd import synth
    say("256^3 bench workload: inputs and oracle solves")
    c = synth.grf_case(N, 3000)
    H = ref.Hierarchy(c["D"], c["mua"])
    rr, _ = H.forward(c["q"], rtol=1e-13, max_cycles=200)
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], rtol=1e-13, max_cycles=200)
    yield c, H, (rr, rqb, rgD, rgmu)
    del H


def rel_res(H, u, f):
    """||f - A u|| / ||f|| over the interior (the oracle's defect is 0 on the
    zero Dirichlet boundary, where f is not an equation's right-hand side)."""
    return np.linalg.norm(H.defect(0, u, f)) / np.linalg.norm(H.defect(0, np.zeros_like(u), f))


def check(H, c, oracle, u, lam, gD, gmu, what):
    rr, rqb, rgD, rgmu = oracle
    res = {"forward": rel_res(H, u, c["q"]), "adjoint": rel_res(H, lam, c["rhobar"])}
    errs = {"u": rel_max(u, rr), "qbar": rel_max(lam, rqb), "logD": rel_max(gD, rgD), "logmua": rel_max(gmu, rgmu)}
    fD, fmu = H.coef_grads(u, lam)
    local = {"logD": rel_max(gD, fD), "logmua": rel_max(gmu, fmu)}
    say(what, "residuals", {k: "%.2e" % v for k, v in res.items()}, "errors vs oracle",
        {k: "%.2e" % v for k, v in errs.items()}, "gradient formula", {k: "%.1e" % v for k, v in local.items()})
    assert max(res.values()) <= 1e-10, res
    assert max(errs.values()) <= 1e-8, errs
    assert max(local.values()) <= 1e-12, local


def test_mixed_precision_concurrent(workload):
    import torch
    from paper_2608_00760_amd.solver import Options, Plan
    c, H, oracle = workload
    say("256^3 float32-in-float64, forward and VJP concurrent")
    t = {k: dev(c[k]) for k in ("logD", "logmua", "q", "rhobar")}
    bufs = [torch.empty_like(t["q"]) for _ in range(4)]
    P = Plan(Options(N, precision="fp32-in-fp64", rtol=1e-10, max_cycles=100))
    P.set_log_coefficients(t["logD"], t["logmua"])
    _, info_f, info_a = P.forward_vjp(t["q"], t["rhobar"], out=bufs)
    torch.cuda.synchronize()
    say("cycles", info_f["cycles"], info_a["cycles"])
    assert info_f["rel_residual"] <= 1e-10 and info_a["rel_residual"] <= 1e-10
    check(H, c, oracle, *(host(b) for b in bufs), "fp32-in-fp64")
    P.close()


def test_float64_sequential(workload):
    from paper_2608_00760_amd.solver import Options, Plan
    c, H, oracle = workload
    say("256^3 float64, forward then VJP")
    P = Plan(Options(N, precision="fp64", rtol=1e-10, max_cycles=100))
    P.set_log_coefficients(dev(c["logD"]), dev(c["logmua"]))
    rho, info = P.forward(dev(c["q"]))
    (qb, gD, gmu), vinfo = P.vjp(rho, dev(c["rhobar"]))
    assert info["rel_residual"] <= 1e-10 and vinfo["rel_residual"] <= 1e-10
    check(H, c, oracle, host(rho), host(qb), host(gD), host(gmu), "fp64")
    P.close()


def test_likelihood_gradient(workload):
    """The likelihood leg of the bench at 256^3: forward solve, epilogue,
    pull-back and gradients (float32-in-float64 to 1e-10) against the
    oracle's, with data drawn from the noise model around the oracle's
    response and a 3-vertex edge mask."""
    from oracle import likelihood
    from paper_2608_00760_amd.solver import Options, Plan
    c, H, (rr, _, _, _) = workload[0], workload[1], workload[2]
    say("256^3 likelihood gradient")
    Le = rr * c["mua"]
    sigma = np.maximum(0.05 * Le, 0.01 * Le.max())
    d = Le + sigma * np.random.default_rng(3005).standard_normal(Le.shape)
    w = likelihood.noise_weights(Le, 3)
    P = Plan(Options(N, precision="fp32-in-fp64", rtol=1e-10, max_cycles=100))
    P.set_log_coefficients(dev(c["logD"]), dev(c["logmua"]))
    (rho, val, (qb, gD, gmu)), fi, vi = P.likelihood_grad(dev(c["q"]), dev(d), dev(w))
    assert fi["status"] == 0 and vi["status"] == 0
    _, (Hv, chi2), (rqb, rgD, rgmu) = likelihood.likelihood_grad(H, c["mua"], c["q"], d, w, rtol=1e-13,
                                                                 max_cycles=300)
    errs = {"H": abs(val["H"] - Hv) / Hv, "chi2": abs(val["chi2"] - chi2) / chi2, "q": rel_max(host(qb), rqb),
            "logD": rel_max(host(gD), rgD), "logmua": rel_max(host(gmu), rgmu)}
    say("chi2 %.4f nvox %d" % (val["chi2"], val["nvox"]), {k: "%.2e" % v for k, v in errs.items()})
    assert errs["H"] <= 1e-9 and errs["chi2"] <= 1e-9
    assert max(errs["q"], errs["logD"], errs["logmua"]) <= 1e-8
    assert val["nvox"] == int(np.count_nonzero(w > 0))
    assert abs(val["chi2"] - 1.0) <= 4.0 * np.sqrt(2.0 / val["nvox"])
    P.close()
