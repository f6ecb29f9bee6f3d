"""torch.autograd.Function over the C ABI: reverse mode, forward mode,
central finite differences, and the 512^3 forward + backward.

Reverse and forward mode must equal the direct dmgs_vjp / dmgs_jvp calls
bitwise (same kernels, same inputs) and the oracle to 1e-8.  Central
differences of <w, u(theta + eps v)> with eps = 1e-4 in log space agree with
<J^T w, v> to O(eps^2) ~ 1e-8 relative; the test allows 1e-6 (the solves run
to 1e-12).
"""
import numpy as np
import pytest

from gpu_util import dev, host, rel_max, say

pytestmark = pytest.mark.gpu


def fields(N, seed):
    from paper_2608_00760_amd import synth
    c = synth.grf_case(N, seed)
    c.update({k: v for k, v in synth.tangents(N, seed + 50).items() if k != "rhobar"})
    return c


@pytest.mark.parametrize("precision", ["fp64", "fp32-in-fp64"])
def test_backward_and_forward_mode_match_abi_and_oracle(precision):
    import torch
    import torch.autograd.forward_ad as fwAD
    from oracle import ref
    from paper_2608_00760_amd.autograd import Solver
    say("autograd", precision)
    N = 32
    c = fields(N, 77)
    S = Solver(N, precision=precision, rtol=1e-12)
    q, logD, logmua = (dev(c[k]).requires_grad_(True) for k in ("q", "logD", "logmua"))
    rho = S(q, logD, logmua)
    w = dev(c["rhobar"])
    gq, gD, gmu = torch.autograd.grad((rho * w).sum(), (q, logD, logmua))
    (dq_, dD_, dmu_), _ = S.plan.vjp(rho.detach(), w)
    assert torch.equal(gq, dq_) and torch.equal(gD, dD_) and torch.equal(gmu, dmu_)
    H = ref.Hierarchy(c["D"], c["mua"])
    rr, _ = H.forward(c["q"], rtol=1e-13)
    (rq, rD, rmu), _ = H.vjp(rr, c["rhobar"], rtol=1e-13)
    for a, b in ((gq, rq), (gD, rD), (gmu, rmu)):
        assert rel_max(host(a), b) <= 1e-8
    # forward mode with dual tensors
    with fwAD.dual_level():
        dq = fwAD.make_dual(dev(c["q"]), dev(c["dq"]))
        dD = fwAD.make_dual(dev(c["logD"]), dev(c["dlogD"]))
        dm = fwAD.make_dual(dev(c["logmua"]), dev(c["dlogmua"]))
        out = S(dq, dD, dm)
        tangent = fwAD.unpack_dual(out).tangent
    direct, _ = S.plan.jvp(rho.detach(), dev(c["dq"]), dev(c["dlogD"]), dev(c["dlogmua"]))
    assert torch.equal(tangent, direct)
    dr, _ = H.jvp(rr, c["dq"], c["dlogD"], c["dlogmua"], rtol=1e-13)
    assert rel_max(host(tangent), dr) <= 1e-8


def test_backward_resets_coefficients_changed_in_between():
    import torch
    from paper_2608_00760_amd.autograd import Solver
    say("coefficient staleness")
    N = 32
    a, b = fields(N, 1), fields(N, 2)
    S = Solver(N)
    qa, Da, ma = (dev(a[k]).requires_grad_(True) for k in ("q", "logD", "logmua"))
    rho_a = S(qa, Da, ma)
    rho_b = S(dev(b["q"]), dev(b["logD"]), dev(b["logmua"]))     # plan now holds b's coefficients
    w = dev(a["rhobar"])
    gq, gD, gmu = torch.autograd.grad((rho_a * w).sum(), (qa, Da, ma))
    S2 = Solver(N)
    S2.plan.set_log_coefficients(dev(a["logD"]), dev(a["logmua"]))
    (eq, eD, emu), _ = S2.plan.vjp(rho_a.detach(), w)
    assert torch.equal(gq, eq) and torch.equal(gD, eD) and torch.equal(gmu, emu)


@pytest.mark.parametrize("precision", ["fp64", "fp32-in-fp64"])
def test_central_differences_128_32_directions(precision):
    """Gradients of <w, u> against central differences, 32 seeded directions
    (the 128^3 workload: float64, as it is named, and the mixed mode)."""
    import torch
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.autograd import Solver
    say("central differences 128^3 %s" % precision)
    N = 128
    c = synth.grf_128()
    S = Solver(N, precision=precision, rtol=1e-12)
    q, logD, logmua = (dev(c[k]).requires_grad_(True) for k in ("q", "logD", "logmua"))
    w = dev(c["rhobar"])
    rho = S(q, logD, logmua)
    gq, gD, gmu = torch.autograd.grad((rho * w).sum(), (q, logD, logmua))
    eps = 1e-4
    worst = 0.0
    with torch.no_grad():
        for d in range(32):
            t = synth.tangents(N, 2100 + 10 * d)
            vq, vD, vm = dev(t["dq"]), dev(t["dlogD"]), dev(t["dlogmua"])
            f = lambda s: float((S(q + s * vq, logD + s * vD, logmua + s * vm) * w).sum())
            fd = (f(eps) - f(-eps)) / (2 * eps)
            ad = float((gq * vq).sum() + (gD * vD).sum() + (gmu * vm).sum())
            worst = max(worst, abs(fd - ad) / abs(ad))
    say("worst relative FD error (%s)" % precision, worst)
    assert worst <= 1e-6


def test_512_forward_backward_memory_and_residuals():
    """512^3 (134M cells): forward + VJP through the autograd Function in
    float32-in-float64 to 1e-10; residuals checked on the host with the
    oracle's operator; gradients spot-checked; peak device memory reported."""
    import torch
    from oracle import ref
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.autograd import Solver
    say("512^3: generating inputs")
    N = 512
    c = synth.grf_512()
    torch.cuda.reset_peak_memory_stats()
    S = Solver(N, precision="fp32-in-fp64")
    q, logD, logmua = (dev(c[k]).requires_grad_(True) for k in ("q", "logD", "logmua"))
    w = dev(c["rhobar"])
    say("512^3: forward + backward")
    rho = S(q, logD, logmua)
    gq, gD, gmu = torch.autograd.grad((rho * w).sum(), (q, logD, logmua))
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() + S.plan.bytes
    say("512^3: peak device bytes %.2f GB (torch %.2f GB + plan %.2f GB)" % (
        peak / 1e9, torch.cuda.max_memory_allocated() / 1e9, S.plan.bytes / 1e9))
    assert peak < 40e9
    u, lam = host(rho), host(gq)
    del rho
    H = ref.Hierarchy(c["D"], c["mua"])
    r = H.defect(0, u, c["q"])
    assert np.linalg.norm(r) / np.linalg.norm(synth.zero_boundary(c["q"])) <= 1e-10
    ra = c["rhobar"] - H.apply(0, lam)
    assert np.linalg.norm(ra) / np.linalg.norm(c["rhobar"]) <= 1e-10
    rgD, rgmu = H.coef_grads(u, lam)
    assert rel_max(host(gD), rgD) <= 1e-12 and rel_max(host(gmu), rgmu) <= 1e-12
