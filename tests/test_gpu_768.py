"""The largest grid of the benchmark sweep, 768^3 (769^3 = 455M vertices),
in float64: the only size whose float64 fields exceed 2 GiB, so its finest
level takes the one-sweep-per-pass kernel instead of the two-sweep pass.

Forward solve and pull-back to a relative residual of 1e-10 (Sec. 2.4) on
log-normal coefficients drawn on the device (as the sweep draws them),
then on the host, with the oracle's operator:
* ||q - A u|| / ||q|| and ||w - A lam|| / ||w|| over the interior <= 1e-10;
* the log D and log mua gradients equal the oracle's pointwise gradient
  formula applied to the GPU's own u and lam, at every vertex, to 1e-12.
Peak device memory is reported.
"""
import numpy as np
import pytest

from gpu_util import host, rel_max, say

pytestmark = pytest.mark.gpu


def test_768_float64_forward_vjp():
    import torch
    from oracle import ref
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.solver import Options, Plan
    N = 768
    say("768^3 float64: inputs on the device")
    g = torch.Generator(device="cuda:0")
    g.manual_seed(7768)
    shp = (N + 1,) * 3
    logD = 0.5 * torch.randn(shp, generator=g, device="cuda:0", dtype=torch.float64)
    logmu = -3.0 + 0.5 * torch.randn(shp, generator=g, device="cuda:0", dtype=torch.float64)
    q = synth.zero_boundary_torch(torch.randn(shp, generator=g, device="cuda:0", dtype=torch.float64))
    w = synth.zero_boundary_torch(torch.randn(shp, generator=g, device="cuda:0", dtype=torch.float64))
    torch.cuda.reset_peak_memory_stats()
    P = Plan(Options(N, precision="fp64"))
    P.set_log_coefficients(logD, logmu)
    say("768^3 float64: forward")
    rho, fi = P.forward(q)
    say("768^3 float64: pull-back")
    (qb, gD, gmu), vi = P.vjp(rho, w)
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() + P.bytes
    say("768^3: cycles %d / %d, rel residuals %.2e / %.2e, peak device %.1f GB" % (
        fi["cycles"], vi["cycles"], fi["rel_residual"], vi["rel_residual"], peak / 1e9))
    P.close()
    del P
    D, mu = np.exp(host(logD)), np.exp(host(logmu))
    del logD, logmu
    qh, wh, u, lam = host(q), host(w), host(rho), host(qb)
    gDh, gmuh = host(gD), host(gmu)
    del q, w, rho, qb, gD, gmu
    torch.cuda.empty_cache()
    say("768^3: host checks with the oracle's operator")
    H = ref.Hierarchy(D, mu)
    res_f = np.linalg.norm(H.defect(0, u, qh)) / np.linalg.norm(qh)
    res_a = np.linalg.norm(H.defect(0, lam, wh)) / np.linalg.norm(wh)
    fD, fmu = H.coef_grads(u, lam)
    e = (rel_max(gDh, fD), rel_max(gmuh, fmu))
    say("768^3: residuals %.2e / %.2e, gradient formula %.1e / %.1e" % (res_f, res_a, e[0], e[1]))
    assert res_f <= 1e-10 and res_a <= 1e-10
    assert max(e) <= 1e-12
