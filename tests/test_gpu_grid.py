"""General-grid plans (different cell counts and spacings per axis) against
the oracle for such grids (oracle/refgrid.py), through the C ABI.

* Fixed cycles (the paper's mode, Sec. 2.4): forward, push-forward and
  pull-back with both coefficient gradients agree with the oracle to 1e-12
  of the largest entry (rounding order only), on ragged shapes, both face
  means, g != 0 and the paper's data grid: (128, 64, 64) cells over
  7.5 x 3.5 x 3.5 cm (Sec. 2.5.1).
* Tolerance mode on the paper's grid: the residual, taken with the oracle's
  operator, is at most 1e-10, and rho, rho' and the gradients agree with the
  oracle's 1e-13 solves to 1e-8.
* The likelihood epilogue on the paper's grid (Eq. (response), Eq. (noise),
  Eq. (likelihood), Eq. (chi2)), with the edges masked to 0.2 cm (4
  vertices at these spacings): noise weights, H, chi2 and all gradients
  against the oracle.
* dmgs_forward_vjp equals the separate calls; the diagnostic entry points
  and the unrolled adjoint reject general grids.
* A plan keeps working after a plan with a smaller coarsest level is created
  (the coarsest inverse's LDS limit is process-wide).
"""
import math

import numpy as np
import pytest

from gpu_util import dev, host, rel_max, say

pytestmark = pytest.mark.gpu

PAPER_CELLS = (128, 64, 64)
PAPER_H = (7.5 / 128, 3.5 / 64, 3.5 / 64)


def make(cells, h, seed, face_mean="arith", g=0.0, fixed_cycles=0):
    from oracle import refgrid
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.solver import Options, Plan
    c = synth.grid_case(cells, seed)
    P = Plan(Options(cells[0], shape=cells, spacing=h, face_mean=face_mean, bc_value=g, fixed_cycles=fixed_cycles))
    P.set_log_coefficients(dev(c["logD"]), dev(c["logmua"]))
    H = refgrid.HierarchyGrid(c["D"], c["mua"], h=h, g=g, face_mean=face_mean)
    return P, H, c


@pytest.mark.parametrize("cells,h,face_mean,g", [
    ((16, 8, 8), (0.5, 1.0, 1.5), "arith", 0.0),
    ((24, 12, 12), (1.0, 0.25, 2.0), "harmonic", 0.3),
    ((12, 24, 24), (1.0, 1.0, 1.0), "arith", 0.0),
    ((64, 64, 32), (1.0, 1.0, 1.0), "harmonic", 0.0),
    (PAPER_CELLS, PAPER_H, "arith", 0.0),
    (PAPER_CELLS, PAPER_H, "harmonic", 0.2),
])
def test_fixed_cycles_against_oracle(cells, h, face_mean, g):
    n = 3
    say("grid fixed cycles", cells, h, face_mean, g)
    P, H, c = make(cells, h, 8000 + sum(cells), face_mean, g, fixed_cycles=n)
    rho, _ = P.forward(dev(c["q"]))
    rr, _ = H.forward(c["q"], fixed_cycles=n)
    assert rel_max(host(rho), rr) <= 1e-12
    drho, _ = P.jvp(rho, dev(c["dq"]), dev(c["dlogD"]), dev(c["dlogmua"]))
    dr, _ = H.jvp(rr, c["dq"], c["dlogD"], c["dlogmua"], fixed_cycles=n)
    assert rel_max(host(drho), dr) <= 1e-12
    (qb, gD, gmu), _ = P.vjp(rho, dev(c["rhobar"]))
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], fixed_cycles=n)
    errs = [rel_max(host(a), b) for a, b in ((qb, rqb), (gD, rgD), (gmu, rgmu))]
    say("  errors", ["%.1e" % e for e in errs])
    assert max(errs) <= 1e-12


def test_tolerance_mode_paper_grid():
    say("grid tolerance mode, paper grid")
    P, H, c = make(PAPER_CELLS, PAPER_H, 8200)
    rho, fi = P.forward(dev(c["q"]))
    u = host(rho)
    res = np.linalg.norm(H.defect(0, u, c["q"])) / np.linalg.norm(H.defect(0, np.zeros_like(u), c["q"]))
    assert fi["rel_residual"] <= 1e-10 and res <= 1e-10
    rr, _ = H.forward(c["q"], rtol=1e-13)
    (qb, gD, gmu), vi = P.vjp(rho, dev(c["rhobar"]))
    lam = host(qb)
    assert vi["rel_residual"] <= 1e-10
    assert np.linalg.norm(c["rhobar"] - H.apply(0, lam)) / np.linalg.norm(c["rhobar"]) <= 1e-10
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], rtol=1e-13)
    drho, ji = P.jvp(rho, dev(c["dq"]), dev(c["dlogD"]), dev(c["dlogmua"]))
    dr, _ = H.jvp(rr, c["dq"], c["dlogD"], c["dlogmua"], rtol=1e-13)
    errs = {"u": rel_max(u, rr), "qbar": rel_max(lam, rqb), "logD": rel_max(host(gD), rgD),
            "logmua": rel_max(host(gmu), rgmu), "drho": rel_max(host(drho), dr)}
    say("  cycles", fi["cycles"], vi["cycles"], ji["cycles"], "errors", {k: "%.1e" % v for k, v in errs.items()})
    assert max(errs.values()) <= 1e-8, errs


def test_likelihood_paper_grid():
    import torch
    from oracle import likelihood
    from paper_2608_00760_amd import synth
    say("grid likelihood, paper grid")
    P, H, c = make(PAPER_CELLS, PAPER_H, 8300, fixed_cycles=15)
    # the paper masks 0.2 cm on all edges: ceil(0.2 / h_a) vertices per axis
    mask = max(math.ceil(0.2 / ha - 1e-12) for ha in PAPER_H)
    assert mask == 4
    rr, _ = H.forward(c["q"], fixed_cycles=15)
    Le = c["mua"] * rr
    w_ref = likelihood.noise_weights(Le, mask)
    w = P.noise_weights(dev(Le), mask)
    torch.cuda.synchronize()
    assert rel_max(host(w), w_ref) <= 1e-15
    sigma = np.sqrt(np.where(w_ref > 0, 1.0 / np.where(w_ref > 0, w_ref, 1.0), 0.0))
    d = Le + sigma * np.random.default_rng(8301).standard_normal(Le.shape)
    (rho, val, (qb, gD, gmu)), _, _ = P.likelihood_grad(dev(c["q"]), dev(d), dev(w_ref))
    _, (Hv, chi2), (rq, rD, rm) = likelihood.likelihood_grad(H, c["mua"], c["q"], d, w_ref, fixed_cycles=15)
    errs = [abs(val["H"] - Hv) / Hv, abs(val["chi2"] - chi2) / chi2] + [
        rel_max(host(a), b) for a, b in ((qb, rq), (gD, rD), (gmu, rm))]
    say("  chi2 %.4f (oracle %.4f), N_vox %d, errors %s" % (val["chi2"], chi2, val["nvox"], ["%.1e" % e for e in errs]))
    assert val["nvox"] == int((w_ref > 0).sum())
    assert max(errs) <= 1e-11
    assert abs(val["chi2"] - 1.0) < 0.05


def test_forward_vjp_and_rejections():
    import torch
    from paper_2608_00760_amd import _abi
    P, H, c = make((32, 16, 16), (1.0, 0.5, 0.5), 8400)
    rho, _ = P.forward(dev(c["q"]))
    (qb, gD, gmu), _ = P.vjp(rho, dev(c["rhobar"]))
    (rho2, (qb2, gD2, gmu2)), _, _ = P.forward_vjp(dev(c["q"]), dev(c["rhobar"]))
    torch.cuda.synchronize()
    for a, b in ((rho, rho2), (qb, qb2), (gD, gD2), (gmu, gmu2)):
        assert torch.equal(a, b)
    assert P.level_shape[-1] == (4, 2, 2) and P.levels == 4
    with pytest.raises(_abi.DMGSError):
        P.debug_apply(0, rho)
    from paper_2608_00760_amd.solver import Options, Plan
    Q = Plan(Options(32, shape=(32, 16, 16), spacing=(1.0, 0.5, 0.5), fixed_cycles=2))
    Q.set_log_coefficients(dev(c["logD"]), dev(c["logmua"]))
    with pytest.raises(_abi.DMGSError):
        Q.vjp_unrolled(dev(c["q"]), dev(c["rhobar"]))


def test_plans_with_different_coarsest_levels():
    """(60, 12, 12) cells coarsen to (15, 3, 3): 56 coarsest unknowns, whose
    inverse takes 50 KB of LDS; (16, 8, 8) coarsens to 3 unknowns.  The first
    plan's coefficient set-up and solve still run after the second exists,
    and match the oracle."""
    from oracle import refgrid
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.solver import Options, Plan
    say("grid plans with different coarsest levels")
    big, small = (60, 12, 12), (16, 8, 8)
    h = (0.5, 1.0, 1.0)
    A = Plan(Options(big[0], shape=big, spacing=h, fixed_cycles=3))
    B = Plan(Options(small[0], shape=small, spacing=h, fixed_cycles=3))
    cb = synth.grid_case(small, 8600)
    B.set_log_coefficients(dev(cb["logD"]), dev(cb["logmua"]))
    c = synth.grid_case(big, 8601)
    A.set_log_coefficients(dev(c["logD"]), dev(c["logmua"]))
    rho, _ = A.forward(dev(c["q"]))
    rr, _ = refgrid.HierarchyGrid(c["D"], c["mua"], h=h).forward(c["q"], fixed_cycles=3)
    assert A.level_shape[-1] == (15, 3, 3)
    assert rel_max(host(rho), rr) <= 1e-12
