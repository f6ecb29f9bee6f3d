"""Parity of the response and likelihood epilogue (dmgs_noise_weights,
dmgs_likelihood_grad) with the oracle (oracle/likelihood.py on the solver
oracles), through the C ABI.

* The noise-model weights equal the oracle's to rounding (same operations).
* Fixed-cycle mode (float64, 3D and 2D): rho, H, chi2, N_vox and the three
  gradients equal the oracle's to 1e-12.
* Tolerance mode (float32-in-float64, 3D): H and chi2 to 1e-9, gradients to
  1e-8 against the oracle solved to 1e-13; data drawn from the noise model
  give chi2 near 1.
"""
import numpy as np
import pytest

from gpu_util import dev, host, rel_max, say

pytestmark = pytest.mark.gpu


def oracle_hier(c, ndim):
    from oracle import ref, ref2d
    return ref.Hierarchy(c["D"], c["mua"]) if ndim == 3 else ref2d.Hierarchy2D(c["D"], c["mua"])


def setup(N, seed, ndim=3, mask=3):
    """Inputs, the oracle hierarchy, and data drawn from the noise model
    around the oracle's response (nothing here comes from the GPU)."""
    from paper_2608_00760_amd import synth
    from oracle import likelihood
    c = synth.grf_case(N, seed, ndim=ndim)
    H = oracle_hier(c, ndim)
    rr, _ = H.forward(c["q"], rtol=1e-12, max_cycles=300)
    Le = rr * c["mua"]
    sigma = np.maximum(0.05 * Le, 0.01 * Le.max())
    d = Le + sigma * np.random.default_rng(seed + 9).standard_normal(Le.shape)
    w = likelihood.noise_weights(Le, mask)
    return c, H, Le, d, w


def plan_for(c, N, ndim=3, **opts):
    from paper_2608_00760_amd.solver import Options, Plan
    P = Plan(Options(N, ndim=ndim, **opts))
    P.set_coefficients(dev(c["D"]), dev(c["mua"]))
    return P


def test_noise_weights_match_oracle():
    from oracle import likelihood
    say("noise weights")
    for ndim, N, mask in ((3, 48, 3), (2, 96, 4)):
        c, _, Le, d, w = setup(N, 40 + N, ndim=ndim, mask=mask)
        P = plan_for(c, N, ndim)
        wg = host(P.noise_weights(dev(Le), mask))
        assert rel_max(wg, w) <= 1e-15
        assert (wg[w == 0] == 0).all()


@pytest.mark.parametrize("ndim,N,n", [(3, 32, 3), (3, 48, 2), (2, 128, 3)])
def test_fixed_cycles_match_oracle(ndim, N, n):
    from oracle import likelihood
    say("likelihood fixed ndim=%d N=%d n=%d" % (ndim, N, n))
    c, H, Le, d, w = setup(N, 70 + N, ndim=ndim)
    P = plan_for(c, N, ndim, fixed_cycles=n)
    (rho, val, (qb, gD, gmu)), fi, vi = P.likelihood_grad(dev(c["q"]), dev(d), dev(w))
    rr, (Hv, chi2), (rqb, rgD, rgmu) = likelihood.likelihood_grad(H, c["mua"], c["q"], d, w, fixed_cycles=n)
    say("H %.6e chi2 %.4f nvox %d" % (val["H"], val["chi2"], val["nvox"]))
    assert fi["cycles"] == n and vi["cycles"] == n
    assert rel_max(host(rho), rr) <= 1e-12
    assert abs(val["H"] - Hv) <= 1e-12 * Hv and abs(val["chi2"] - chi2) <= 1e-12 * chi2
    assert val["nvox"] == int(np.count_nonzero(w > 0))
    for g, r in ((qb, rqb), (gD, rgD), (gmu, rgmu)):
        assert rel_max(host(g), r) <= 1e-12


def test_tolerance_mode_matches_oracle():
    from oracle import likelihood
    say("likelihood tolerance fp32-in-fp64 N=64")
    N = 64
    c, H, Le, d, w = setup(N, 900)
    P = plan_for(c, N, precision="fp32-in-fp64")
    (rho, val, (qb, gD, gmu)), fi, vi = P.likelihood_grad(dev(c["q"]), dev(d), dev(w))
    assert fi["status"] == 0 and vi["status"] == 0
    rr, (Hv, chi2), (rqb, rgD, rgmu) = likelihood.likelihood_grad(H, c["mua"], c["q"], d, w, rtol=1e-13,
                                                                    max_cycles=300)
    errs = {"H": abs(val["H"] - Hv) / Hv, "chi2": abs(val["chi2"] - chi2) / chi2, "q": rel_max(host(qb), rqb),
            "logD": rel_max(host(gD), rgD), "logmua": rel_max(host(gmu), rgmu)}
    say("chi2 %.4f" % val["chi2"], {k: "%.2e" % v for k, v in errs.items()})
    assert errs["H"] <= 1e-9 and errs["chi2"] <= 1e-9
    assert max(errs["q"], errs["logD"], errs["logmua"]) <= 1e-8
    assert abs(val["chi2"] - 1.0) <= 4.0 * np.sqrt(2.0 / val["nvox"])



@pytest.mark.parametrize("precision,N,fixed,g", [
    ("fp32-in-fp64", 64, 0, 0.0), ("fp32-in-fp64", 96, 0, 0.3), ("fp32-in-fp64", 64, 3, 0.0),
    ("fp32-in-fp64", 48, 2, 0.3), ("fp64", 64, 0, 0.0), ("fp64", 48, 3, 0.3)])
def test_fused_epilogue_matches_separate_pass(precision, N, fixed, g, monkeypatch):
    """The epilogue (rhobar, the sums of H and of the kept voxels) rides on
    the forward solve's last pass over the iterate: a refining plan's last
    refinement step, a float64 plan's last residual pass.  With and without
    that fusion (DMGS_EPI_FUSE) the solves are the same: rho is bitwise
    equal, H and chi2 agree to 1e-13, the gradients to 1e-13 in fixed-cycle
    mode (1e-9 with tolerances, where a last-bit change of rhobar may move
    the adjoint's stopping point); the timing counts show that the separate
    epilogue pass ran only without fusion."""
    say("fused epilogue %s N=%d fixed=%d g=%g" % (precision, N, fixed, g))
    c, H, Le, d, w = setup(N, 950 + N + fixed)
    fused_vs_separate(lambda: plan_for(c, N, precision=precision, fixed_cycles=fixed, bc_value=g),
                      c["q"], d, w, fixed, monkeypatch)


@pytest.mark.parametrize("fixed", [0, 4])
def test_fused_epilogue_general_grid(fixed, monkeypatch):
    """General grids take the epilogue in the last half-sweep of the last
    V-cycle (in tolerance mode: of the cycle the last contraction predicts to
    be the last); the same comparison with the separate pass."""
    from oracle import likelihood
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.solver import Options, Plan
    cells, h = (64, 32, 32), (7.5 / 64, 3.5 / 32, 3.5 / 32)
    say("fused epilogue grid", cells, "fixed", fixed)
    c = synth.grid_case(cells, 960 + fixed)
    from oracle import refgrid
    Hg = refgrid.HierarchyGrid(c["D"], c["mua"], h=h)
    rr, _ = Hg.forward(c["q"], rtol=1e-12)
    Le = c["mua"] * rr
    w = likelihood.noise_weights(Le, 2)
    sigma = np.sqrt(np.where(w > 0, 1.0 / np.where(w > 0, w, 1.0), 0.0))
    d = Le + sigma * np.random.default_rng(961).standard_normal(Le.shape)

    def make():
        P = Plan(Options(cells[0], shape=cells, spacing=h, fixed_cycles=fixed))
        P.set_log_coefficients(dev(c["logD"]), dev(c["logmua"]))
        return P
    fused_vs_separate(make, c["q"], d, w, fixed, monkeypatch)


def fused_vs_separate(make, q, d, w, fixed, monkeypatch):
    import torch
    res = {}
    for fuse in (1, 0):
        monkeypatch.setenv("DMGS_EPI_FUSE", str(fuse))
        P = make()
        P.timing(True)
        (rho, val, grads), fi, vi = P.likelihood_grad(dev(q), dev(d), dev(w))
        torch.cuda.synchronize()
        res[fuse] = (host(rho), val, [host(x) for x in grads], P.timing_read()["grad"]["launches"], fi)
    (r1, v1, g1, n1, f1), (r0, v0, g0, n0, f0) = res[1], res[0]
    say("  cycles %d, grad-class launches fused %d separate %d, chi2 %.4f" % (f1["cycles"], n1, n0, v1["chi2"]))
    assert f1["cycles"] == f0["cycles"] and f1["cycles"] >= 1
    assert n1 == n0 - 1
    assert np.array_equal(r1, r0)
    assert abs(v1["H"] - v0["H"]) <= 1e-13 * v0["H"] and abs(v1["chi2"] - v0["chi2"]) <= 1e-13 * v0["chi2"]
    assert v1["nvox"] == v0["nvox"] == int(np.count_nonzero(w > 0))
    tol = 1e-13 if fixed else 1e-9
    for a, b in zip(g1, g0):
        assert rel_max(a, b) <= tol
