"""Parity of the two-dimensional (five-point) variant with the 2D oracle,
through the C ABI (plans with ndim = 2, float64).

* Fixed-cycle mode: forward, push-forward and pull-back with all gradients
  equal the oracle's to 1e-12 of the largest entry (both face means, ragged
  c = 3 sizes, V(2,2) and V(2,1), Dirichlet value g != 0); the dot-product
  identity holds on the GPU alone.
* Tolerance mode: residual <= 1e-10 by the oracle's operator; solution and
  gradients against the oracle's (solved to 1e-13) to 1e-8.
* Single-level grids (N = 2, 3), the constant-coefficient closed form, the
  replayed adjoint schedule, forward + VJP together, bitwise determinism.
* The largest size of the benchmark sweep (8192^2 cells, 15 fixed cycles):
  the dot-product identity <S_15 q, w> = <q, S_15^T w>, which holds at any
  size, and the residual reduction.
"""
import numpy as np
import pytest

from gpu_util import dev, host, rel_max, say

pytestmark = pytest.mark.gpu


def case(N, seed):
    from paper_2608_00760_amd import synth
    c = synth.grf_case(N, seed, ndim=2)
    c.update({k: v for k, v in synth.tangents(N, seed + 100, ndim=2).items() if k != "rhobar"})
    return c


def plan_for(c, **kw):
    from paper_2608_00760_amd.solver import Options, Plan
    N = c["D"].shape[0] - 1
    P = Plan(Options(N, ndim=2, **kw))
    P.set_coefficients(dev(c["D"]), dev(c["mua"]))
    return P


def oracle_for(c, **kw):
    from oracle import ref2d
    return ref2d.Hierarchy2D(c["D"], c["mua"], **kw)


@pytest.mark.parametrize("N,n,face_mean,nu", [(8, 4, "arith", (2, 2)), (48, 3, "harmonic", (2, 2)),
                                              (128, 3, "arith", (2, 1)), (96, 2, "arith", (1, 3)),
                                              (256, 3, "harmonic", (2, 2))])
def test_fixed_cycles_match_oracle(N, n, face_mean, nu):
    say("2d fixed N=%d n=%d %s nu=%s" % (N, n, face_mean, nu))
    c = case(N, 50 + N)
    P = plan_for(c, fixed_cycles=n, face_mean=face_mean, nu_pre=nu[0], nu_post=nu[1])
    H = oracle_for(c, face_mean=face_mean)
    kw = dict(fixed_cycles=n, nu1=nu[0], nu2=nu[1])
    rho, info = P.forward(dev(c["q"]))
    rr, _ = H.forward(c["q"], **kw)
    assert info["cycles"] == n
    assert rel_max(host(rho), rr) <= 1e-12
    drho, _ = P.jvp(rho, dev(c["dq"]), dev(c["dlogD"]), dev(c["dlogmua"]))
    dr, _ = H.jvp(rr, c["dq"], c["dlogD"], c["dlogmua"], **kw)
    assert rel_max(host(drho), dr) <= 1e-12
    (qb, gD, gmu), _ = P.vjp(rho, dev(c["rhobar"]))
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], **kw)
    for g, r in ((qb, rqb), (gD, rgD), (gmu, rgmu)):
        assert rel_max(host(g), r) <= 1e-12
    lhs = float((drho * dev(c["rhobar"])).sum())
    rhs = float((dev(c["dq"]) * qb).sum() + (dev(c["dlogD"]) * gD).sum() + (dev(c["dlogmua"]) * gmu).sum())
    assert abs(lhs - rhs) <= 1e-12 * float(drho.norm()) * float(np.linalg.norm(c["rhobar"]))


@pytest.mark.parametrize("N,chunk,nu,g,face_mean", [(48, 8, (2, 2), 0.0, "arith"), (128, 16, (2, 1), 0.3, "arith"),
                                                    (256, 0, (3, 2), 0.0, "arith"), (96, 24, (1, 3), 0.0, "arith"),
                                                    (192, 32, (2, 2), 0.2, "harmonic")])
def test_two_sweep_passes_on_every_level(monkeypatch, N, chunk, nu, g, face_mean):
    """The two-sweep passes (used on large levels) forced onto every level
    that smooths, with short row chunks, odd sweep counts and g != 0."""
    monkeypatch.setenv("DMGS_2D_SWEEP2_MIN", "4")
    if chunk:
        monkeypatch.setenv("DMGS_2D_CHUNK", str(chunk))
    say("2d two-sweep passes N=%d chunk=%d nu=%s g=%g" % (N, chunk, nu, g))
    c = case(N, 60 + N)
    n = 3
    P = plan_for(c, fixed_cycles=n, nu_pre=nu[0], nu_post=nu[1], bc_value=g, face_mean=face_mean)
    H = oracle_for(c, g=g, face_mean=face_mean)
    kw = dict(fixed_cycles=n, nu1=nu[0], nu2=nu[1])
    rho, _ = P.forward(dev(c["q"]))
    rr, _ = H.forward(c["q"], **kw)
    assert rel_max(host(rho), rr) <= 1e-12
    (qb, gD, gmu), _ = P.vjp(rho, dev(c["rhobar"]))
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], **kw)
    for a, b in ((qb, rqb), (gD, rgD), (gmu, rgmu)):
        assert rel_max(host(a), b) <= 1e-12
    drho, _ = P.jvp(rho, dev(c["dq"]), dev(c["dlogD"]), dev(c["dlogmua"]))
    dr, _ = H.jvp(rr, c["dq"], c["dlogD"], c["dlogmua"], **kw)
    assert rel_max(host(drho), dr) <= 1e-12


@pytest.mark.parametrize("N,nu,g,face_mean", [(48, (2, 2), 0.0, "arith"), (96, (2, 2), 0.3, "harmonic"),
                                              (192, (2, 2), 0.0, "arith"), (96, (2, 1), 0.0, "arith")])
def test_block_passes_on_every_level(monkeypatch, N, nu, g, face_mean):
    """The LDS block passes (used on mid-size levels) forced onto every
    level that smooths, the finest included (g != 0); V(2,1) takes the
    per-operator path."""
    monkeypatch.setenv("DMGS_2D_BLOCK_MIN", "4")
    say("2d block passes N=%d nu=%s g=%g %s" % (N, nu, g, face_mean))
    c = case(N, 80 + N)
    n = 3
    P = plan_for(c, fixed_cycles=n, nu_pre=nu[0], nu_post=nu[1], bc_value=g, face_mean=face_mean)
    H = oracle_for(c, g=g, face_mean=face_mean)
    kw = dict(fixed_cycles=n, nu1=nu[0], nu2=nu[1])
    rho, _ = P.forward(dev(c["q"]))
    rr, _ = H.forward(c["q"], **kw)
    assert rel_max(host(rho), rr) <= 1e-12
    (qb, gD, gmu), _ = P.vjp(rho, dev(c["rhobar"]))
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], **kw)
    for a, b in ((qb, rqb), (gD, rgD), (gmu, rgmu)):
        assert rel_max(host(a), b) <= 1e-12


def test_large_grid_fixed_cycles_match_oracle():
    """768^2 cells: the two-sweep passes on levels 0 (and the half-sweeps
    below), against the oracle."""
    say("2d fixed N=768")
    N = 768
    c = case(N, 768)
    P = plan_for(c, fixed_cycles=2)
    H = oracle_for(c)
    rho, _ = P.forward(dev(c["q"]))
    rr, _ = H.forward(c["q"], fixed_cycles=2)
    assert rel_max(host(rho), rr) <= 1e-12
    (qb, _, _), _ = P.vjp(rho, dev(c["rhobar"]), coef_grads=False)
    rqb, _ = H.pullback(c["rhobar"], fixed_cycles=2)
    assert rel_max(host(qb), rqb) <= 1e-12


@pytest.mark.parametrize("N", [2, 3, 4, 6, 12])
def test_small_grids_and_boundary_value(N):
    say("2d small N=%d" % N)
    c = case(N, 7 + N)
    g = 0.45
    P = plan_for(c, fixed_cycles=2, bc_value=g)
    H = oracle_for(c, g=g)
    rho, _ = P.forward(dev(c["q"]))
    rr, _ = H.forward(c["q"], fixed_cycles=2)
    assert rel_max(host(rho), rr) <= 1e-12
    (qb, gD, gmu), _ = P.vjp(rho, dev(c["rhobar"]))
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], fixed_cycles=2)
    for a, b in ((qb, rqb), (gD, rgD), (gmu, rgmu)):
        assert rel_max(host(a), b) <= 1e-12


def test_tolerance_mode_matches_oracle():
    say("2d tolerance N=512")
    N = 512
    c = case(N, 91)
    P = plan_for(c)
    H = oracle_for(c)
    rho, info = P.forward(dev(c["q"]))
    u = host(rho)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-10
    assert np.linalg.norm(H.defect(0, u, c["q"])) <= 1e-10 * np.linalg.norm(H.defect(0, 0 * u, c["q"]))
    (qb, gD, gmu), vinfo = P.vjp(rho, dev(c["rhobar"]))
    assert vinfo["status"] == 0 and vinfo["rel_residual"] <= 1e-10
    rr, _ = H.forward(c["q"], rtol=1e-13)
    (rqb, rgD, rgmu), _ = H.vjp(rr, c["rhobar"], rtol=1e-13)
    errs = {"u": rel_max(u, rr), "q": rel_max(host(qb), rqb), "logD": rel_max(host(gD), rgD),
            "logmua": rel_max(host(gmu), rgmu)}
    say("errors", {k: "%.2e" % v for k, v in errs.items()}, "cycles", info["cycles"], vinfo["cycles"])
    assert max(errs.values()) <= 1e-8, errs


def test_constant_coefficients_closed_form():
    import scipy.fft
    say("2d closed form")
    N, Dc, muc = 64, 1.3, 0.2
    D = np.full((N + 1, N + 1), Dc)
    mu = np.full((N + 1, N + 1), muc)
    from paper_2608_00760_amd import synth
    q = synth.zero_boundary(synth.blob(N, (0.4 * N, 0.55 * N), 7.0))
    P = plan_for({"D": D, "mua": mu}, rtol=1e-13)
    rho, info = P.forward(dev(q))
    k = np.arange(1, N)
    lam = Dc * ((2 - 2 * np.cos(np.pi * k / N))[:, None] + (2 - 2 * np.cos(np.pi * k / N))[None, :]) + muc
    exact = scipy.fft.idstn(scipy.fft.dstn(q[1:-1, 1:-1], type=1) / lam, type=1)
    assert info["status"] == 0
    assert np.abs(host(rho)[1:-1, 1:-1] - exact).max() <= 1e-11 * np.abs(exact).max()


def test_adjoint_schedule_forward_vjp_and_determinism():
    say("2d adjoint schedule, forward_vjp")
    N = 256
    c = case(N, 33)
    P = plan_for(c, adjoint_schedule=True)
    rho, fi = P.forward(dev(c["q"]))
    n = fi["cycles"]
    (qb, gD, gmu), vi = P.vjp(rho, dev(c["rhobar"]))
    assert vi["cycles"] == n
    H = oracle_for(c)
    rr, _ = H.forward(c["q"], fixed_cycles=n)
    (rqb, _, _), _ = H.vjp(rr, c["rhobar"], fixed_cycles=n)
    assert rel_max(host(qb), rqb) <= 1e-12
    for rep in range(2):
        (rho2, (qb2, gD2, gmu2)), f2, v2 = P.forward_vjp(dev(c["q"]), dev(c["rhobar"]))
        assert f2["status"] == 0 and v2["cycles"] == n
        for a, b in ((rho, rho2), (qb, qb2), (gD, gD2), (gmu, gmu2)):
            assert bool((a == b).all()), rep
    P2 = plan_for(c)
    (rho3, (qb3, _, _)), _, v3 = P2.forward_vjp(dev(c["q"]), dev(c["rhobar"]))
    assert bool((rho3 == rho).all()) and v3["status"] == 0
    (qb4, _, _), _ = P2.vjp(rho, dev(c["rhobar"]))
    assert bool((qb3 == qb4).all())


def test_benchmark_size_dot_product_identity():
    """8192^2 cells (2^26 vertices), 15 fixed V(2,2)-cycles."""
    import torch
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.solver import Options, Plan
    say("2d N=8192 fixed 15")
    N, n = 8192, 15
    g = torch.Generator(device="cuda:0")
    g.manual_seed(8192)
    logD = synth.grf_torch(N, g, "cuda:0", ndim=2).clamp_(-np.log(100.0), np.log(100.0))
    logmu = np.log(0.05) + synth.grf_torch(N, g, "cuda:0", ndim=2)
    q = synth.zero_boundary_torch(torch.randn((N + 1, N + 1), generator=g, device="cuda:0", dtype=torch.float64))
    w = synth.zero_boundary_torch(torch.randn((N + 1, N + 1), generator=g, device="cuda:0", dtype=torch.float64))
    P = Plan(Options(N, ndim=2, fixed_cycles=n))
    P.set_log_coefficients(logD, logmu)
    rho, info = P.forward(q)
    assert info["cycles"] == n and info["rel_residual"] <= 1e-6, info
    (qb, _, _), _ = P.vjp(rho, w, coef_grads=False)
    lhs = float((rho * w).sum())
    rhs = float((q * qb).sum())
    say("identity", lhs, rhs, "rel residual", info["rel_residual"])
    assert abs(lhs - rhs) <= 1e-12 * float(rho.norm()) * float(w.norm())
