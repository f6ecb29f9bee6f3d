"""Residual histories (DMGS_TRACE=1, dmgs_trace_read), through the C ABI.

* Fixed-cycle mode, float64: after every cycle the recorded relative
  residual equals the oracle's for its own iterate after as many cycles
  (Sec. 2.4; the two iterates agree to 1e-12, so the residuals agree to
  1e-6 of their size), and the last entry is the reported one.
* Tolerance mode, float64 (where each iterate's norm comes from the next
  cycle's first pass) and float32-in-float64 (one entry per refinement
  step): one entry per cycle or step, the last equal to the reported
  relative residual and V-cycle count; the pull-back of dmgs_forward_vjp
  (run on the plan's second stream) is recorded under order 1.
* General-grid and 2D plans record one entry per cycle; the plan times its
  kernels without dmgs_timing_enable; reading with tracing off is an error.
"""
import numpy as np
import pytest

from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


def make(N, monkeypatch, seed, **kw):
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.solver import Options, Plan
    monkeypatch.setenv("DMGS_TRACE", "1")
    c = synth.grf_case(N, seed, ndim=kw.get("ndim", 3))
    P = Plan(Options(N, **kw))
    P.set_coefficients(dev(c["D"]), dev(c["mua"]))
    return P, c


def test_fixed_cycles_history_matches_oracle(monkeypatch):
    from oracle import ref
    N, n = 48, 6
    say("trace fixed N=%d n=%d" % (N, n))
    P, c = make(N, monkeypatch, 5100, fixed_cycles=n)
    rho, info = P.forward(dev(c["q"]))
    tr = P.trace(0)
    assert [t[0] for t in tr] == list(range(1, n + 1)) and [t[1] for t in tr] == list(range(1, n + 1))
    assert tr[-1][2] == info["rel_residual"]
    H = ref.Hierarchy(c["D"], c["mua"])
    r0 = np.linalg.norm(H.defect(0, np.zeros_like(c["q"]), c["q"]))
    for k, (_, _, rel) in enumerate(tr, start=1):
        u, _ = H.forward(c["q"], fixed_cycles=k)
        ref_rel = np.linalg.norm(H.defect(0, u, c["q"])) / r0
        say("  cycle %d: %.6e (oracle %.6e)" % (k, rel, ref_rel))
        assert abs(rel - ref_rel) <= 1e-6 * ref_rel
    assert all(b < a for (_, _, a), (_, _, b) in zip(tr, tr[1:]))


@pytest.mark.parametrize("precision", ["fp64", "fp32-in-fp64"])
def test_tolerance_history(precision, monkeypatch):
    N = 64
    say("trace tolerance %s N=%d" % (precision, N))
    P, c = make(N, monkeypatch, 5200, precision=precision)
    rho, fi = P.forward(dev(c["q"]))
    tr = P.trace(0)
    say("  forward", [(s, v, "%.2e" % r) for s, v, r in tr])
    assert len(tr) == fi["cycles"] and [t[0] for t in tr] == list(range(1, fi["cycles"] + 1))
    assert tr[-1][2] == fi["rel_residual"] and tr[-1][1] == fi["vcycles"]
    assert tr[-1][2] <= 1e-10 < tr[-2][2]
    (qb, _, _), vi = P.vjp(rho, dev(c["rhobar"]))
    ta = P.trace(1)
    assert len(ta) == vi["cycles"] and ta[-1][2] == vi["rel_residual"]
    assert P.trace(0) == tr   # the pull-back keeps the forward's history
    (_, _), fi2, vi2 = P.forward_vjp(dev(c["q"]), dev(c["rhobar"]))
    tb = P.trace(1)
    assert len(tb) == vi2["cycles"] and tb[-1][2] == vi2["rel_residual"]
    t = P.timing_read()
    assert t["smooth"]["launches"] > 0


def test_grid_2d_and_errors(monkeypatch):
    from paper_2608_00760_amd import _abi, synth
    from paper_2608_00760_amd.solver import Options, Plan
    say("trace grid / 2d / errors")
    monkeypatch.setenv("DMGS_TRACE", "1")
    cells = (32, 16, 16)
    g = synth.grid_case(cells, 5300)
    P = Plan(Options(cells[0], shape=cells, spacing=(1.0, 0.5, 0.5), fixed_cycles=3))
    P.set_log_coefficients(dev(g["logD"]), dev(g["logmua"]))
    _, info = P.forward(dev(g["q"]))
    tr = P.trace(0)
    assert len(tr) == 3 and tr[-1][2] == info["rel_residual"]
    Q, c = make(128, monkeypatch, 5400, ndim=2)
    _, info = Q.forward(dev(c["q"]))
    tr = Q.trace(0)
    assert len(tr) == info["cycles"] and tr[-1][2] == info["rel_residual"]
    with pytest.raises(_abi.DMGSError):
        Q.trace(2)
    monkeypatch.setenv("DMGS_TRACE", "0")
    c = synth.grf_case(32, 5500)
    R2 = Plan(Options(32))
    R2.set_coefficients(dev(c["D"]), dev(c["mua"]))
    R2.forward(dev(c["q"]))
    with pytest.raises(_abi.DMGSError):
        R2.trace(0)
