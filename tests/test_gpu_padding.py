"""Padded rows on the finest level of refinement plans (DMGS_PAD), through
the C ABI.

The padded layout changes only where the finest level's float32 arrays sit
in memory: every pass computes the same values in the same order, so each
entry point returns bitwise the result of a plan with dense arrays
(DMGS_PAD=0).  Checked for the forward solve, push-forward, pull-back, the
concurrent forward + pull-back and the likelihood gradient, for both face
means, tolerance and fixed-cycle modes, and with pre-smoothing passes that
do not write the defect (the restriction then reads the padded iterate,
right-hand side and coefficients itself).  The float32 passes on padded
levels also meet the oracle pass by pass in test_gpu_kernels (N = 96, 128).
"""
import numpy as np
import pytest

from gpu_util import dev, say

pytestmark = pytest.mark.gpu

CASES = [
    (96, "arith", 0, {}),
    (128, "harmonic", 0, {}),
    (96, "harmonic", 3, {"DMGS_SWEEP2_DEFECT": "0"}),
    (128, "arith", 0, {"DMGS_SWEEP2_DEFECT": "1"}),
]


def run_all(N, face_mean, fixed, env, pad, monkeypatch):
    import torch
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.solver import Options, Plan
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    monkeypatch.setenv("DMGS_PAD", "1" if pad else "0")
    c = synth.grf_case(N, 9100 + N)
    t = synth.tangents(N, 9200 + N)
    P = Plan(Options(N, precision="fp32-in-fp64", face_mean=face_mean, fixed_cycles=fixed))
    P.set_coefficients(dev(c["D"]), dev(c["mua"]))
    out = {"bytes": P.bytes}
    rho, fi = P.forward(dev(c["q"]))
    out["rho"] = rho
    out["drho"], _ = P.jvp(rho, dev(t["dq"]), dev(t["dlogD"]), dev(t["dlogmua"]))
    out["vjp"], vi = P.vjp(rho, dev(c["rhobar"]))
    (r2, g2), _, _ = P.forward_vjp(dev(c["q"]), dev(c["rhobar"]))
    out["fv"] = (r2,) + tuple(g2)
    # data and weights of a synthetic measurement (no solver output involved)
    d = c["mua"] * np.abs(synth.normal(N, 9300 + N))
    w = np.zeros_like(d)
    w[3:-3, 3:-3, 3:-3] = 4.0
    (r3, val, g3), _, _ = P.likelihood_grad(dev(c["q"]), dev(d), dev(w))
    out["lik"] = (r3,) + tuple(g3)
    out["val"] = (val["H"], val["chi2"], val["nvox"])
    out["cycles"] = (fi["cycles"], fi["vcycles"], vi["cycles"])
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("N,face_mean,fixed,env", CASES)
def test_padded_equals_dense(N, face_mean, fixed, env, monkeypatch):
    import torch
    say("padding N=%d %s fixed=%d %s" % (N, face_mean, fixed, env))
    a = run_all(N, face_mean, fixed, env, True, monkeypatch)
    b = run_all(N, face_mean, fixed, env, False, monkeypatch)
    # the padded plan really is padded: its float32 arrays are larger
    assert a["bytes"] > b["bytes"]
    assert a["cycles"] == b["cycles"] and a["val"] == b["val"]
    for key in ("rho", "drho", "vjp", "fv", "lik"):
        xa = a[key] if isinstance(a[key], tuple) else (a[key],)
        xb = b[key] if isinstance(b[key], tuple) else (b[key],)
        for i, (u, v) in enumerate(zip(xa, xb)):
            if u is None:
                assert v is None
                continue
            assert torch.equal(u, v), (key, i)
