"""dmgs_solve_once_noalloc (the solve in the library's static scratch array)
against dmgs_solve_once, through the C ABI.

Two calls in a row on each case, the second with a smaller grid, so the
second runs on what the first left in the array.  Tolerance-mode results of
both entry points run the same kernels in the same order, so they agree to
rounding (asserted to 1e-13 of the largest entry; they are normally bitwise
equal); the residual the call reports meets the tolerance.  Also: a plan
beyond the array's size is rejected before any device work, and errors of
the inputs are reported like dmgs_solve_once's.
"""
import numpy as np
import pytest

from gpu_util import dev, rel_max, say

pytestmark = pytest.mark.gpu


def run_pair(opts, case):
    from paper_2608_00760_amd import solver
    D, mu, q = dev(case["D"]), dev(case["mua"]), dev(case["q"])
    ref, ri = solver.solve_once(opts, D, mu, q)
    out, oi = solver.solve_once_noalloc(opts, D, mu, q)
    import torch
    torch.cuda.synchronize()
    e = rel_max(out.cpu().numpy(), ref.cpu().numpy())
    same = bool(torch.equal(out, ref))
    say("noalloc N=%d ndim=%d %s fixed=%d: cycles %d/%d rel res %.2e, max rel diff %.1e, bitwise %s"
        % (opts.N, opts.ndim, opts.precision, opts.fixed_cycles, oi["cycles"], ri["cycles"], oi["rel_residual"], e, same))
    assert oi["status"] == 0 and ri["status"] == 0
    assert oi["cycles"] == ri["cycles"]
    assert e <= 1e-13
    if opts.fixed_cycles == 0:
        assert oi["rel_residual"] <= opts.rtol
    return out


@pytest.mark.parametrize("precision", ["fp32-in-fp64", "fp64"])
def test_noalloc_matches_solve_once_twice(precision):
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.solver import Options
    for N in (96, 64):   # the second call smaller than the first
        case = synth.grf_case(N, 6100 + N)
        run_pair(Options(N, precision=precision), case)


def test_noalloc_fixed_cycles_2d_and_ragged():
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.solver import Options
    run_pair(Options(128, precision="fp32-in-fp64", fixed_cycles=4), synth.grf_case(128, 6201))
    run_pair(Options(48, fixed_cycles=3, face_mean="harmonic", bc_value=0.5), synth.grf_case(48, 6202))
    run_pair(Options(512, ndim=2), synth.grf_case(512, 6203, ndim=2))
    run_pair(Options(24, ndim=3), synth.grf_case(24, 6204))


def test_noalloc_rejects_what_does_not_fit_and_bad_input():
    import torch
    from paper_2608_00760_amd import _abi, synth
    from paper_2608_00760_amd.solver import Options, solve_once_noalloc, workspace_bytes
    big = Options(192, precision="fp32-in-fp64")
    assert workspace_bytes(big) > _abi.DMGS_NOALLOC_SCRATCH_BYTES
    z = torch.zeros((193,) * 3, dtype=torch.float64, device="cuda:0")
    with pytest.raises(_abi.DMGSError) as ei:
        solve_once_noalloc(big, z + 1.0, z + 0.1, z)
    assert ei.value.status == _abi.DMGS_ERR_INVALID and "static scratch" in str(ei.value)
    c = synth.grf_case(32, 6301)
    D = c["D"].copy()
    D[5, 5, 5] = -1.0
    with pytest.raises(_abi.DMGSError) as ei:
        solve_once_noalloc(Options(32), dev(D), dev(c["mua"]), dev(c["q"]))
    assert ei.value.status == _abi.DMGS_ERR_INVALID
    # a good call right after the failed one
    from paper_2608_00760_amd.solver import solve_once
    out, _ = solve_once_noalloc(Options(32), dev(c["D"]), dev(c["mua"]), dev(c["q"]))
    ref, _ = solve_once(Options(32), dev(c["D"]), dev(c["mua"]), dev(c["q"]))
    assert rel_max(out.cpu().numpy(), ref.cpu().numpy()) <= 1e-13
