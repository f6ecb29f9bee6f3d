"""Fixed-cycle solves captured into a HIP graph.

With fixed_cycles > 0, timing off and a NULL info, dmgs_forward, dmgs_jvp
and dmgs_vjp make no host synchronisation and allocate nothing, so a caller
can capture them on its own stream.  One graph holds a forward solve, a JVP
at its result and a VJP with both coefficient gradients.  It is replayed
three times, with the outputs poisoned before each replay and the plan's own
eager calls run between replays, and every replay must give the bits of the
eager calls (3D float64, 3D float32-in-float64 through the two-sweep and
block passes, 2D).
"""
import ctypes as C

import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


@pytest.mark.parametrize("ndim,N,precision", [(3, 24, "fp64"), (3, 64, "fp32-in-fp64"), (2, 96, "fp64")])
def test_captured_fixed_cycle_calls_replay_bitwise(ndim, N, precision):
    import torch
    from paper_2608_00760_amd import _abi, synth
    from paper_2608_00760_amd.solver import Options, Plan
    say("graph capture ndim=%d N=%d %s" % (ndim, N, precision))
    lib = _abi.lib()
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(900 + N)
    shape = (N + 1,) * ndim
    rnd = lambda: torch.randn(shape, generator=g, device=dev, dtype=torch.float64)
    logD, logmu = 0.5 * rnd(), -3.0 + 0.5 * rnd()
    q, w, dq, dD, dm = rnd(), rnd(), rnd(), rnd(), rnd()
    for t in (q, w, dq, dm):
        synth.zero_boundary_torch(t)
    P = Plan(Options(N, precision=precision, fixed_cycles=4, ir_inner_cycles=1, ir_adaptive=False, ndim=ndim))
    P.set_log_coefficients(logD, logmu)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()

    def calls(outs, st):
        rho, drho, qb, gD, gmu = outs
        sp = C.c_void_p(st.cuda_stream)
        for name, args in (("dmgs_forward", (ptr(q), ptr(rho))),
                           ("dmgs_jvp", (ptr(rho), ptr(dq), ptr(dD), ptr(dm), ptr(drho))),
                           ("dmgs_vjp", (ptr(rho), ptr(w), ptr(qb), ptr(gD), ptr(gmu)))):
            status = getattr(lib, name)(P._h, *args, None, sp)
            assert status == 0, (name, status, lib.dmgs_last_error())

    eager = [torch.empty_like(q) for _ in range(5)]
    with torch.cuda.stream(s):
        calls(eager, s)
    s.synchronize()
    ref = [t.clone() for t in eager]
    assert all(bool(torch.isfinite(t).all()) for t in ref)

    outs = [torch.empty_like(q) for _ in range(5)]
    G = torch.cuda.CUDAGraph()
    with torch.cuda.graph(G, stream=s):
        calls(outs, s)
    torch.cuda.synchronize()
    for rep in range(3):
        for t in outs:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        G.replay()
        torch.cuda.synchronize()
        same = [bool(torch.equal(a, b)) for a, b in zip(outs, ref)]
        say("replay", rep, "bitwise equal", same)
        assert all(same), same
        # the plan's own eager calls between replays
        with torch.cuda.stream(s):
            calls(eager, s)
        s.synchronize()
        assert all(bool(torch.equal(a, b)) for a, b in zip(eager, ref))
    del G
    P.close()
