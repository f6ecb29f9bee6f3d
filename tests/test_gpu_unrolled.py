"""Parity of the unrolled adjoint (dmgs_vjp_unrolled) with its oracle
(oracle/unrolled.py), through the C ABI.

* rho, qbar, logD_bar and logmua_bar equal the oracle's to 1e-12 of the
  largest entry (2 and 3 levels of recursion, ragged c = 3 sizes, both face
  means, V(2,2), V(2,1), V(1,2) and V(0,2), g != 0).  At 128^3 and 192^3 the
  finest level runs the column-tile kernels with their boundary-plane
  companions and the coarser levels the x-march kernels.
* qbar equals dmgs_vjp's fixed-cycle pull-back.
* At 64^3, central differences of the library's own fixed-cycle forward map
  along random log D and log mua directions match <grad, direction>.
* Both policies for the recorded states (every cycle kept, or checkpoints
  and a second recording) meet the oracle.
* Plans the entry point does not take are rejected.
"""
import numpy as np
import pytest

from gpu_util import dev, host, rel_max, say

pytestmark = pytest.mark.gpu


def case(N, seed):
    from paper_2608_00760_amd import synth
    logD, logmu = synth.log_coefficients(N, seed, seed + 1)
    return logD, logmu, synth.normal(N, seed + 2), synth.normal(N, seed + 3)


def plan_for(N, logD, logmu, **kw):
    from paper_2608_00760_amd.solver import Options, Plan
    P = Plan(Options(N, **kw))
    P.set_log_coefficients(dev(logD), dev(logmu))
    return P


@pytest.mark.parametrize("N,n,nu,harmonic,g", [(8, 2, (2, 2), False, 0.0), (16, 3, (2, 1), True, 0.4),
                                               (24, 2, (2, 2), False, 0.0), (48, 2, (1, 2), True, 0.0),
                                               (16, 2, (0, 2), False, 0.3), (128, 2, (2, 2), True, 0.3),
                                               (192, 1, (2, 1), False, 0.0)])
def test_matches_oracle(N, n, nu, harmonic, g):
    from oracle import unrolled
    say("unrolled N=%d n=%d nu=%s harmonic=%s g=%g" % (N, n, nu, harmonic, g))
    logD, logmu, q, w = case(N, 200 + N)
    fm = "harmonic" if harmonic else "arith"
    P = plan_for(N, logD, logmu, fixed_cycles=n, nu_pre=nu[0], nu_post=nu[1], face_mean=fm, bc_value=g)
    (rho, (qb, gD, gmu)), info = P.vjp_unrolled(dev(q), dev(w))
    U = unrolled.Unrolled(np.exp(logD), np.exp(logmu), g=g, harmonic=harmonic)
    rr, (rqb, rgD, rgmu) = U.vjp(q, w, n, nu[0], nu[1])
    errs = {name: rel_max(host(a), b) for name, a, b in (("rho", rho, rr), ("qbar", qb, rqb), ("logD", gD, rgD),
                                                         ("logmua", gmu, rgmu))}
    say("errors", {k: "%.1e" % v for k, v in errs.items()})
    assert max(errs.values()) <= 1e-12, errs
    # the q-part is the fixed-cycle pull-back
    (qb2, _, _), _ = P.vjp(rho, dev(w), coef_grads=False)
    assert rel_max(host(qb), host(qb2)) <= 1e-12


@pytest.mark.parametrize("store", ["0", "1"])
@pytest.mark.parametrize("N,n,nu,harmonic,g", [(48, 3, (2, 1), True, 0.2), (96, 2, (1, 2), False, 0.0),
                                               (24, 3, (2, 0), False, 0.1), (96, 2, (1, 1), True, 0.0)])
def test_both_state_policies(store, N, n, nu, harmonic, g, monkeypatch):
    """The forward pass either keeps every cycle's recorded states or keeps
    the finest iterate per cycle and records each cycle again before its
    reverse pass (DMGS_UNROLLED_STORE = 1 / 0, read when the plan first
    allocates its buffers): both meet the oracle to 1e-12 (96^3: the finest
    level on the column tiles; V(2,0): the cycle's last state is its working
    iterate)."""
    from oracle import unrolled
    monkeypatch.setenv("DMGS_UNROLLED_STORE", store)
    say("unrolled store=%s N=%d n=%d nu=%s harmonic=%s g=%g" % (store, N, n, nu, harmonic, g))
    logD, logmu, q, w = case(N, 300 + N)
    fm = "harmonic" if harmonic else "arith"
    P = plan_for(N, logD, logmu, fixed_cycles=n, nu_pre=nu[0], nu_post=nu[1], face_mean=fm, bc_value=g)
    (rho, (qb, gD, gmu)), _ = P.vjp_unrolled(dev(q), dev(w))
    U = unrolled.Unrolled(np.exp(logD), np.exp(logmu), g=g, harmonic=harmonic)
    rr, (rqb, rgD, rgmu) = U.vjp(q, w, n, nu[0], nu[1])
    errs = {name: rel_max(host(a), b) for name, a, b in (("rho", rho, rr), ("qbar", qb, rqb), ("logD", gD, rgD),
                                                         ("logmua", gmu, rgmu))}
    say("errors", {k: "%.1e" % v for k, v in errs.items()})
    assert max(errs.values()) <= 1e-12, errs
    P.close()


def test_state_policy_falls_back_when_memory_is_short(monkeypatch):
    """With the policy left to the library, a plan whose states of every
    cycle would fit in a quarter of device memory tries to keep them; when
    the device has less free memory than that (the test occupies nearly all
    of it first), the first call falls back to checkpoints and still returns
    the checkpointed result, bitwise."""
    import torch
    monkeypatch.delenv("DMGS_UNROLLED_STORE", raising=False)
    N, n = 128, 15
    say("unrolled fallback N=%d n=%d" % (N, n))
    logD, logmu, q, w = case(N, 400)
    monkeypatch.setenv("DMGS_UNROLLED_STORE", "0")
    R = plan_for(N, logD, logmu, fixed_cycles=n)
    (r0, (qb0, gD0, gm0)), _ = R.vjp_unrolled(dev(q), dev(w))
    torch.cuda.synchronize()
    R.close()
    monkeypatch.delenv("DMGS_UNROLLED_STORE")
    P = plan_for(N, logD, logmu, fixed_cycles=n)
    qd, wd = dev(q), dev(w)
    torch.cuda.synchronize()
    # leave about 1.5 GB free: less than the 2.7 GB of every cycle's states,
    # more than the 0.6 GB of checkpoints and one cycle's states
    hog = []
    chunk = 8 << 30
    while True:
        free = torch.cuda.mem_get_info()[0]
        if free < (2 << 30):
            break
        size = min(chunk, free - (3 << 29))
        try:
            hog.append(torch.empty(size, dtype=torch.uint8, device="cuda:0"))
        except RuntimeError:
            chunk //= 2
            if chunk < (64 << 20):
                break
    say("  free while the call runs: %.2f GB" % (torch.cuda.mem_get_info()[0] / 1e9))
    try:
        (r1, (qb1, gD1, gm1)), _ = P.vjp_unrolled(qd, wd)
        torch.cuda.synchronize()
    finally:
        del hog
        torch.cuda.empty_cache()
    for a, b in ((r0, r1), (qb0, qb1), (gD0, gD1), (gm0, gm1)):
        assert torch.equal(a, b)
    P.close()


def test_central_differences_at_64():
    import torch
    say("unrolled 64^3 central differences")
    N, n = 64, 3
    logD, logmu, q, w = case(N, 64)
    P = plan_for(N, logD, logmu, fixed_cycles=n)
    (rho, (qb, gD, gmu)), _ = P.vjp_unrolled(dev(q), dev(w))
    rng = np.random.default_rng(65)
    eps = 1e-5
    for which in ("logD", "logmua"):
        v = rng.standard_normal(q.shape)
        vals = []
        for sgn in (1.0, -1.0):
            lD = logD + sgn * eps * v if which == "logD" else logD
            lm = logmu + sgn * eps * v if which == "logmua" else logmu
            Pe = plan_for(N, lD, lm, fixed_cycles=n)
            r, _ = Pe.forward(dev(q))
            vals.append(float((r * dev(w)).sum()))
            Pe.close()
        fd = (vals[0] - vals[1]) / (2 * eps)
        g = float(np.sum(host(gD if which == "logD" else gmu) * v))
        say(which, "fd %.10e grad %.10e" % (fd, g))
        assert abs(fd - g) <= 1e-6 * abs(g), (which, fd, g)


@pytest.mark.parametrize("N", [256, 512])
def test_paper_mode_at_full_size(N):
    """The paper's mode, 15 fixed V(2,2)-cycles, at 256^3 and 512^3 (inputs
    drawn on the device): qbar equals the fixed-cycle pull-back dmgs_vjp to
    1e-12, and central differences of the fixed-cycle forward map along one
    random log D and one random log mua direction match <grad, direction> to
    1e-6 (properties that hold at any size; the oracle pins the map at the
    small sizes above)."""
    import math
    import torch
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.solver import Options, Plan
    say("unrolled %d^3, 15 cycles" % N)
    n = 15
    d = torch.device("cuda:0")
    g = torch.Generator(device=d)
    g.manual_seed(7000 + N)
    logD = synth.grf_torch(N, g, d).clamp_(-math.log(100.0), math.log(100.0))
    logmu = math.log(0.05) + synth.grf_torch(N, g, d)
    q = synth.zero_boundary_torch(torch.randn(logD.shape, generator=g, device=d, dtype=torch.float64))
    w = synth.zero_boundary_torch(torch.randn(logD.shape, generator=g, device=d, dtype=torch.float64))

    def plan(lD, lm):
        P = Plan(Options(N, fixed_cycles=n))
        P.set_log_coefficients(lD, lm)
        return P
    P = plan(logD, logmu)
    (rho, (qb, gD, gmu)), _ = P.vjp_unrolled(q, w)
    (qb2, _, _), _ = P.vjp(rho, w)
    torch.cuda.synchronize()
    err = float((qb - qb2).abs().max() / qb2.abs().max())
    say("  qbar vs dmgs_vjp %.1e" % err)
    assert err <= 1e-12
    P.close()
    eps = 1e-5
    for which in ("logD", "logmua"):
        v = torch.randn(logD.shape, generator=g, device=d, dtype=torch.float64)
        vals = []
        for sgn in (1.0, -1.0):
            Pe = plan(logD + sgn * eps * v if which == "logD" else logD,
                      logmu + sgn * eps * v if which == "logmua" else logmu)
            r, _ = Pe.forward(q)
            vals.append(float((r * w).sum()))
            Pe.close()
        fd = (vals[0] - vals[1]) / (2 * eps)
        gr = float(((gD if which == "logD" else gmu) * v).sum())
        say("  %s fd %.10e grad %.10e" % (which, fd, gr))
        assert abs(fd - gr) <= 1e-6 * abs(gr), (which, fd, gr)


def test_rejects_other_plans():
    from paper_2608_00760_amd import _abi
    say("unrolled rejects")
    logD, logmu, q, w = case(16, 7)
    for kw in (dict(), dict(fixed_cycles=2, precision="fp32-in-fp64"), dict(fixed_cycles=2, smoother="wjacobi")):
        P = plan_for(16, logD, logmu, **kw)
        with pytest.raises(_abi.DMGSError) as e:
            P.vjp_unrolled(dev(q), dev(w))
        assert e.value.status == _abi.DMGS_ERR_INVALID


def test_autograd_unrolled_backward():
    """solve_unrolled's backward gives the bits of dmgs_vjp_unrolled."""
    import torch
    from paper_2608_00760_amd.autograd import solve_unrolled
    say("unrolled autograd")
    N, n = 24, 3
    logD, logmu, q, w = case(N, 24)
    P = plan_for(N, logD, logmu, fixed_cycles=n)
    tq, tD, tm = (dev(a).requires_grad_(True) for a in (q, logD, logmu))
    rho = solve_unrolled(tq, tD, tm, P)
    (rho * dev(w)).sum().backward()
    (rho2, (qb, gD, gmu)), _ = P.vjp_unrolled(dev(q), dev(w))
    assert bool((rho.detach() == rho2).all()) or rel_max(host(rho.detach()), host(rho2)) <= 1e-14
    for a, b in ((tq.grad, qb), (tD.grad, gD), (tm.grad, gmu)):
        assert bool((a == b).all())
