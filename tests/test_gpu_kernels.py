"""Kernel-level parity of the HIP passes with the oracle (through the C ABI).

Each pass of the cycle -- coefficient hierarchy, operator, pre-smoothing pass
(sweeps, defect, restriction), post-smoothing pass (prolongation, sweeps) and
the coarsest exact solve -- runs on the GPU and in the oracle on the same
seeded inputs, on every level of grids that span several tiles and have
ragged tails.

Tolerances: float64 passes agree to 1e-13 of the largest entry (rounding
order and fused multiply-adds only).  The restricted defect R(q - A u) is a
difference of terms of size |q| and |A u| that largely cancel after
smoothing, so its rounding error is measured against max|q| + max|A u|
rather than against its own size.  Float32 passes run on float32-rounded
inputs and coefficients rounded to float32, so they agree to 2e-5 on the
same scales (a few float32 roundings per update, over two sweeps).
"""
import numpy as np
import pytest

from gpu_util import dev, host, rel_max, say

pytestmark = pytest.mark.gpu

SIZES = [8, 24, 32, 96, 128]


def make(N, seed, precision="fp64", face_mean="arith"):
    from oracle import ref
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.solver import Options, Plan
    logD, logmu = synth.log_coefficients(N, seed, seed + 1)
    D, mu = np.exp(logD), np.exp(logmu)
    P = Plan(Options(N, precision=precision, face_mean=face_mean))
    P.set_coefficients(dev(D), dev(mu))
    H = ref.Hierarchy(D, mu, face_mean=face_mean)
    return P, H


def oracle_pre(H, k, u, q, order, nu=2):
    first = 1 if order else 0
    for _ in range(nu):
        u = H.gs_half(k, first, u, q)
        u = H.gs_half(k, 1 - first, u, q)
    return u, H.restrict(k, H.defect(k, u, q))


def defect_scale(H, k, u, q):
    """Size of the terms whose difference is the defect q - A u."""
    return np.abs(q).max() + np.abs(H.apply(k, u)).max()


def oracle_post(H, k, u, ec, q, order, nu=2):
    u = H.prolong_add(k, ec, u)
    first = 1 if order else 0
    for _ in range(nu):
        u = H.gs_half(k, first, u, q)
        u = H.gs_half(k, 1 - first, u, q)
    return u


@pytest.mark.parametrize("N", SIZES)
@pytest.mark.parametrize("face_mean", ["arith", "harmonic"])
def test_coefficient_hierarchy(N, face_mean):
    say("hierarchy N=%d %s" % (N, face_mean))
    P, H = make(N, 10 + N, face_mean=face_mean)
    assert P.levels == H.L and P.level_N == H.Ns
    for k in range(P.levels):
        D, mu = P.debug_level_coefficients(k)
        Dr, mur = H.level_coef(k)
        assert rel_max(host(D), Dr) <= 1e-15
        assert rel_max(host(mu), mur) <= 1e-15


@pytest.mark.parametrize("N", SIZES)
def test_operator_apply(N):
    from paper_2608_00760_amd import synth
    say("apply N=%d" % N)
    P, H = make(N, 20 + N)
    for k in range(P.levels):
        u = synth.normal(H.Ns[k], 7)
        assert rel_max(host(P.debug_apply(k, dev(u))), H.apply(k, u)) <= 1e-13


# Float64 pass variants: the plan's default (two-sweep passes from N = 16)
# and one-sweep streaming passes on every level.
FP64_VARIANTS = {"default": {}, "one_sweep": {"DMGS_SWEEP2_MIN": "100000"}}


@pytest.mark.parametrize("N", SIZES)
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("face_mean", ["arith", "harmonic"])
@pytest.mark.parametrize("variant", list(FP64_VARIANTS))
def test_pre_and_post_passes_fp64(N, order, face_mean, variant, monkeypatch):
    from paper_2608_00760_amd import synth
    say("passes fp64 N=%d order=%d %s %s" % (N, order, face_mean, variant))
    for key, val in FP64_VARIANTS[variant].items():
        monkeypatch.setenv(key, val)
    P, H = make(N, 30 + N, face_mean=face_mean)
    for k in range(P.levels - 1):
        Nk = H.Ns[k]
        u, q = synth.normal(Nk, 1 + k), synth.normal(Nk, 2 + k)
        ec = synth.normal(H.Ns[k + 1], 3 + k)
        gu, gqc = P.debug_pre(k, dev(u), dev(q), order=order)
        ru, rqc = oracle_pre(H, k, u, q, order)
        assert rel_max(host(gu), ru) <= 1e-13, (k, "pre u")
        assert np.abs(host(gqc) - rqc).max() <= 1e-13 * defect_scale(H, k, ru, q), (k, "pre qc")
        gp = P.debug_post(k, dev(u), dev(ec), dev(q), order=order)
        assert rel_max(host(gp), oracle_post(H, k, u, ec, q, order)) <= 1e-13, (k, "post")


# Float32 smoothing-pass variants: the plan's default choice, two-sweep
# passes forced on every level with N >= 16 (several x-chunks), and the same
# with one chunk per tile column.
# the two-sweep pre-smoothing writes the defect (the restriction then reads
# it) unless DMGS_SWEEP2_DEFECT=0, which keeps the fused defect-restriction
PASS_VARIANTS = {"default": {}, "sweep2": {"DMGS_SWEEP2_MIN": "16"},
                 "sweep2_one_chunk": {"DMGS_SWEEP2_MIN": "16", "DMGS_SWEEP2_WGS": "16"},
                 "sweep2_no_defect": {"DMGS_SWEEP2_MIN": "16", "DMGS_SWEEP2_DEFECT": "0"}}


@pytest.mark.parametrize("N", SIZES)
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("variant", list(PASS_VARIANTS))
def test_pre_and_post_passes_fp32(N, order, variant, monkeypatch):
    from paper_2608_00760_amd import synth
    import torch
    say("passes fp32 N=%d order=%d %s" % (N, order, variant))
    for key, val in PASS_VARIANTS[variant].items():
        monkeypatch.setenv(key, val)
    P, H = make(N, 40 + N, precision="fp32-in-fp64")
    for k in range(P.levels - 1):
        Nk = H.Ns[k]
        f32 = lambda a: a.astype(np.float32).astype(np.float64)
        u, q = f32(synth.normal(Nk, 1 + k)), f32(synth.normal(Nk, 2 + k))
        ec = f32(synth.normal(H.Ns[k + 1], 3 + k))
        gu, gqc = P.debug_pre(k, dev(u, torch.float32), dev(q, torch.float32), order=order, fp32=True)
        ru, rqc = oracle_pre(H, k, u, q, order)
        assert rel_max(host(gu), ru) <= 2e-5, (k, "pre u")
        assert np.abs(host(gqc) - rqc).max() <= 2e-5 * defect_scale(H, k, ru, q), (k, "pre qc")
        # from the zero iterate (coarse levels, first float32 cycle)
        gz, gzc = P.debug_pre(k, None, dev(q, torch.float32), order=order, fp32=True)
        rz, rzc = oracle_pre(H, k, np.zeros_like(q), q, order)
        assert rel_max(host(gz), rz) <= 2e-5, (k, "pre from zero u")
        assert np.abs(host(gzc) - rzc).max() <= 2e-5 * defect_scale(H, k, rz, q), (k, "pre from zero qc")
        gp = P.debug_post(k, dev(u, torch.float32), dev(ec, torch.float32), dev(q, torch.float32), order=order, fp32=True)
        assert rel_max(host(gp), oracle_post(H, k, u, ec, q, order)) <= 2e-5, (k, "post")


@pytest.mark.parametrize("N", [8, 24, 2, 3])
def test_coarsest_exact_solve(N):
    from paper_2608_00760_amd import synth
    import torch
    say("coarsest N=%d" % N)
    for prec in ("fp64", "fp32-in-fp64"):
        P, H = make(N, 50 + N, precision=prec)
        k = P.levels - 1
        q = synth.normal(H.Ns[k], 5)
        expect = H.exact_solve(k, q)
        if prec == "fp64":
            got = host(P.debug_coarsest(dev(q)))
            assert rel_max(got, expect) <= 1e-13
        else:
            q32 = q.astype(np.float32).astype(np.float64)
            got = host(P.debug_coarsest(dev(q32, torch.float32), fp32=True))
            assert rel_max(got, H.exact_solve(k, q32)) <= 1e-6


@pytest.mark.parametrize("N,n", [(32, 3), (96, 2), (128, 2)])
@pytest.mark.parametrize("order", [0, 1])
def test_fixed_cycles_match_oracle(N, n, order):
    from paper_2608_00760_amd import synth
    say("cycles N=%d n=%d order=%d" % (N, n, order))
    P, H = make(N, 60 + N)
    q = synth.blob_source(N, 3)
    u0 = synth.normal(N, 4)
    got = host(P.debug_cycles(dev(q), dev(u0), n, order=order))
    assert rel_max(got, H.cycles(q, u0, n, order=order)) <= 1e-12
