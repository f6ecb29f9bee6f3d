"""Invariant pins of the oracle and the values the paper prints.

* restriction of a unit spike reproduces the printed 1D stencil 1/4 [1 2 1]
  (Eq. (rest)) along each axis, as a tensor product;
* prolongation has the scaling of Sec. 2.3.3 and reproduces constants and
  linear functions away from the boundary; restriction and the coefficient
  transfer reproduce constants and linear functions;
* the operator is an M-matrix: a non-negative source gives a non-negative
  solution;
* the V(2,2) red-black cycle contracts the residual by well under 0.15 per
  cycle for constant coefficients (textbook behaviour, Sec. 2.2);
* the fixed cycle count of the paper's experiments runs (Sec. 2.4).
"""
import numpy as np
import pytest

from conftest import golden
from oracle import ref
from paper_2608_00760_amd import synth


def const_hier(N, D=1.0, mu=0.1):
    return ref.Hierarchy(np.full(synth.shape(N), D), np.full(synth.shape(N), mu))


def test_restriction_spike_reproduces_printed_stencil():
    w1 = np.array([float(v) for v in golden("restriction_1d.txt")[0]])
    N = 8
    H = const_hier(N)
    # a unit spike at the fine vertex under coarse vertex X contributes to the
    # coarse value at X with weight w(0)^3; a spike next to it with w(1) w(0)^2 ...
    X = (2, 2, 2)
    got = np.zeros((3, 3, 3))
    for a in range(3):
        for b in range(3):
            for c in range(3):
                r = np.zeros(synth.shape(N))
                r[2 * X[0] + a - 1, 2 * X[1] + b - 1, 2 * X[2] + c - 1] = 1.0
                got[a, b, c] = H.restrict(0, r)[X]
    expect = np.einsum("i,j,k->ijk", w1, w1, w1)
    assert np.array_equal(got, expect)


def test_prolongation_scaling_of_printed_relation():
    rows = dict((r[0], float(r[1])) for r in golden("transfer_scaling.txt"))
    factor = rows["factor"]
    assert factor == 2 ** rows["dimension"]
    N = 16
    H = const_hier(N)
    rng = np.random.default_rng(0)
    for _ in range(3):
        r = synth.zero_boundary(rng.standard_normal(synth.shape(N)))
        y = synth.zero_boundary(rng.standard_normal(synth.shape(N // 2)))
        lhs = np.sum(H.prolong_add(0, y, np.zeros_like(r)) * r)
        rhs = factor * np.sum(y * H.restrict(0, r))
        assert abs(lhs - rhs) <= 1e-13 * abs(rhs) + 1e-13


def test_transfers_reproduce_constants_and_linears():
    N = 16
    H = const_hier(N)
    X, Y, Z = synth.coords(N)
    lin = 0.3 + 0.1 * X - 0.2 * Y + 0.05 * Z + 0 * X * Y * Z
    Xc, Yc, Zc = synth.coords(N // 2)
    linc = 0.3 + 0.2 * Xc - 0.4 * Yc + 0.1 * Zc + 0 * Xc * Yc * Zc
    inner_c = (slice(1, N // 2),) * 3
    for f, fc in ((np.ones(synth.shape(N)), np.ones(synth.shape(N // 2))), (lin, linc)):
        assert np.allclose(H.restrict(0, f)[inner_c], fc[inner_c], rtol=0, atol=1e-14)
        cf = ref.coarsen_field(f)
        assert np.allclose(cf, fc, rtol=0, atol=1e-14)   # interior full weighting, boundary injection
        # prolongation of a coarse linear field, away from the boundary
        pf = H.prolong_add(0, fc, np.zeros(synth.shape(N)))
        inner = (slice(2, N - 1),) * 3
        assert np.allclose(pf[inner], f[inner], rtol=0, atol=1e-13)


def test_m_matrix_nonnegative_solution():
    N = 32
    logD, logmu = synth.log_coefficients(N, 7, 8)
    H = ref.Hierarchy(np.exp(logD), np.exp(logmu))
    q = synth.blob_source(N, 9, noise=0.0)
    rho, _ = H.forward(q, rtol=1e-13)
    assert rho.min() >= -1e-13 * rho.max()
    assert rho[1:-1, 1:-1, 1:-1].min() > 0.0


@pytest.mark.parametrize("N", [32, 48])
def test_vcycle_contraction_constant_coefficients(N):
    H = const_hier(N, 1.0, 0.1)
    q = synth.normal(N, 1)
    _, hist, st = H.forward_history(q, rtol=1e-12, max_cycles=40)
    assert st == 0
    rates = hist[1:] / hist[:-1]
    assert rates.max() < 0.15, rates


def test_paper_fixed_schedule_runs():
    n = int(golden("paper_schedule.txt")[0][1])
    assert n == 15
    N = 32
    logD, logmu = synth.log_coefficients(N, 70, 71)
    H = ref.Hierarchy(np.exp(logD), np.exp(logmu))
    rho, info = H.forward(synth.blob_source(N, 72), fixed_cycles=n)
    assert info["cycles"] == n and info["rel_residual"] < 1e-9


def test_invalid_inputs_are_rejected():
    with pytest.raises(ref.OracleError):
        ref.Hierarchy(np.ones((6, 6, 6)), np.ones((6, 6, 6)))       # N = 5 is not c 2^m
    D = np.ones(synth.shape(8)); D[3, 3, 3] = 0.0
    with pytest.raises(ref.OracleError):
        ref.Hierarchy(D, np.ones(synth.shape(8)))
    mu = np.ones(synth.shape(8)); mu[2, 2, 2] = -1e-3
    with pytest.raises(ref.OracleError):
        ref.Hierarchy(np.ones(synth.shape(8)), mu)
    H = const_hier(8)
    q = np.zeros(synth.shape(8)); q[4, 4, 4] = np.nan
    with pytest.raises(ref.OracleError):
        H.forward(q)
    rho, info = H.forward(synth.normal(8, 1), rtol=1e-14, max_cycles=2, check=False)
    assert info["status"] == 3 and info["cycles"] == 2
