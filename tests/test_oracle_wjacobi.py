"""Pins of the oracle's weighted-Jacobi smoother (the alternative smoother;
u <- u + omega (q - A u) / diag(A), omega = 6/7 by default).

* one sweep equals the formula evaluated with an independently assembled
  dense operator (brute force);
* for constant coefficients a discrete sine mode is an eigenvector of A and
  of diag(A), and one sweep with q = 0 scales it by 1 - omega lambda / d
  (closed form);
* the sweep's adjoint is its exact transpose (dot-product identity);
* n fixed V-cycles with weighted Jacobi: the reversed composition of adjoints
  equals n cycles with the pre- and post-smoothing counts exchanged, and the
  pull-back is the transpose of the push-forward;
* the cycle converges on log-normal coefficients.
"""
import numpy as np
import pytest

from oracle import ref
from paper_2608_00760_amd import synth
from tests._dense import assemble_dense, scatter

OMEGA = 6.0 / 7.0


def dot(a, b):
    return float(np.sum(a * b))


def grf_hier(N, seed, **kw):
    logD, logmu = synth.log_coefficients(N, seed, seed + 1)
    return ref.Hierarchy(np.exp(logD), np.exp(logmu), smoother="wjacobi", **kw), np.exp(logD), np.exp(logmu)


@pytest.mark.parametrize("N,harmonic", [(6, False), (8, True), (12, False)])
def test_sweep_matches_dense_formula(N, harmonic):
    H, D, mu = grf_hier(N, 3 + N, face_mean="harmonic" if harmonic else "arith")
    u, q = synth.normal(N, 1), synth.normal(N, 2)
    A, _, idx = assemble_dense(D, mu, harmonic=harmonic)
    ui, qi = u[idx >= 0], q[idx >= 0]
    # interior vectors in the ordering of interior_index: x, y, z loops
    order = np.argsort(idx[idx >= 0])
    ui, qi = ui[order], qi[order]
    expect = ui + OMEGA * (qi - A @ ui) / np.diag(A)
    got = H.wj_sweep(0, u, q)
    assert np.abs(got - scatter(expect, idx)).max() <= 1e-13 * np.abs(expect).max()


@pytest.mark.parametrize("kx,ky,kz", [(1, 1, 1), (3, 1, 2), (7, 5, 6)])
def test_sweep_scales_sine_mode(kx, ky, kz):
    N, Dc, muc, h = 8, 1.7, 0.3, 1.0
    shape = synth.shape(N)
    H = ref.Hierarchy(np.full(shape, Dc), np.full(shape, muc), h=h, smoother="wjacobi")
    x = np.arange(N + 1)
    mode = (np.sin(np.pi * kx * x / N)[:, None, None] * np.sin(np.pi * ky * x / N)[None, :, None]
            * np.sin(np.pi * kz * x / N)[None, None, :])
    lam = Dc / h ** 2 * sum(2.0 - 2.0 * np.cos(np.pi * k / N) for k in (kx, ky, kz)) + muc
    d = 6.0 * Dc / h ** 2 + muc
    got = H.wj_sweep(0, mode, np.zeros(shape))
    assert np.abs(got - (1.0 - OMEGA * lam / d) * mode).max() <= 1e-14


def test_sweep_adjoint_is_transpose():
    H, _, _ = grf_hier(16, 21)
    N = 16
    u, q, ub = synth.normal(N, 4), synth.normal(N, 5), synth.normal(N, 6)
    out = H.wj_sweep(0, u, q)
    ubar, qbar = H.wj_sweep_adj(0, ub, np.zeros_like(ub))
    lhs, rhs = dot(out, ub), dot(u, ubar) + dot(q, qbar)
    assert abs(lhs - rhs) <= 1e-14 * np.linalg.norm(out) * np.linalg.norm(ub)


@pytest.mark.parametrize("N,nu1,nu2", [(16, 2, 2), (24, 2, 1), (32, 1, 3)])
def test_fixed_cycles_pullback_is_transpose(N, nu1, nu2):
    H, _, _ = grf_hier(N, 30 + N)
    q, w = synth.normal(N, 7), synth.normal(N, 8)
    n = 4
    rho, _ = H.forward(q, fixed_cycles=n, nu1=nu1, nu2=nu2)
    (qbar, _, _), _ = H.vjp(rho, w, fixed_cycles=n, nu1=nu1, nu2=nu2)
    # dot-product identity: <S_n q, w> = <q, S_n^T w>
    assert abs(dot(rho, w) - dot(q, qbar)) <= 1e-12 * np.linalg.norm(rho) * np.linalg.norm(w)
    # the literal reversed composition equals n cycles with nu1 and nu2 exchanged
    qbr, _ = H.pullback_br(w, fixed_cycles=n, nu1=nu1, nu2=nu2)
    assert np.abs(qbar - qbr).max() <= 1e-12 * np.abs(qbar).max()


def test_converges_on_grf():
    H, _, _ = grf_hier(32, 41)
    q = synth.normal(32, 9)
    rho, info = H.forward(q, rtol=1e-10, max_cycles=200)
    r = H.defect(0, rho, q)
    assert info["status"] == 0 and np.linalg.norm(r) <= 1e-10 * np.linalg.norm(H.defect(0, 0 * rho, q))
    # slower than red-black Gauss-Seidel, but a multigrid rate
    assert info["cycles"] <= 60, info
