"""Pins of the oracle against brute force on tiny grids.

* The multigrid solve reaches the solution of the densely assembled system
  (np.linalg.solve), for variable coefficients, both face means, a non-zero
  Dirichlet value and both level structures (c = 2 and c = 3).
* The push-forward and pull-back with respect to (q, log D, log mua) equal the
  Jacobian of the exact discrete solution, obtained column by column by the
  complex-step method (Squire & Trapp 1998: d u / d theta_j =
  Im u(theta + i eps e_j) / eps, exact to rounding for eps = 1e-30).
"""
import numpy as np
import pytest

from oracle import ref
from paper_2608_00760_amd import synth

from _dense import assemble_dense, gather, scatter


def fields(N, seed):
    rng = np.random.default_rng(seed)
    logD = 0.8 * rng.standard_normal(synth.shape(N))
    logmu = np.log(0.05) + 0.8 * rng.standard_normal(synth.shape(N))
    q = rng.standard_normal(synth.shape(N))
    return logD, logmu, q


@pytest.mark.parametrize("N", [4, 6, 8, 12])
@pytest.mark.parametrize("harmonic", [False, True])
@pytest.mark.parametrize("g", [0.0, 0.7])
def test_forward_equals_dense_solve(N, harmonic, g):
    logD, logmu, q = fields(N, 10 + N)
    D, mu = np.exp(logD), np.exp(logmu)
    A, b, idx = assemble_dense(D, mu, h=1.0, g=g, harmonic=harmonic)
    exact = scatter(np.linalg.solve(A, gather(q, idx) + b), idx, bc=g)
    H = ref.Hierarchy(D, mu, bc=g, face_mean="harmonic" if harmonic else "arith")
    rho, info = H.forward(q, rtol=1e-14, max_cycles=200)
    assert np.abs(rho - exact).max() <= 1e-12 * np.abs(exact).max(), info


def _solve_complex(logD, logmu, q, harmonic):
    A, b, idx = assemble_dense(np.exp(logD), np.exp(logmu), harmonic=harmonic)
    return np.linalg.solve(A, gather(q, idx).astype(A.dtype)), idx


@pytest.mark.parametrize("harmonic", [False, True])
def test_derivatives_equal_complex_step_jacobian(harmonic):
    N = 8
    logD, logmu, q = fields(N, 99)
    fm = "harmonic" if harmonic else "arith"
    H = ref.Hierarchy(np.exp(logD), np.exp(logmu), face_mean=fm)
    rho, _ = H.forward(q, rtol=1e-15, max_cycles=300)
    eps = 1e-30
    u0, idx = _solve_complex(logD, logmu, q, harmonic)
    n = N + 1
    # Jacobian of the interior solution w.r.t. every log D vertex (729 of them),
    # every interior log mua and every interior q.
    JD = np.zeros((u0.size, n ** 3))
    for v in range(n ** 3):
        pert = logD.astype(complex).ravel()
        pert[v] += 1j * eps
        u, _ = _solve_complex(pert.reshape(logD.shape), logmu, q, harmonic)
        JD[:, v] = u.imag / eps
    m = u0.size
    Jmu = np.zeros((m, n ** 3))
    Jq = np.zeros((m, n ** 3))
    interior = np.flatnonzero((idx >= 0).ravel())
    for v in interior:
        pert = logmu.astype(complex).ravel()
        pert[v] += 1j * eps
        u, _ = _solve_complex(logD, pert.reshape(logmu.shape), q, harmonic)
        Jmu[:, v] = u.imag / eps
    A, _, _ = assemble_dense(np.exp(logD), np.exp(logmu), harmonic=harmonic)
    Ainv = np.linalg.inv(A)
    for col, v in enumerate(interior):
        Jq[:, v] = Ainv[:, idx.ravel()[v]]

    rng = np.random.default_rng(7)
    rhobar = synth.zero_boundary(rng.standard_normal(synth.shape(N)))
    (qbar, gD, gmu), _ = H.vjp(rho, rhobar, rtol=1e-15, max_cycles=300)
    w = gather(rhobar, idx)
    for got, J in ((qbar, Jq), (gD, JD), (gmu, Jmu)):
        expect = (w @ J).reshape(logD.shape)
        assert np.abs(got - expect).max() <= 1e-11 * np.abs(expect).max()

    dq = synth.zero_boundary(rng.standard_normal(synth.shape(N)))
    dD = rng.standard_normal(synth.shape(N))
    dmu = synth.zero_boundary(rng.standard_normal(synth.shape(N)))
    drho, _ = H.jvp(rho, dq, dD, dmu, rtol=1e-15, max_cycles=300)
    expect = Jq @ dq.ravel() + JD @ dD.ravel() + Jmu @ dmu.ravel()
    got = gather(drho, idx)
    assert np.abs(got - expect).max() <= 1e-11 * np.abs(expect).max()
    # the boundary of the tangent solution is homogeneous
    assert np.abs(drho - scatter(got, idx)).max() == 0.0


def test_jvp_ignores_boundary_of_q_and_mua_tangent():
    N = 8
    logD, logmu, q = fields(N, 5)
    H = ref.Hierarchy(np.exp(logD), np.exp(logmu))
    rho, _ = H.forward(q, rtol=1e-14)
    rng = np.random.default_rng(3)
    dq, dmu = rng.standard_normal((2,) + synth.shape(N))
    a, _ = H.jvp(rho, dq, None, dmu, rtol=1e-14)
    b, _ = H.jvp(rho, synth.zero_boundary(dq), None, synth.zero_boundary(dmu), rtol=1e-14)
    assert np.array_equal(a, b)
