"""Pins of the oracle against closed forms (constant coefficients).

With constant D and mua the operator is (D/h^2)(-Laplacian_h) + mua I on the
interior vertices with homogeneous Dirichlet boundary, which the 3D type-I
discrete sine transform diagonalises with eigenvalues
(4 D / h^2) sum_axes sin^2(pi j_a / 2N) + mua,  j_a = 1..N-1.
"""
import numpy as np
import pytest
import scipy.fft as sfft

from oracle import ref
from paper_2608_00760_amd import synth


def dst_solve(q, D, mu, h):
    N = q.shape[0] - 1
    j = np.arange(1, N)
    lam1 = 4.0 * D / h ** 2 * np.sin(np.pi * j / (2 * N)) ** 2
    eig = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :] + mu
    qi = q[1:N, 1:N, 1:N]
    ui = sfft.idstn(sfft.dstn(qi, type=1) / eig, type=1)
    u = np.zeros_like(q)
    u[1:N, 1:N, 1:N] = ui
    return u


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("N,D,mu,h", [(32, 1.0, 0.1, 1.0), (24, 2.5, 0.0, 1.0), (16, 0.7, 3.0, 0.25),
                                      (6, 1.3, 0.2, 1.0), (2, 1.0, 0.5, 1.0), (3, 1.0, 0.5, 2.0)])
@pytest.mark.parametrize("face_mean", ["arith", "harmonic"])
def test_forward_matches_dst(N, D, mu, h, face_mean):
    rng = np.random.default_rng(N)
    q = rng.standard_normal(synth.shape(N))
    H = ref.Hierarchy(np.full(synth.shape(N), D), np.full(synth.shape(N), mu), h=h, face_mean=face_mean)
    rho, info = H.forward(q, rtol=1e-14, max_cycles=100)
    exact = dst_solve(q, D, mu, h)
    assert rel(rho, exact) <= 1e-12, info


def test_small_constant_workload_forward_and_adjoint():
    """32^3, D = 1, mua = 0.1, centred blob: solution and adjoint state vs DST-I."""
    c = synth.small_constant()
    H = ref.Hierarchy(c["D"], c["mua"])
    rho, info = H.forward(c["q"], rtol=1e-10)
    assert info["rel_residual"] <= 1e-10
    exact = dst_solve(c["q"], 1.0, 0.1, 1.0)
    assert rel(rho, exact) <= 1e-9
    (qbar, _, _), vinfo = H.vjp(rho, c["rhobar"], rtol=1e-13)
    assert rel(qbar, dst_solve(c["rhobar"], 1.0, 0.1, 1.0)) <= 1e-11
    # the eigenvalue check itself: A applied to a sine mode scales it
    N = 32
    x = np.arange(N + 1)
    mode = (np.sin(np.pi * 3 * x / N)[:, None, None] * np.sin(np.pi * 5 * x / N)[None, :, None]
            * np.sin(np.pi * 7 * x / N)[None, None, :])
    lam = sum(4 * np.sin(np.pi * j / (2 * N)) ** 2 for j in (3, 5, 7)) + 0.1
    Am = H.apply(0, mode)
    inner = (slice(1, N),) * 3
    assert np.abs(Am[inner] - lam * mode[inner]).max() <= 1e-13


def test_constant_boundary_value_is_reproduced():
    """D = 1, mua = 0, q = 0, Dirichlet value g = 1: the exact solution is 1."""
    N = 16
    H = ref.Hierarchy(np.ones(synth.shape(N)), np.zeros(synth.shape(N)), bc=1.0)
    rho, info = H.forward(np.zeros(synth.shape(N)), rtol=1e-13)
    assert np.abs(rho - 1.0).max() <= 1e-12


def test_exact_solve_single_unknown():
    """N = 2: one unknown, u = (q + sum c g) / (sum c + mua)."""
    D = np.arange(27, dtype=float).reshape(3, 3, 3) + 1.0
    mu = np.full((3, 3, 3), 0.3)
    H = ref.Hierarchy(D, mu, h=0.5, bc=2.0)
    q = np.zeros((3, 3, 3)); q[1, 1, 1] = 1.7
    rho, _ = H.forward(q, rtol=1e-14)
    c = [(D[1, 1, 1] + D[j]) / 2 / 0.25 for j in [(0, 1, 1), (2, 1, 1), (1, 0, 1), (1, 2, 1), (1, 1, 0), (1, 1, 2)]]
    expect = (1.7 + 2.0 * sum(c)) / (sum(c) + 0.3)
    assert abs(rho[1, 1, 1] - expect) <= 1e-14 * abs(expect)
