"""Pins of the oracle against the continuous problem and independent solvers.

* method of manufactured solutions: with u* = prod sin(pi x_a),
  D = exp(0.5 prod sin(2 pi x_a)) and mua = 0.1 on the unit cube, the source
  q = -div(D grad u*) + mua u* is known in closed form; the discrete solution
  must approach u* at second order (Eq. (maineq) discretised by second-order
  finite differences, Sec. 2);
* conjugate gradients on the sparse assembled operator reach the same
  solution and adjoint state as the multigrid solve;
* central finite differences of <w, u(theta)> along random directions of
  (q, log D, log mua) agree with the pull-back.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import ref
from paper_2608_00760_amd import synth

from _dense import assemble_sparse, gather, scatter


def mms_case(N):
    h = 1.0 / N
    x = np.arange(N + 1) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    pi = np.pi
    u = np.sin(pi * X) * np.sin(pi * Y) * np.sin(pi * Z)
    P = np.sin(2 * pi * X) * np.sin(2 * pi * Y) * np.sin(2 * pi * Z)
    D = np.exp(0.5 * P)
    dD = [D * pi * np.cos(2 * pi * X) * np.sin(2 * pi * Y) * np.sin(2 * pi * Z),
          D * pi * np.sin(2 * pi * X) * np.cos(2 * pi * Y) * np.sin(2 * pi * Z),
          D * pi * np.sin(2 * pi * X) * np.sin(2 * pi * Y) * np.cos(2 * pi * Z)]
    du = [pi * np.cos(pi * X) * np.sin(pi * Y) * np.sin(pi * Z),
          pi * np.sin(pi * X) * np.cos(pi * Y) * np.sin(pi * Z),
          pi * np.sin(pi * X) * np.sin(pi * Y) * np.cos(pi * Z)]
    mu = np.full_like(u, 0.1)
    q = 3 * pi ** 2 * D * u - sum(a * b for a, b in zip(dD, du)) + mu * u
    return h, D, mu, q, u


@pytest.mark.parametrize("face_mean", ["arith", "harmonic"])
def test_manufactured_solution_second_order(face_mean):
    errs = []
    for N in (16, 32, 64):
        h, D, mu, q, u = mms_case(N)
        H = ref.Hierarchy(D, mu, h=h, face_mean=face_mean)
        rho, _ = H.forward(q, rtol=1e-12)
        errs.append(np.abs(rho - u).max())
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert all(3.6 <= r <= 4.4 for r in ratios), (errs, ratios)


def test_discrete_manufactured_solution():
    N = 32
    logD, logmu = synth.log_coefficients(N, 61, 62)
    H = ref.Hierarchy(np.exp(logD), np.exp(logmu))
    ustar = synth.zero_boundary(synth.grf(N, 63))
    q = H.apply(0, ustar)
    rho, _ = H.forward(q, rtol=1e-13)
    assert np.abs(rho - ustar).max() <= 1e-9 * np.abs(ustar).max()


@pytest.mark.parametrize("N", [32, 64])
def test_conjugate_gradients_agree(N):
    logD, logmu = synth.log_coefficients(N, 80 + N, 81 + N)
    D, mu = np.exp(logD), np.exp(logmu)
    A, idx = assemble_sparse(D, mu)
    H = ref.Hierarchy(D, mu)
    x = synth.normal(N, 3)
    assert np.abs(gather(H.apply(0, x), idx) - A @ gather(x, idx)).max() <= 1e-12 * np.abs(A @ gather(x, idx)).max()
    q = synth.blob_source(N, 4)
    b = gather(q, idx)
    ucg, info = spla.cg(A, b, rtol=1e-14, atol=0.0, maxiter=20000)
    assert info == 0
    rho, _ = H.forward(q, rtol=1e-13)
    assert np.abs(rho - scatter(ucg, idx)).max() <= 1e-10 * np.abs(rho).max()
    w = synth.normal(N, 5)
    lcg, info = spla.cg(A, gather(w, idx), rtol=1e-14, atol=0.0, maxiter=20000)
    (qbar, _, _), _ = H.vjp(rho, w, rtol=1e-13)
    assert np.abs(qbar - scatter(lcg, idx)).max() <= 1e-10 * np.abs(qbar).max()


def test_central_differences_match_pullback():
    N = 24
    logD, logmu = synth.log_coefficients(N, 91, 92)
    q = synth.blob_source(N, 93)
    w = synth.normal(N, 94)
    H = ref.Hierarchy(np.exp(logD), np.exp(logmu))
    rho, _ = H.forward(q, rtol=1e-14, max_cycles=100)
    (qb, gD, gmu), _ = H.vjp(rho, w, rtol=1e-14, max_cycles=100)
    eps = 1e-4
    for d in range(4):
        t = synth.tangents(N, 1000 + 10 * d)

        def J(s):
            Hs = ref.Hierarchy(np.exp(logD + s * t["dlogD"]), np.exp(logmu + s * t["dlogmua"]))
            u, _ = Hs.forward(q + s * t["dq"], rtol=1e-14, max_cycles=100)
            return np.sum(w * u)

        fd = (J(eps) - J(-eps)) / (2 * eps)
        ad = np.sum(t["dq"] * qb) + np.sum(t["dlogD"] * gD) + np.sum(t["dlogmua"] * gmu)
        assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
